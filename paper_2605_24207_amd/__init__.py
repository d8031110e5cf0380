"""relnn for MI355X: one relational layer (join -> Concat+Linear ->
group-by SUM/MEAN/MAX) as hand-written gfx950 HIP kernels behind a C ABI.

The C ABI is declared in include/relnn.h; this package is its Python
binding (argument marshalling only).  The library is loaded on first use and
its absence raises ImportError: there is no CPU or eager fallback.
"""
from .api import (Index, Layer, RelLayerFn, Server, layer_bwd, layer_fwd,  # noqa: F401
                  Union, UnionFn, attn_bwd, attn_fwd, layer_fwd_static, out_dense, static_scratch_bytes, union_bwd,
                  union_fwd, workspace, workspace_size)
from ._lib import RelnnError  # noqa: F401
