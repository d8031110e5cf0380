"""Python binding of librelnn with the C ABI's names.

Argument marshalling only: every step of the layer runs in the library's
HIP kernels.  Torch supplies device memory and the current stream.
"""
from __future__ import annotations

import ctypes as C
from typing import List, Optional, Sequence

import torch

from . import _lib as L
from ._lib import check, lib

_DTYPES = {"f32": (L.F32, torch.float32), "bf16": (L.BF16, torch.bfloat16)}
_AGGS = {"sum": L.SUM, "mean": L.MEAN, "max": L.MAX}
_ACTS = {"none": L.ACT_NONE, "relu": L.ACT_RELU}


def _vp(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def _i32(t: torch.Tensor, what: str) -> torch.Tensor:
    if t.dtype != torch.int32 or not t.is_cuda or not t.is_contiguous():
        raise TypeError(f"{what} must be a contiguous int32 CUDA tensor")
    return t


class Index:
    """relnn_build_index: the join of one rule in canonical order plus its
    group CSR (device-resident, library-owned).

    cols: link columns, int32 [n_link] each.  atoms: (n_rows, col, keys)
    per body atom in Concat order (keys None = dense ids).  chains:
    (src_col, vals, keys) derived columns.  two_hop: (mid_col, cap) or None.
    steps: (cols, on, key) further link relations joined in order (on / key:
    one or two column numbers).  preds: (a, op, b, mul_a, mul_b, add)
    filter predicates, op one of eq ne lt le gt ge.
    """

    def __init__(self, cols: Sequence[torch.Tensor], atoms, group_col: int, chains=(),
                 two_hop=None, bwd: bool = False, steps=(), preds=(), stream=None):
        lib()
        self._handle = None
        cols = [_i32(c, "link column") for c in cols]
        n_link = int(cols[0].numel())
        col_arr = (C.c_void_p * len(cols))(*[c.data_ptr() for c in cols])
        at = (L.Atom * len(atoms))()
        keep = list(cols)
        for j, (n_rows, col, keys) in enumerate(atoms):
            at[j].n_rows = int(n_rows)
            at[j].col = int(col)
            at[j].keys = None if keys is None else _i32(keys, "atom keys").data_ptr()
            keep.append(keys)
        ch = (L.Chain * max(1, len(chains)))()
        for i, (src, vals, keys) in enumerate(chains):
            ch[i].src_col = int(src)
            ch[i].n_rows = int(vals.numel())
            ch[i].vals = _i32(vals, "chain values").data_ptr()
            ch[i].keys = None if keys is None else _i32(keys, "chain keys").data_ptr()
            keep += [vals, keys]
        d = L.JoinDesc()
        d.n_link = n_link
        d.n_cols = len(cols)
        d.cols = col_arr
        d.n_chains = len(chains)
        d.chains = ch
        d.n_atoms = len(atoms)
        d.atoms = at
        d.group_col = int(group_col)
        d.two_hop_mid, d.two_hop_cap = (-1, 0) if two_hop is None else (int(two_hop[0]), int(two_hop[1]))
        d.flags = L.IDX_BWD if bwd else 0
        sa = (L.JoinStep * max(1, len(steps)))()
        for i, (scols, on, key) in enumerate(steps):
            scols = [_i32(c, "step column") for c in scols]
            arr = (C.c_void_p * len(scols))(*[c.data_ptr() for c in scols])
            keep += scols + [arr]
            sa[i].n_rows = int(scols[0].numel())
            sa[i].n_cols = len(scols)
            sa[i].cols = arr
            if len(on) != len(key) or not 1 <= len(on) <= 2:
                raise ValueError("a step joins on one or two column pairs")
            sa[i].n_on = len(on)
            for q in range(len(on)):
                sa[i].on[q] = int(on[q])
                sa[i].key[q] = int(key[q])
        pa = (L.Pred * max(1, len(preds)))()
        for i, (a, op, b, mul_a, mul_b, add) in enumerate(preds):
            pa[i].a, pa[i].b = int(a), int(b)
            pa[i].mul_a, pa[i].mul_b, pa[i].add = int(mul_a), int(mul_b), int(add)
            pa[i].op = L.CMP[op]
        d.n_steps, d.steps = len(steps), sa
        d.n_preds, d.preds = len(preds), pa
        h = C.c_void_p()
        check(lib().relnn_build_index(C.byref(d), _stream(stream), C.byref(h)))
        self._handle = h
        self.k = len(atoms)
        self.n_rows = [int(a[0]) for a in atoms]
        self.bwd = bwd
        E, G, B = C.c_int64(), C.c_int64(), C.c_int64()
        check(lib().relnn_index_query(h, C.byref(E), C.byref(G), C.byref(B)))
        self.E, self.G, self.dev_bytes = E.value, G.value, B.value
        self.device = cols[0].device

    @property
    def handle(self):
        return self._handle

    def export(self, stream=None):
        """group_keys [G], offsets [G+1], link_rows [E], tuple_rows [k, E]."""
        dev = self.device
        gk = torch.empty(self.G, dtype=torch.int32, device=dev)
        off = torch.empty(self.G + 1, dtype=torch.int32, device=dev)
        lr = torch.empty(self.E, dtype=torch.int32, device=dev)
        tr = torch.empty(self.k, self.E, dtype=torch.int32, device=dev)
        check(lib().relnn_index_export(self._handle, _vp(gk), _vp(off), _vp(lr), _vp(tr), _stream(stream)))
        return {"group_keys": gk, "offsets": off, "link_rows": lr, "tuple_rows": tr}

    def free(self):
        if self._handle is not None and _lib_alive():
            check(lib().relnn_index_free(self._handle))
        self._handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def _attn_desc(d, dv, heads, scale, dtype):
    a = L.AttnDesc()
    a.heads, a.d, a.dv, a.scale, a.dtype = int(heads), int(d), int(dv), float(scale), _DTYPES[dtype][0]
    return a


def _attn_inputs(index: "Index", q, k, v):
    if index.k != 3:
        raise ValueError("attention needs an index with three atoms (Q, K, V)")
    dt = q.dtype
    for name, t in (("q", q), ("k", k), ("v", v)):
        if t.dtype != dt or t.dtype not in (torch.float32, torch.bfloat16) or not t.is_cuda \
                or not t.is_contiguous() or t.dim() != 2:
            raise TypeError(f"{name} must be a contiguous 2-d float32 or bfloat16 CUDA tensor like q")
    if k.shape[1] != q.shape[1]:
        raise ValueError("q and k must have the same width")
    return "bf16" if dt == torch.bfloat16 else "f32"


def attn_fwd(index: "Index", q, k, v, heads: int, scale: float, stream=None):
    """relnn_attn_fwd: (out [G, dv], lse [G, heads])."""
    dtype = _attn_inputs(index, q, k, v)
    a = _attn_desc(q.shape[1], v.shape[1], heads, scale, dtype)
    n = C.c_size_t()
    check(lib().relnn_attn_workspace_size(index.handle, C.byref(a), 0, C.byref(n)))
    ws = torch.empty(max(n.value, 256), dtype=torch.uint8, device=index.device)
    out = torch.empty(index.G, v.shape[1], dtype=torch.float32, device=index.device)
    lse = torch.empty(index.G, heads, dtype=torch.float32, device=index.device)
    check(lib().relnn_attn_fwd(index.handle, C.byref(a), _vp(q), _vp(k), _vp(v), _vp(out), _vp(lse), _vp(ws),
                               ws.numel(), _stream(stream)))
    return out, lse


def attn_bwd(index: "Index", q, k, v, heads: int, scale: float, out, lse, dout, dq, dk, dv, stream=None):
    """relnn_attn_bwd: adds the gradients into dq, dk, dv (FP32, may alias)."""
    dtype = _attn_inputs(index, q, k, v)
    for name, t, ref in (("dq", dq, q), ("dk", dk, k), ("dv", dv, v)):
        if t.dtype != torch.float32 or tuple(t.shape) != tuple(ref.shape) or not t.is_contiguous():
            raise TypeError(f"{name} must be a contiguous float32 tensor shaped like its input")
    if dout.dtype != torch.float32 or tuple(dout.shape) != (index.G, v.shape[1]) or not dout.is_contiguous():
        raise TypeError("dout must be a contiguous float32 [G, dv] tensor")
    a = _attn_desc(q.shape[1], v.shape[1], heads, scale, dtype)
    n = C.c_size_t()
    check(lib().relnn_attn_workspace_size(index.handle, C.byref(a), 1, C.byref(n)))
    ws = torch.empty(max(n.value, 256), dtype=torch.uint8, device=index.device)
    check(lib().relnn_attn_bwd(index.handle, C.byref(a), _vp(q), _vp(k), _vp(v), _vp(out), _vp(lse), _vp(dout),
                               _vp(dq), _vp(dk), _vp(dv), _vp(ws), ws.numel(), _stream(stream)))


class Union:
    """relnn_union_build: the k-ary projected union of the head keys of k
    join indices (device-resident, library-owned; the indices must outlive
    it)."""

    def __init__(self, branches: Sequence["Index"], stream=None):
        lib()
        self._handle = None
        self.branches = list(branches)
        arr = (C.c_void_p * len(branches))(*[b.handle.value for b in branches])
        h = C.c_void_p()
        check(lib().relnn_union_build(arr, len(branches), _stream(stream), C.byref(h)))
        self._handle = h
        G = C.c_int64()
        check(lib().relnn_union_query(h, C.byref(G)))
        self.G = G.value
        self.k = len(branches)
        self.device = branches[0].device

    @property
    def handle(self):
        return self._handle

    def export(self, stream=None):
        keys = torch.empty(self.G, dtype=torch.int32, device=self.device)
        cnt = torch.empty(self.G, dtype=torch.int32, device=self.device)
        check(lib().relnn_union_export(self._handle, _vp(keys), _vp(cnt), _stream(stream)))
        return {"keys": keys, "counts": cnt}

    def free(self):
        if self._handle is not None and _lib_alive():
            check(lib().relnn_union_free(self._handle))
        self._handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def _union_args(union: Union, layers, embs, Ws, bs, W_post, dw_accum=None):
    k = union.k
    if not (len(layers) == len(embs) == len(Ws) == k):
        raise ValueError("one layer, embedding list and W per branch")
    acc = [False] * k if dw_accum is None else [bool(x) for x in dw_accum]
    if len(acc) != k:
        raise ValueError("one dw_accum flag per branch")
    descs = [l.desc(dw_accum=a) for l, a in zip(layers, acc)]
    dptr = (C.POINTER(L.LayerDesc) * k)(*[C.pointer(d) for d in descs])
    emb_arrs = [(C.c_void_p * len(e))(*[t.data_ptr() for t in e]) for e in embs]
    for l, e, W in zip(layers, embs, Ws):
        _check_embs(l, e)
        if W.dtype != l.torch_dtype or W.shape != (l.K, l.h) or not W.is_contiguous():
            raise TypeError(f"W must be a contiguous {l.torch_dtype} [{l.K}, {l.h}] tensor")
    emb_pp = (C.POINTER(C.c_void_p) * k)(*[C.cast(a, C.POINTER(C.c_void_p)) for a in emb_arrs])
    W_arr = (C.c_void_p * k)(*[W.data_ptr() for W in Ws])
    b_arr = None if bs is None else (C.c_void_p * k)(*[None if b is None else b.data_ptr() for b in bs])
    h = layers[0].h
    h_out = h if W_post is None else int(W_post.shape[1])
    if W_post is not None and (W_post.dtype != torch.float32 or tuple(W_post.shape) != (h, h_out)
                               or not W_post.is_contiguous()):
        raise TypeError(f"W_post must be a contiguous float32 [{h}, h_out] tensor")
    # the ctypes arrays must outlive the call: keep them with the pointers
    return (descs, emb_arrs), dptr, emb_pp, W_arr, b_arr, h, h_out


def union_fwd(union: Union, layers: Sequence["Layer"], agg: str, act_post: str, embs, Ws, bs=None,
              W_post: Optional[torch.Tensor] = None, b_post: Optional[torch.Tensor] = None, want_pre: bool = True,
              want_argmax: bool = True, stream=None):
    """relnn_union_fwd.  embs[i]: the branch's embedding tensors; Ws[i],
    bs[i]: its transform.  Returns (out [G, h_out], pre [G, h] or None,
    argmax [G, h] int32 for MAX (positions in the concatenation of the
    branches' tuple orders) or None)."""
    keep, dptr, emb_pp, W_arr, b_arr, h, h_out = _union_args(union, layers, embs, Ws, bs, W_post)
    dev = union.device
    out = torch.empty(union.G, h_out, dtype=torch.float32, device=dev)
    pre = torch.empty(union.G, h, dtype=torch.float32, device=dev) if want_pre else None
    am = torch.empty(union.G, h, dtype=torch.int32, device=dev) if (want_argmax and agg == "max") else None
    n = C.c_size_t()
    check(lib().relnn_union_workspace_size(union.handle, dptr, _AGGS[agg], C.byref(n)))
    ws = torch.empty(max(n.value, 256), dtype=torch.uint8, device=dev)
    check(lib().relnn_union_fwd(union.handle, dptr, _AGGS[agg], _ACTS[act_post], emb_pp, W_arr, b_arr,
                                _vp(W_post), _vp(b_post), h_out, _vp(out), _vp(pre), _vp(am), _vp(ws), ws.numel(),
                                _stream(stream)))
    return out, pre, am


def union_bwd(union: Union, layers: Sequence["Layer"], agg: str, act_post: str, embs, Ws, bs,
              W_post: Optional[torch.Tensor], b_post: Optional[torch.Tensor], pre: Optional[torch.Tensor],
              argmax: Optional[torch.Tensor], dout: torch.Tensor, demb, dWs, dbs=None,
              dW_post: Optional[torch.Tensor] = None, db_post: Optional[torch.Tensor] = None, dw_accum=None,
              stream=None):
    """relnn_union_bwd.  demb[i]: FP32 gradient tensors shaped as embs[i]
    (accumulated, may alias); dWs[i], dbs[i]: FP32 gradients of Ws[i], bs[i]
    (written, or added where dw_accum[i] is true, so branches sharing one W
    can share one buffer); dW_post, db_post: of the union rule's transform
    (written)."""
    keep, dptr, emb_pp, W_arr, b_arr, h, h_out = _union_args(union, layers, embs, Ws, bs, W_post, dw_accum)

    def f32(t, shape, what):
        if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous() or tuple(t.shape) != shape:
            raise TypeError(f"{what} must be a contiguous float32 CUDA tensor of shape {shape}")

    f32(dout, (union.G, h_out), "dout")
    if pre is not None:
        f32(pre, (union.G, h), "pre")
    if argmax is not None and (argmax.dtype != torch.int32 or tuple(argmax.shape) != (union.G, h)
                               or not argmax.is_contiguous()):
        raise TypeError("argmax must be a contiguous int32 [G, h] tensor")
    for l, e, d, dW in zip(layers, embs, demb, dWs):
        if len(d) != len(e):
            raise ValueError("one gradient per embedding")
        for t, g in zip(e, d):
            f32(g, tuple(t.shape), "demb")
        f32(dW, (l.K, l.h), "dW")
    if dbs is not None:
        for db in dbs:
            if db is not None:
                f32(db, (h,), "db")
    if W_post is not None:
        if dW_post is None:
            raise ValueError("dW_post is required with W_post")
        f32(dW_post, (h, h_out), "dW_post")
        if db_post is not None:
            f32(db_post, (h_out,), "db_post")
    k = union.k
    demb_arrs = [(C.c_void_p * len(d))(*[g.data_ptr() for g in d]) for d in demb]
    demb_pp = (C.POINTER(C.c_void_p) * k)(*[C.cast(a, C.POINTER(C.c_void_p)) for a in demb_arrs])
    dW_arr = (C.c_void_p * k)(*[dW.data_ptr() for dW in dWs])
    db_arr = None if dbs is None else (C.c_void_p * k)(*[None if db is None else db.data_ptr() for db in dbs])
    n = C.c_size_t()
    check(lib().relnn_union_bwd_workspace_size(union.handle, dptr, _AGGS[agg], h_out, C.byref(n)))
    ws = torch.empty(max(n.value, 256), dtype=torch.uint8, device=union.device)
    check(lib().relnn_union_bwd(union.handle, dptr, _AGGS[agg], _ACTS[act_post], emb_pp, W_arr, b_arr,
                                _vp(W_post), _vp(b_post), h_out, _vp(pre), _vp(argmax), _vp(dout), demb_pp, dW_arr,
                                db_arr, _vp(dW_post), _vp(db_post), _vp(ws), ws.numel(), _stream(stream)))


class UnionFn(torch.autograd.Function):
    """out = union rule over the branches, with the hand-written backward.

    Usage: UnionFn.apply(union, layers, agg, act_post, W_post, b_post,
    *params) with params = W_0, b_0, embs_0..., W_1, b_1, embs_1, ...
    (b_i may be None; branch i has len(layers[i].dims) embeddings).  Gradients
    flow to every W_i, b_i, embedding, W_post and b_post; tensors shared
    by several atoms or branches get one buffer."""

    @staticmethod
    def forward(ctx, union: Union, layers, agg: str, act_post: str, W_post, b_post, *params):
        Ws, bs, embs, i = [], [], [], 0
        for l in layers:
            Ws.append(params[i])
            bs.append(params[i + 1])
            embs.append(list(params[i + 2: i + 2 + len(l.dims)]))
            i += 2 + len(l.dims)
        out, pre, am = union_fwd(union, layers, agg, act_post, embs, Ws, bs, W_post, b_post)
        ctx.union, ctx.layers, ctx.agg, ctx.act_post = union, layers, agg, act_post
        ctx.has_b = [b is not None for b in bs]
        ctx.save_for_backward(W_post, b_post, pre, am, *params)
        return out

    @staticmethod
    def backward(ctx, dout):
        W_post, b_post, pre, am, *params = ctx.saved_tensors
        layers = ctx.layers
        dev = dout.device
        Ws, bs, embs, i = [], [], [], 0
        for l in layers:
            Ws.append(params[i])
            bs.append(params[i + 1])
            embs.append(list(params[i + 2: i + 2 + len(l.dims)]))
            i += 2 + len(l.dims)
        bufs = {}

        def buf(t):
            key = t.data_ptr()
            first = key not in bufs
            if first:
                bufs[key] = torch.zeros(t.shape, dtype=torch.float32, device=dev)
            return bufs[key], first

        demb = [[buf(t)[0] for t in e] for e in embs]
        dWs = [torch.empty(l.K, l.h, dtype=torch.float32, device=dev) for l in layers]
        dbs = [torch.empty(l.h, dtype=torch.float32, device=dev) if hb else None
               for l, hb in zip(layers, ctx.has_b)]
        dW_post = None if W_post is None else torch.empty(W_post.shape, dtype=torch.float32, device=dev)
        db_post = None if b_post is None else torch.empty(b_post.shape, dtype=torch.float32, device=dev)
        union_bwd(ctx.union, layers, ctx.agg, ctx.act_post, embs, Ws, bs, W_post, b_post, pre, am,
                  dout.to(torch.float32).contiguous(), demb, dWs, dbs, dW_post, db_post)
        grads, seen = [], set()
        for l, dW, db, e in zip(layers, dWs, dbs, embs):
            grads += [dW, db]
            for t in e:
                key = t.data_ptr()
                grads.append(bufs[key] if key not in seen else None)
                seen.add(key)
        return (None, None, None, None, dW_post, db_post) + tuple(grads)


def out_dense(keys: torch.Tensor, compact: torch.Tensor, n_out: int, want_present: bool = True, stream=None):
    """relnn_out_dense: rows of ``compact`` ([G, h] FP32, one per key of the
    ascending ``keys`` [G] int32) placed at row key of a dense [n_out, h]
    tensor, zero elsewhere; returns (dense, present [n_out] uint8 or None)."""
    if keys.dtype != torch.int32 or keys.dim() != 1 or not keys.is_contiguous():
        raise TypeError("keys must be a contiguous int32 vector")
    G = keys.numel()
    if compact.dtype != torch.float32 or compact.dim() != 2 or compact.shape[0] != G or not compact.is_contiguous():
        raise TypeError("compact must be a contiguous float32 [G, h] tensor")
    h = compact.shape[1]
    dense = torch.empty(n_out, h, dtype=torch.float32, device=compact.device)
    present = torch.empty(n_out, dtype=torch.uint8, device=compact.device) if want_present else None
    check(lib().relnn_out_dense(_vp(keys), G, _vp(compact), h, n_out, _vp(dense), _vp(present), _stream(stream)))
    return dense, present


def _lib_alive():
    return L._lib is not None


class Layer:
    """relnn_layer_desc: widths, output width, dtype, aggregate, activations.
    transform: "linear" (Concat + Linear) or "product" (the elementwise
    product of the atoms' embeddings, no weights)."""

    def __init__(self, dims: Sequence[int], h: int, dtype: str = "f32", agg: str = "sum",
                 act_pre: str = "none", act_post: str = "none", plain: bool = False,
                 out_dtype: str = "f32", pushdown: bool = False, transform: str = "linear"):
        if transform not in ("linear", "product"):
            raise ValueError("transform is 'linear' or 'product'")
        self.transform = transform
        self.out_dtype = out_dtype
        self.pushdown = pushdown
        self.dims = [int(x) for x in dims]
        self.h = int(h)
        self.dtype = dtype
        self.agg = agg
        self.act_pre = act_pre
        self.act_post = act_post
        self.plain = plain
        self._d = (C.c_int32 * len(self.dims))(*self.dims)

    @property
    def K(self):
        return sum(self.dims)

    @property
    def torch_dtype(self):
        return _DTYPES[self.dtype][1]

    def desc(self, dw_accum=False, bwd=False) -> L.LayerDesc:
        """The ABI descriptor; for the backward without the output-storage
        flag (the backward reads pre and dout, not the stored output)."""
        d = L.LayerDesc()
        d.k = len(self.dims)
        d.d = self._d
        d.h = self.h
        d.dtype = _DTYPES[self.dtype][0]
        d.agg = _AGGS[self.agg]
        d.act_pre = _ACTS[self.act_pre]
        d.act_post = _ACTS[self.act_post]
        d.flags = ((L.PLAIN if self.plain else L.FUSED) | (L.DW_ACCUM if dw_accum else 0)
                   | (L.OUT_BF16 if self.out_dtype == "bf16" and not bwd else 0)
                   | (L.PUSHDOWN if self.pushdown else 0)
                   | (L.TF_PRODUCT if self.transform == "product" else 0))
        return d


def workspace_size(index: Index, layer: Layer, bwd: bool = False) -> int:
    n = C.c_size_t()
    d = layer.desc(bwd=bwd)
    check(lib().relnn_workspace_size(index.handle, C.byref(d), int(bwd), C.byref(n)))
    return int(n.value)


def workspace(index: Index, layer: Layer, bwd: bool = False) -> torch.Tensor:
    return torch.empty(max(1, workspace_size(index, layer, bwd)), dtype=torch.uint8, device=index.device)


def _check_embs(layer: Layer, embs: Sequence[torch.Tensor]):
    if len(embs) != len(layer.dims):
        raise ValueError("one embedding per atom is required")
    for j, e in enumerate(embs):
        if e.dtype != layer.torch_dtype or not e.is_cuda or not e.is_contiguous():
            raise TypeError(f"embedding {j} must be a contiguous {layer.torch_dtype} CUDA tensor")
        if e.dim() != 2 or e.shape[1] != layer.dims[j]:
            raise ValueError(f"embedding {j} must be [n, {layer.dims[j]}]")


def layer_fwd(index: Index, layer: Layer, embs: Sequence[torch.Tensor], W: torch.Tensor,
              b: Optional[torch.Tensor] = None, want_pre: bool = True, want_argmax: bool = True,
              ws: Optional[torch.Tensor] = None, out: Optional[torch.Tensor] = None, stream=None):
    """relnn_layer_fwd.  Returns (out [G,h], pre [G,h] or None, argmax [G,h] or None)."""
    _check_embs(layer, embs)
    if layer.transform == "product":
        W = b = None                                   # no weights
    elif W.dtype != layer.torch_dtype or W.shape != (layer.K, layer.h) or not W.is_contiguous():
        raise TypeError(f"W must be a contiguous {layer.torch_dtype} [{layer.K}, {layer.h}] tensor")
    if b is not None and (b.dtype != torch.float32 or b.numel() != layer.h):
        raise TypeError("b must be float32 [h]")
    dev = index.device
    G, h = index.G, layer.h
    if out is None:
        odt = torch.bfloat16 if layer.out_dtype == "bf16" else torch.float32
        out = torch.empty(G, h, dtype=odt, device=dev)
    pre = torch.empty(G, h, dtype=torch.float32, device=dev) if want_pre else None
    am = torch.empty(G, h, dtype=torch.int32, device=dev) if (want_argmax and layer.agg == "max") else None
    if ws is None:
        ws = workspace(index, layer, False)
    emb_arr = (C.c_void_p * len(embs))(*[e.data_ptr() for e in embs])
    d = layer.desc()
    check(lib().relnn_layer_fwd(index.handle, C.byref(d), emb_arr, _vp(W), _vp(b), _vp(out), _vp(pre),
                                _vp(am), _vp(ws), ws.numel(), _stream(stream)))
    return out, pre, am


def layer_fwd_static(index: Index, layer: Layer, embs: Sequence[torch.Tensor], W: torch.Tensor,
                     b: Optional[torch.Tensor] = None, out: torch.Tensor = None, pre: Optional[torch.Tensor] = None,
                     argmax: Optional[torch.Tensor] = None, stream=None):
    """relnn_layer_fwd_static: the forward without a workspace argument (the
    library's static per-device scratch).  The caller passes the outputs, so
    the call itself allocates nothing."""
    _check_embs(layer, embs)
    if W.dtype != layer.torch_dtype or W.shape != (layer.K, layer.h) or not W.is_contiguous():
        raise TypeError(f"W must be a contiguous {layer.torch_dtype} [{layer.K}, {layer.h}] tensor")
    if b is not None and (b.dtype != torch.float32 or b.numel() != layer.h):
        raise TypeError("b must be float32 [h]")
    G, h = index.G, layer.h
    odt = torch.bfloat16 if layer.out_dtype == "bf16" else torch.float32
    if out is None or out.dtype != odt or tuple(out.shape) != (G, h) or not out.is_contiguous():
        raise TypeError(f"out must be a contiguous {odt} tensor of shape {(G, h)}")
    if pre is not None and (pre.dtype != torch.float32 or tuple(pre.shape) != (G, h) or not pre.is_contiguous()):
        raise TypeError(f"pre must be a contiguous float32 tensor of shape {(G, h)}")
    if argmax is not None and (argmax.dtype != torch.int32 or tuple(argmax.shape) != (G, h)
                               or not argmax.is_contiguous()):
        raise TypeError(f"argmax must be a contiguous int32 tensor of shape {(G, h)}")
    emb_arr = (C.c_void_p * len(embs))(*[e.data_ptr() for e in embs])
    d = layer.desc()
    check(lib().relnn_layer_fwd_static(index.handle, C.byref(d), emb_arr, _vp(W), _vp(b), _vp(out), _vp(pre),
                                       _vp(argmax), _stream(stream)))
    return out, pre, argmax


def static_scratch_bytes() -> int:
    n = C.c_size_t()
    check(lib().relnn_static_scratch_bytes(C.byref(n)))
    return n.value


def layer_bwd(index: Index, layer: Layer, embs: Sequence[torch.Tensor], W: torch.Tensor,
              b: Optional[torch.Tensor], pre: Optional[torch.Tensor], argmax: Optional[torch.Tensor],
              dout: torch.Tensor, demb: Sequence[torch.Tensor], dW: Optional[torch.Tensor],
              db: Optional[torch.Tensor] = None, dw_accum: bool = False,
              ws: Optional[torch.Tensor] = None, stream=None):
    """relnn_layer_bwd.  demb entries are accumulated (+=) and may alias.
    The product transform has no weights: W, b, dW and db are ignored."""
    _check_embs(layer, embs)
    G, h = index.G, layer.h
    if layer.transform == "product":
        W = b = dW = db = None

    def f32(t, shape, what):
        if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous() or tuple(t.shape) != shape:
            raise TypeError(f"{what} must be a contiguous float32 CUDA tensor of shape {shape}")

    f32(dout, (G, h), "dout")
    if dW is not None:
        f32(dW, (layer.K, h), "dW")
    if db is not None:
        f32(db, (h,), "db")
    if pre is not None:
        f32(pre, (G, h), "pre")
    if argmax is not None and (argmax.dtype != torch.int32 or not argmax.is_contiguous()
                               or tuple(argmax.shape) != (G, h)):
        raise TypeError(f"argmax must be a contiguous int32 tensor of shape {(G, h)}")
    if len(demb) != len(embs):
        raise ValueError("one gradient buffer per atom is required")
    for j, (g, e) in enumerate(zip(demb, embs)):
        f32(g, tuple(e.shape), f"demb[{j}]")
    if ws is None:
        ws = workspace(index, layer, True)
    emb_arr = (C.c_void_p * len(embs))(*[e.data_ptr() for e in embs])
    demb_arr = (C.c_void_p * len(demb))(*[g.data_ptr() for g in demb])
    d = layer.desc(dw_accum=dw_accum, bwd=True)
    check(lib().relnn_layer_bwd(index.handle, C.byref(d), emb_arr, _vp(W), _vp(b), _vp(pre), _vp(argmax),
                                _vp(dout), demb_arr, _vp(dW), _vp(db), _vp(ws), ws.numel(),
                                _stream(stream)))


class RelLayerFn(torch.autograd.Function):
    """out = layer(embs; W, b) with the hand-written backward of librelnn.

    Usage: RelLayerFn.apply(index, layer, W, b, *embs).  Gradients flow to
    W, b and every embedding (FP32 master gradients; autograd casts them to
    the parameter dtype).  Atoms that share one tensor get one buffer."""

    @staticmethod
    def forward(ctx, index: Index, layer: Layer, W, b, *embs):
        out, pre, am = layer_fwd(index, layer, embs, W, b, want_pre=layer.act_post != "none",
                                 want_argmax=True)
        ctx.index, ctx.layer = index, layer
        ctx.save_for_backward(W, b, pre, am, *embs)
        return out

    @staticmethod
    def backward(ctx, dout):
        W, b, pre, am, *embs = ctx.saved_tensors
        index, layer = ctx.index, ctx.layer
        dev = dout.device
        bufs, grads = {}, []
        for e in embs:
            key = e.data_ptr()
            if key not in bufs:
                bufs[key] = torch.zeros(e.shape, dtype=torch.float32, device=dev)
                grads.append(bufs[key])
            else:
                grads.append(None)
        demb = [bufs[e.data_ptr()] for e in embs]
        # the ABI takes an FP32 gradient (a bf16 output receives a bf16 one)
        dout = dout.to(torch.float32).contiguous()
        if layer.transform == "product":                 # no weights
            layer_bwd(index, layer, embs, None, None, pre, am, dout, demb, None)
            return (None, None, None, None) + tuple(grads)
        dW = torch.empty(layer.K, layer.h, dtype=torch.float32, device=dev)
        db = torch.empty(layer.h, dtype=torch.float32, device=dev) if b is not None else None
        layer_bwd(index, layer, embs, W, b, pre, am, dout, demb, dW, db)
        return (None, None, dW, db) + tuple(grads)


def timing_enable(on: bool = True):
    """relnn_timing_enable: bracket the main kernels with HIP events."""
    check(lib().relnn_timing_enable(int(on)))


def timing_reset():
    check(lib().relnn_timing_reset())


def timing_read(kernel: str):
    """(total milliseconds, launches) of one kernel class since the reset."""
    ms, n = C.c_double(), C.c_int64()
    check(lib().relnn_timing_read(kernel.encode(), C.byref(ms), C.byref(n)))
    return ms.value, n.value


class Server:
    """relnn_serve_*: continuous-batching server of the two-layer ER network
    on sampled two-hop neighbourhoods (semantics in include/relnn.h).

    The resident tensors (Buys columns, BelongsTo, embeddings, weights) stay
    owned by the caller; this object keeps references to them."""

    def __init__(self, buys_user, buys_item, item_cat, user, item, cat, W_user, W_item1, W_item2,
                 b_user=None, b_item1=None, b_item2=None, fanout1=15, fanout2=10, dtype="f32",
                 max_seeds=4096, max_slots=64, budget_bytes=64 << 30):
        import numpy as np

        lib()
        self._np = np
        self._keep = [buys_user, buys_item, item_cat, user, item, cat, W_user, W_item1, W_item2,
                      b_user, b_item1, b_item2]
        d = L.ServeDesc()
        d.n_user, d.n_item, d.n_cat = user.shape[0], item.shape[0], cat.shape[0]
        d.n_buys = buys_user.numel()
        d.buys_user, d.buys_item, d.item_cat = (_i32(buys_user, "buys_user").data_ptr(),
                                                _i32(buys_item, "buys_item").data_ptr(),
                                                _i32(item_cat, "item_cat").data_ptr())
        d.user_emb, d.item_emb, d.cat_emb = user.data_ptr(), item.data_ptr(), cat.data_ptr()
        d.d, d.h = user.shape[1], W_user.shape[1]
        d.W_user, d.W_item1, d.W_item2 = W_user.data_ptr(), W_item1.data_ptr(), W_item2.data_ptr()
        d.b_user = None if b_user is None else b_user.data_ptr()
        d.b_item1 = None if b_item1 is None else b_item1.data_ptr()
        d.b_item2 = None if b_item2 is None else b_item2.data_ptr()
        d.fanout1, d.fanout2 = fanout1, fanout2
        d.dtype = _DTYPES[dtype][0]
        d.max_seeds, d.max_slots, d.budget_bytes = max_seeds, max_slots, int(budget_bytes)
        self.h = d.h
        self._handle = None
        h = C.c_void_p()
        check(lib().relnn_serve_create(C.byref(d), C.byref(h)))
        self._handle = h

    def submit(self, seeds, req_seed: int) -> int:
        np = self._np
        a = np.ascontiguousarray(seeds, dtype=np.int32)
        t = C.c_uint64()
        check(lib().relnn_serve_submit(self._handle, a.ctypes.data_as(C.c_void_p), int(a.size),
                                       C.c_uint64(req_seed & ((1 << 64) - 1)), C.byref(t)))
        return t.value

    def poll(self, ticket: int, n: int):
        """None while not ready, else (out [n, h] float32, present [n] bool, stats dict)."""
        np = self._np
        out = np.empty((n, self.h), np.float32)
        pres = np.empty(n, np.uint8)
        st = L.ReqStats()
        r = lib().relnn_serve_poll(self._handle, C.c_uint64(ticket), out.ctypes.data_as(C.c_void_p),
                                   pres.ctypes.data_as(C.c_void_p), C.byref(st))
        if r == L.E_NOT_READY:
            return None
        check(r)
        stats = {k: getattr(st, k) for k, _ in L.ReqStats._fields_}
        return out, pres.astype(bool), stats

    def cancel(self, ticket: int) -> bool:
        """Cancel a request; True if it was taken into a step already (its
        result is dropped), False if it was still queued (it never runs)."""
        adm = C.c_int32()
        check(lib().relnn_serve_cancel(self._handle, C.c_uint64(ticket), C.byref(adm)))
        return bool(adm.value)

    def wait(self, ticket: int, n: int, timeout_s: float = 120.0, poll_s: float = 0.0002):
        import time

        t0 = time.perf_counter()
        while True:
            r = self.poll(ticket, n)
            if r is not None:
                return r
            if time.perf_counter() - t0 > timeout_s:
                raise TimeoutError(f"request {ticket} not done after {timeout_s}s")
            time.sleep(poll_s)

    def close(self):
        if self._handle is not None and _lib_alive():
            check(lib().relnn_serve_destroy(self._handle))
        self._handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
