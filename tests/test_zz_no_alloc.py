"""The allocation-free forward (relnn_layer_fwd_static, through the C ABI)
against relnn_layer_fwd: the same results bit for bit, on two calls in a
row (the second smaller, so the static scratch holds the first call's
contents when it starts), FP32 and BF16, SUM and MAX with maximiser
positions; and the size and mode limits."""
import numpy as np
import pytest

import relgen
from tests.helpers import distinct_embs, gpu_index, gpu_layer, to_dev

pytestmark = pytest.mark.gpu


def both(rule, dtype):
    import torch

    from paper_2605_24207_amd import layer_fwd, layer_fwd_static

    gi = gpu_index(rule)
    lay = gpu_layer(rule, dtype)
    embs = distinct_embs(rule, dtype)
    W, b = to_dev(rule.W, dtype), to_dev(rule.b)
    out, pre, am = layer_fwd(gi, lay, embs, W, b)
    s_out = torch.full_like(out, float("nan"))
    s_pre = torch.full_like(pre, float("nan"))
    s_am = torch.full_like(am, -7) if am is not None else None
    layer_fwd_static(gi, lay, embs, W, b, s_out, s_pre, s_am)
    torch.cuda.synchronize()
    assert torch.equal(out, s_out) and torch.equal(pre, s_pre)
    if am is not None:
        assert torch.equal(am, s_am)
    return gi.E


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_static_forward_equals_workspace_forward_two_calls(dtype):
    g = relgen.er_graph(seed=8, n_user=30_000, n_item=10_000, n_cat=40, n_buys=300_000, n_layers=1)
    big = both(relgen.er_item_rule(g), dtype)                          # K = 384, SUM, many tiles
    small = both(relgen.node_edge(seed=9, d=32, h=32, agg="max", bias_std=0.3), dtype)   # MAX, argmax
    assert big > 10 * small


def test_static_forward_limits():
    import torch

    from paper_2605_24207_amd import RelnnError, layer_fwd_static, static_scratch_bytes, workspace_size

    assert static_scratch_bytes() == 32 << 20
    rule = relgen.node_edge(seed=10, n_nodes=4000, n_edges=200_000, d=64, h=64)
    gi = gpu_index(rule)
    embs = distinct_embs(rule, "f32")
    W, b = to_dev(rule.W), to_dev(rule.b)
    out = torch.empty(gi.G, 64, device="cuda")
    with pytest.raises(RelnnError, match="UNSUPPORTED"):          # a library GEMM may allocate
        layer_fwd_static(gi, gpu_layer(rule, "f32", plain=True), embs, W, b, out)
    push = gpu_layer(rule, "f32", pushdown=True)                   # node products: 4000 x 64 x 4 bytes: fits
    assert workspace_size(gi, push, False) <= 32 << 20
    layer_fwd_static(gi, push, embs, W, b, out)
    big = relgen.node_edge(seed=11, n_nodes=600_000, n_edges=700_000, d=64, h=64)
    gb = gpu_index(big)
    lay = gpu_layer(big, "f32", pushdown=True)                      # 2 x 600k x 64 x 4 bytes: too large
    assert workspace_size(gb, lay, False) > 32 << 20
    ob = torch.empty(gb.G, 64, device="cuda")
    with pytest.raises(RelnnError, match="RANGE"):
        layer_fwd_static(gb, lay, distinct_embs(big, "f32"), to_dev(big.W), to_dev(big.b), ob)
    torch.cuda.synchronize()
