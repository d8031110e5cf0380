"""GPU parity of the product transform (RELNN_TF_PRODUCT, through the C
ABI): tau = z_1 * ... * z_k elementwise, aggregated with SUM, MEAN or MAX
(with maximiser positions), FP32 within 1e-5 and BF16 within 2e-2 of the
FP64 oracle; two and three atoms; ReLU per tuple; a group spanning many
waves' ranges; the backward is refused."""
import numpy as np
import pytest

import relgen
from oracle import relnn_oracle as orc
from tests.helpers import distinct_embs, gpu_index, rel_rows, to_dev

pytestmark = pytest.mark.gpu

TOL = {"f32": 1e-5, "bf16": 2e-2}


def run(rule, dtype):
    import torch

    from paper_2605_24207_amd import Layer, layer_fwd

    gi = gpu_index(rule, bwd=True)
    lay = Layer([a.d for a in rule.atoms], rule.h, dtype, rule.agg, rule.act_pre, rule.act_post, transform="product")
    out, pre, am = layer_fwd(gi, lay, distinct_embs(rule, dtype), None)
    torch.cuda.synchronize()
    return gi, lay, out.cpu().numpy(), pre.cpu().numpy(), None if am is None else am.cpu().numpy()


def check(rule, dtype):
    gi, lay, out, pre, am = run(rule, dtype)
    idx = orc.build_index(rule)
    embs = [a.emb for a in rule.atoms]
    o_out, o_pre, o_am = orc.layer_fwd(idx, embs, None, None, rule.agg, rule.act_pre, rule.act_post, tf="product")
    # the product of two N(0,1) rows cancels freely in a sum: judge each row
    # against the sum of the magnitudes of its terms
    _, mag, _ = orc.layer_fwd(idx, [np.abs(e) for e in embs], None, None,
                              "max" if rule.agg == "max" else rule.agg, "none", "none", tf="product")
    assert rel_rows(pre, o_pre, scale_ref=mag).max() <= TOL[dtype]
    assert rel_rows(out, o_out, scale_ref=mag).max() <= TOL[dtype]
    if rule.agg == "max":
        if dtype == "f32":
            assert (am == o_am).mean() > 0.999
        y = orc.product(idx, embs, slice(None), rule.act_pre)
        picked = y[am.reshape(-1), np.tile(np.arange(rule.h), len(am))].reshape(am.shape)
        assert np.abs(picked - o_pre).max() <= 4 * TOL[dtype] * np.abs(o_pre).max()
    return gi, lay


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
@pytest.mark.parametrize("agg", ["sum", "mean", "max"])
def test_product_two_atoms(agg, dtype):
    rule = relgen.node_edge(seed=40, n_nodes=3000, n_edges=80_000, d=64, h=64, agg=agg, act_post="relu")
    check(rule, dtype)


def test_product_three_atoms_relu_and_hot_group():
    """Item(i; mean(relu(z_u * z_i * z_c))) over Buys with a hot item."""
    g = relgen.er_graph(seed=9, n_user=20_000, n_item=5000, n_cat=40, n_buys=300_000, n_layers=1)
    rule = relgen.er_item_rule(g)
    rule.agg, rule.act_pre = "mean", "relu"
    rule.W = np.zeros((3 * 128, 128), np.float32)
    gi, _ = check(rule, "f32")
    assert np.diff(gi.export()["offsets"].cpu().numpy()).max() > 10_000


def test_product_backward_is_refused():
    import torch

    from paper_2605_24207_amd import RelnnError, layer_bwd

    rule = relgen.node_edge(seed=41, d=32, h=32)
    gi, lay, out, pre, am = run(rule, "f32")
    z = distinct_embs(rule)[0]
    with pytest.raises(RelnnError, match="UNSUPPORTED"):
        layer_bwd(gi, lay, [z, z], to_dev(np.zeros((64, 32), np.float32)), None, torch.from_numpy(pre).cuda(), None,
                  torch.zeros(gi.G, 32, device="cuda"), [torch.zeros_like(z)] * 2,
                  torch.zeros(64, 32, device="cuda"))
