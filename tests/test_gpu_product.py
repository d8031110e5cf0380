"""GPU parity of the product transform (RELNN_TF_PRODUCT, through the C
ABI): tau = z_1 * ... * z_k elementwise, aggregated with SUM, MEAN or MAX
(with maximiser positions), FP32 within 1e-5 and BF16 within 2e-2 of the
FP64 oracle; two and three atoms; ReLU per tuple; a group spanning many
waves' ranges; the backward (embedding gradients) against the oracle's."""
import numpy as np
import pytest

import relgen
from oracle import relnn_oracle as orc
from tests.helpers import distinct_embs, gpu_index, oracle_inputs, rel_rows, to_dev

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


def run_bwd(rule, dtype, dout_seed=3):
    """Forward, then relnn_layer_bwd with no weights; one gradient buffer per
    distinct relation (a self-join adds both roles into it)."""
    import torch

    from paper_2605_24207_amd import layer_bwd

    gi, lay, out, pre, am = run(rule, dtype)
    embs = distinct_embs(rule, dtype)
    dout = np.random.default_rng(dout_seed).standard_normal((gi.G, rule.h)).astype(np.float32)
    uniq, demb = {}, []
    for e in embs:
        if e.data_ptr() not in uniq:
            uniq[e.data_ptr()] = torch.zeros(e.shape, dtype=torch.float32, device="cuda")
        demb.append(uniq[e.data_ptr()])
    layer_bwd(gi, lay, embs, None, None, torch.from_numpy(pre).cuda(),
              None if am is None else torch.from_numpy(am).cuda(), to_dev(dout), demb, None)
    torch.cuda.synchronize()
    return dout.astype(np.float64), [d.cpu().numpy() for d in demb], pre, am


def oracle_grad(rule, dtype, dout, pre, am):
    """Oracle gradient per atom (summed over atoms sharing a relation) and
    the matching magnitude scale: the same gradient with |z| and |dout| and
    the per-tuple ReLU mask of the signed product, i.e. the sum of the
    magnitudes of the terms of each row.  The forward's decisions (pre for
    ReLU after the aggregate, the MAX maximisers) are the kernel's."""
    idx = orc.build_index(rule)
    embs = oracle_inputs(rule, dtype)[0]
    demb = orc.product_bwd(idx, embs, pre, am, dout, rule.agg, rule.act_pre, rule.act_post)
    mask = orc.product(idx, embs, slice(None), "none") > 0 if rule.act_pre == "relu" else None
    mag = orc.product_bwd(idx, [np.abs(e) for e in embs], pre, am, np.abs(dout), rule.agg, rule.act_pre,
                          rule.act_post, pre_mask=mask)
    tot, tmag = {}, {}
    for a, g, m in zip(rule.atoms, demb, mag):
        tot[id(a.emb)] = tot.get(id(a.emb), 0) + g
        tmag[id(a.emb)] = tmag.get(id(a.emb), 0) + m
    return [tot[id(a.emb)] for a in rule.atoms], [tmag[id(a.emb)] for a in rule.atoms]


def check_bwd(rule, dtype):
    dout, demb, pre, am = run_bwd(rule, dtype)
    # the kernel's arithmetic is FP32 on the layer's stored values: against
    # the oracle on those values (bf16-rounded for a BF16 layer) it is held
    # to the FP32 bound ...
    ref, mag = oracle_grad(rule, dtype, dout, pre, am)
    for g, r, m in zip(demb, ref, mag):
        assert rel_rows(g, r, scale_ref=m).max() <= TOL["f32"]
    # ... and against the FP32 master values to the layer's own bound
    if dtype == "bf16":
        ref, mag = oracle_grad(rule, "f32", dout, pre, am)
        for g, r, m in zip(demb, ref, mag):
            assert rel_rows(g, r, scale_ref=m).max() <= TOL["bf16"]
    # rows that no tuple joins get no gradient
    idx = orc.build_index(rule)
    for a, g, r in zip(rule.atoms, demb, idx.rows):
        joined = np.zeros(len(g), bool)
        for b, rr in zip(rule.atoms, idx.rows):
            if b.emb is a.emb:
                joined[rr] = True
        assert not np.any(g[~joined])


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
@pytest.mark.parametrize("agg", ["sum", "mean", "max"])
@pytest.mark.parametrize("acts", [("none", "relu"), ("relu", "none")])
def test_product_backward_self_join(agg, dtype, acts):
    """Node(t; agg(act_pre(z_s * z_t))) over an edge relation: both atoms
    read one relation, so its gradient sums both roles."""
    rule = relgen.node_edge(seed=42, n_nodes=3000, n_edges=80_000, d=64, h=64, agg=agg, act_pre=acts[0],
                            act_post=acts[1])
    check_bwd(rule, dtype)


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_product_backward_three_atoms_hot_group(dtype):
    """Item(i; mean(relu(z_u * z_i * z_c))) over Buys with a hot item: the
    item's gradient row sums tens of thousands of tuples across many waves'
    ranges (carries and the fix-up)."""
    g = relgen.er_graph(seed=9, n_user=20_000, n_item=5000, n_cat=40, n_buys=300_000, n_layers=1)
    rule = relgen.er_item_rule(g)
    rule.agg, rule.act_pre = "mean", "relu"
    rule.W = np.zeros((3 * 128, 128), np.float32)
    check_bwd(rule, dtype)


def four_atom_rule(agg, act_pre, seed=46, n_link=40_000, h=32):
    """T(a; agg(act_pre(z_a * z_b * z_c * z_d))) over a link relation with
    four columns into four relations of different sizes (the most atoms a
    rule may have)."""
    rng = np.random.default_rng(seed)
    sizes = [3000, 5000, 200, 40]
    cols = [rng.integers(0, n, n_link).astype(np.int32) for n in sizes]
    atoms = [relgen.Atom(j, rng.standard_normal((n, h)).astype(np.float32)) for j, n in enumerate(sizes)]
    return relgen.Rule(cols=cols, atoms=atoms, group_col=0, W=np.zeros((4 * h, h), np.float32),
                       b=np.zeros(h, np.float32), agg=agg, act_pre=act_pre)


@pytest.mark.parametrize("agg", ["sum", "max"])
@pytest.mark.parametrize("act_pre", ["none", "relu"])
def test_product_four_atoms(agg, act_pre):
    rule = four_atom_rule(agg, act_pre)
    check(rule, "f32")
    check_bwd(rule, "f32")


@pytest.mark.parametrize("agg", ["mean", "max"])
def test_product_backward_no_group_constant_atom(agg):
    """Grouped by a link column that no atom reads: every atom varies inside
    a group (one pass per atom over its transpose order)."""
    rng = np.random.default_rng(47)
    n_link, h = 30_000, 32
    cols = [rng.integers(0, 4000, n_link).astype(np.int32), rng.integers(0, 700, n_link).astype(np.int32),
            rng.integers(0, 2500, n_link).astype(np.int32)]
    atoms = [relgen.Atom(0, rng.standard_normal((4000, h)).astype(np.float32)),
             relgen.Atom(1, rng.standard_normal((700, h)).astype(np.float32))]
    rule = relgen.Rule(cols=cols, atoms=atoms, group_col=2, W=np.zeros((2 * h, h), np.float32),
                       b=np.zeros(h, np.float32), agg=agg, act_pre="relu")
    check(rule, "f32")
    check_bwd(rule, "f32")


@pytest.mark.parametrize("h", [16, 48, 144])
def test_product_backward_ragged_width(h):
    """Widths that leave lanes idle in the last 128-column pass (rows stay
    multiples of 16, as every layer requires)."""
    rule = relgen.node_edge(seed=43, n_nodes=500, n_edges=6000, d=h, h=h, agg="max", act_post="none")
    check_bwd(rule, "f32")


@pytest.mark.parametrize("case", ["empty", "one_tuple", "one_group"])
def test_product_backward_degenerate(case):
    """No tuple (the gradients stay zero), one tuple, and one group holding
    every tuple."""
    n_edges = {"empty": 0, "one_tuple": 1, "one_group": 20_000}[case]
    rule = relgen.node_edge(seed=44, n_nodes=300, n_edges=n_edges, d=32, h=32, agg="mean")
    if case == "one_group":
        rule.cols[1][:] = 5
    check_bwd(rule, "f32")


def test_product_autograd_matches_explicit_call():
    """RelLayerFn over a product layer returns no weight gradients and the
    embedding gradient of an explicit relnn_layer_bwd call."""
    import torch

    from paper_2605_24207_amd import RelLayerFn

    rule = relgen.node_edge(seed=45, n_nodes=800, n_edges=9000, d=32, h=32, agg="sum", act_post="relu")
    gi, lay, _, _, _ = run(rule, "f32")
    z = to_dev(rule.atoms[0].emb).requires_grad_(True)
    out = RelLayerFn.apply(gi, lay, None, None, z, z)
    dout = np.random.default_rng(3).standard_normal((gi.G, rule.h)).astype(np.float32)
    out.backward(to_dev(dout))
    ref, mag = oracle_grad(rule, "f32", dout.astype(np.float64), out.detach().cpu().numpy(), None)
    assert rel_rows(z.grad.cpu().numpy(), ref[0], scale_ref=mag[0]).max() <= TOL["f32"]
