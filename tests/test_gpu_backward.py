"""GPU parity of the hand-written backward (through the C ABI) against the
FP64 oracle gradient: dW, db and every embedding gradient, FP32 within 1e-5
and BF16 within 2e-2 (relative, Frobenius for dW / db, per row for the
embeddings), plus the autograd.Function wrapper on a two-layer net."""
import numpy as np
import pytest

import relgen
from oracle import relnn_oracle as orc
from tests.helpers import distinct_embs, gpu_index, gpu_layer, oracle_inputs, to_dev

pytestmark = pytest.mark.gpu

TOL = {"f32": 1e-5, "bf16": 2e-2}
# BF16 layers run the backward products on bf16 operands with FP32
# accumulation: each operand the kernel forms in FP32 (the summed gradient
# rows, the per-group sums of the joined rows) is rounded once to bf16,
# a relative error of at most 2^-9 per element.  With two rounded operands
# per product the expected relative error of a gradient row is about
# 2^-9 sqrt(2/3) = 1.6e-3; against the oracle run on the bf16-rounded inputs
# (the kernel's own arithmetic) the check allows 4 * 2^-9.
TOL_BF16_KERNEL = 4 * 2.0 ** -9


def fro(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)


def row_err(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    nb = np.linalg.norm(b, axis=1)
    den = np.maximum(nb, 1e-3 * np.median(nb[nb > 0]) if np.any(nb > 0) else 1.0)
    return np.linalg.norm(a - b, axis=1) / den


def run_bwd(rule, dtype, dout_seed=0, dw_accum=False):
    import torch

    from paper_2605_24207_amd import layer_bwd, layer_fwd

    idx = gpu_index(rule, bwd=True)
    layer = gpu_layer(rule, dtype)
    embs = distinct_embs(rule, dtype)
    W, b = to_dev(rule.W, dtype), to_dev(rule.b)
    out, pre, am = layer_fwd(idx, layer, embs, W, b)
    dout = torch.from_numpy(np.random.default_rng(dout_seed).standard_normal((idx.G, rule.h)).astype(np.float32)).cuda()
    uniq = {}
    demb = []
    for e in embs:
        if e.data_ptr() not in uniq:
            uniq[e.data_ptr()] = torch.zeros(e.shape, dtype=torch.float32, device="cuda")
        demb.append(uniq[e.data_ptr()])
    dW = torch.full((rule.K, rule.h), 0.5 if dw_accum else float("nan"), dtype=torch.float32, device="cuda")
    db = torch.full((rule.h,), 0.5 if dw_accum else float("nan"), dtype=torch.float32, device="cuda")
    layer_bwd(idx, layer, embs, W, b, pre, am, dout, demb, dW, db, dw_accum=dw_accum)
    torch.cuda.synchronize()
    decisions = (pre.cpu().numpy().astype(np.float64), None if am is None else am.cpu().numpy())
    return (dout.cpu().numpy().astype(np.float64), [d.cpu().numpy() for d in demb], dW.cpu().numpy(),
            db.cpu().numpy(), decisions)


def oracle_bwd(rule, dtype, dout, decisions=None):
    """Oracle gradient.  ``decisions`` = (pre, argmax) of the kernel's forward:
    the ReLU-after-aggregate mask and the MAX routing are then taken from
    the kernel, so both sides make those integer decisions in the kernel's
    precision.  With decisions, the per-tuple act_pre' mask (which the kernel
    recomputes and does not export) is taken in the kernel's precision too:
    from the bf16-rounded inputs."""
    idx = orc.build_index(rule)
    embs, W, b = oracle_inputs(rule, dtype)
    _, pre, am = orc.layer_fwd(idx, embs, W, b, rule.agg, rule.act_pre, rule.act_post)
    mask = None
    if decisions is not None:
        pre, am = decisions[0], (decisions[1] if rule.agg == "max" else am)
        if rule.act_pre != "none":
            embs_k, W_k, _ = oracle_inputs(rule, "bf16")
            mask = orc.act_pre_mask(idx, embs_k, W_k, b)
    demb, dW, db = orc.layer_bwd(idx, embs, W, b, pre, am, dout, rule.agg, rule.act_pre, rule.act_post,
                                 pre_mask=mask)
    # atoms sharing one relation: one gradient buffer
    tot = {}
    for a, g in zip(rule.atoms, demb):
        tot[id(a.emb)] = tot.get(id(a.emb), 0) + g
    return [tot[id(a.emb)] for a in rule.atoms], dW, db


def compare(got, ref, tol):
    demb, dW, db = got
    r_demb, r_dW, r_db = ref
    assert fro(dW, r_dW) <= tol, fro(dW, r_dW)
    assert fro(db, r_db) <= tol, fro(db, r_db)
    for g, r in zip(demb, r_demb):
        e = row_err(g, r)
        assert e.max() <= tol, (e.max(), np.percentile(e, 99))


def check(rule, dtype, dw_accum=False):
    dout, demb, dW, db, dec = run_bwd(rule, dtype, dw_accum=dw_accum)
    if dw_accum:
        dW = dW - 0.5
        db = db - 0.5
    got = (demb, dW, db)
    if dtype == "f32":
        compare(got, oracle_bwd(rule, "f32", dout), TOL["f32"])
        return
    # BF16: kernel arithmetic against the oracle on the bf16-rounded inputs ...
    compare(got, oracle_bwd(rule, "bf16", dout), TOL_BF16_KERNEL)
    # ... and against the oracle on the FP32 master values at the BF16 bound,
    # with the decisions taken in the kernel's precision
    compare(got, oracle_bwd(rule, "f32", dout, dec), TOL["bf16"])


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
@pytest.mark.parametrize("agg", ["sum", "mean", "max"])
@pytest.mark.parametrize("acts", [("none", "relu"), ("relu", "none")])
def test_bwd_node_edge(dtype, agg, acts):
    rule = relgen.node_edge(seed=21, agg=agg, act_pre=acts[0], act_post=acts[1], bias_std=0.3)
    check(rule, dtype)


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
@pytest.mark.parametrize("agg", ["sum", "max"])
def test_bwd_power_law_hot_rows(dtype, agg):
    """2k nodes / 10k edges, s ~ Zipf(1.2): hot source rows span many tiles of
    the transpose scatter."""
    p = relgen.power_graph(seed=5, n_nodes=2000, n_edges=10_000, d=128, h=128, bias_std=0.2)
    rule = relgen.power_rule(p, 0 if agg == "sum" else 1)
    check(rule, dtype)


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_bwd_er_three_atoms(dtype):
    g = relgen.er_graph(seed=4, n_user=3000, n_item=1500, n_cat=20, n_buys=40_000, n_layers=1)
    check(relgen.er_item_rule(g), dtype)
    check(relgen.er_user_rule(g), dtype)


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_bwd_max_width_not_multiple_of_32(dtype):
    """MAX routing bits with a partial last word (h = 48: 32 + 16 columns)."""
    rule = relgen.node_edge(seed=24, d=32, h=48, agg="max", act_post="relu", bias_std=0.3)
    check(rule, dtype)


@pytest.mark.parametrize("case", ["one_tuple", "one_group"])
@pytest.mark.parametrize("agg", ["sum", "mean", "max"])
def test_bwd_degenerate_sizes(case, agg):
    """Backward of a one-tuple join, and of one group holding every tuple."""
    n_edges = 1 if case == "one_tuple" else 20_000
    rule = relgen.node_edge(seed=32, n_nodes=300, n_edges=n_edges, agg=agg, bias_std=0.3)
    if case == "one_group":
        rule.cols[1][:] = 5
    check(rule, "f32")


def test_bwd_dw_accumulate():
    check(relgen.node_edge(seed=22, agg="mean", bias_std=0.2), "f32", dw_accum=True)


def test_bwd_large_segment_ragged():
    rule = relgen.node_edge(seed=23, n_nodes=500, n_edges=30_001, agg="sum", bias_std=0.1)
    rule.cols[0][:20_000] = 3          # one source row with 20k tuples
    rule.cols[1][20_000:25_000] = 4    # one group with 5k tuples
    check(rule, "f32")


@pytest.mark.parametrize("pushdown", [False, True])
def test_autograd_two_layer_power_net(pushdown):
    """The differentiation form on a small instance: layer 1 SUM + ReLU, layer
    2 MAX, MSE against targets; torch.autograd drives the hand-written
    backward.  Gradients of W1, W2 and z against the FP64 oracle chain, with
    the forward fused or pushed below the join (both layers are affine)."""
    import torch

    from paper_2605_24207_amd import RelLayerFn

    p = relgen.power_graph(seed=6, n_nodes=2000, n_edges=10_000, d=128, h=128)
    dev = "cuda"
    s = torch.from_numpy(p.s).to(dev)
    t = torch.from_numpy(p.t).to(dev)
    from paper_2605_24207_amd import Index, Layer

    n = p.z.shape[0]
    ix1 = Index([s, t], [(n, 0, None), (n, 1, None)], 1, bwd=True)
    keys1 = ix1.export()["group_keys"]
    ix2 = Index([s, t], [(ix1.G, 0, keys1), (ix1.G, 1, keys1)], 1, bwd=True)
    L1 = Layer([128, 128], 128, "f32", "sum", "none", "relu", pushdown=pushdown)
    L2 = Layer([128, 128], 128, "f32", "max", "none", "none", pushdown=pushdown)
    z = torch.from_numpy(p.z).to(dev).requires_grad_(True)
    W1 = torch.from_numpy(p.W[0]).to(dev).requires_grad_(True)
    W2 = torch.from_numpy(p.W[1]).to(dev).requires_grad_(True)
    b1 = torch.from_numpy(p.b[0]).to(dev).requires_grad_(True)
    b2 = torch.from_numpy(p.b[1]).to(dev).requires_grad_(True)
    h1 = RelLayerFn.apply(ix1, L1, W1, b1, z, z)
    h2 = RelLayerFn.apply(ix2, L2, W2, b2, h1, h1)
    keys2 = ix2.export()["group_keys"].long()
    target = torch.from_numpy(p.target).to(dev)[keys2]
    loss = ((h2 - target) ** 2).mean()
    loss.backward()

    # oracle chain in FP64
    r1 = relgen.power_rule(p, 0)
    i1 = orc.build_index(r1)
    o1, pre1, am1 = orc.layer_fwd(i1, [p.z, p.z], p.W[0], p.b[0], "sum", "none", "relu")
    r2 = relgen.power_rule(p, 1, z=o1, z_keys=i1.group_keys.astype(np.int32))
    i2 = orc.build_index(r2)
    o2, pre2, am2 = orc.layer_fwd(i2, [o1, o1], p.W[1], p.b[1], "max", "none", "none")
    tg = p.target[i2.group_keys].astype(np.float64)
    dout2 = 2.0 * (o2 - tg) / o2.size
    d2, dW2, db2 = orc.layer_bwd(i2, [o1, o1], p.W[1], p.b[1], pre2, am2, dout2, "max", "none", "none")
    dout1 = d2[0] + d2[1]
    d1, dW1, db1 = orc.layer_bwd(i1, [p.z, p.z], p.W[0], p.b[0], pre1, am1, dout1, "sum", "none", "relu")
    assert fro(W2.grad.cpu().numpy(), dW2) <= 1e-5
    assert fro(b2.grad.cpu().numpy(), db2) <= 1e-5
    assert fro(W1.grad.cpu().numpy(), dW1) <= 1e-5
    assert fro(b1.grad.cpu().numpy(), db1) <= 1e-5
    assert row_err(z.grad.cpu().numpy(), d1[0] + d1[1]).max() <= 1e-5


def test_autograd_bf16_chain_matches_explicit_calls():
    """BF16 two-layer net through RelLayerFn: layer 1 writes a bf16 output
    that layer 2 reads, so autograd hands layer 1 a bf16 gradient, which the
    binding widens to the FP32 gradient the ABI takes.  The gradients equal,
    bit for bit, those of explicit layer_fwd / layer_bwd calls that apply the
    same rounding (the per-layer BF16 arithmetic is checked against the
    oracle by the tests above)."""
    import torch

    from paper_2605_24207_amd import Index, Layer, RelLayerFn, layer_bwd, layer_fwd

    p = relgen.power_graph(seed=7, n_nodes=2000, n_edges=10_000, d=128, h=128)
    dev = "cuda"
    s = torch.from_numpy(p.s).to(dev)
    t = torch.from_numpy(p.t).to(dev)
    n = p.z.shape[0]
    ix1 = Index([s, t], [(n, 0, None), (n, 1, None)], 1, bwd=True)
    keys1 = ix1.export()["group_keys"]
    ix2 = Index([s, t], [(ix1.G, 0, keys1), (ix1.G, 1, keys1)], 1, bwd=True)
    L1 = Layer([128, 128], 128, "bf16", "sum", "none", "relu", out_dtype="bf16")
    L2 = Layer([128, 128], 128, "bf16", "max", "none", "none")
    bf = lambda a: torch.from_numpy(a).to(dev).to(torch.bfloat16)
    z0, W10, W20 = bf(p.z), bf(p.W[0]), bf(p.W[1])
    b10 = torch.from_numpy(p.b[0]).to(dev)
    b20 = torch.from_numpy(p.b[1]).to(dev)
    C = torch.from_numpy(np.random.default_rng(5).standard_normal((ix2.G, 128)).astype(np.float32)).to(dev)

    z, W1, W2 = (x.clone().requires_grad_(True) for x in (z0, W10, W20))
    b1, b2 = (x.clone().requires_grad_(True) for x in (b10, b20))
    h1 = RelLayerFn.apply(ix1, L1, W1, b1, z, z)
    h2 = RelLayerFn.apply(ix2, L2, W2, b2, h1, h1)
    assert h1.dtype == torch.bfloat16 and h2.dtype == torch.float32
    (h2 * C).sum().backward()

    o1, pre1, am1 = layer_fwd(ix1, L1, [z0, z0], W10, b10)
    o2, pre2, am2 = layer_fwd(ix2, L2, [o1, o1], W20, b20)
    dh1 = torch.zeros(o1.shape, dtype=torch.float32, device=dev)
    dW2 = torch.empty(256, 128, device=dev)
    db2 = torch.empty(128, device=dev)
    layer_bwd(ix2, L2, [o1, o1], W20, b20, pre2, am2, C, [dh1, dh1], dW2, db2)
    dout1 = dh1.to(torch.bfloat16).to(torch.float32)          # the gradient of a bf16 tensor
    dz = torch.zeros(z0.shape, dtype=torch.float32, device=dev)
    dW1 = torch.empty(256, 128, device=dev)
    db1 = torch.empty(128, device=dev)
    layer_bwd(ix1, L1, [z0, z0], W10, b10, pre1, am1, dout1, [dz, dz], dW1, db1)
    torch.cuda.synchronize()
    assert torch.equal(h2.detach(), o2)
    assert torch.equal(W2.grad, dW2.to(torch.bfloat16)) and torch.equal(b2.grad, db2)
    assert torch.equal(W1.grad, dW1.to(torch.bfloat16)) and torch.equal(b1.grad, db1)
    assert torch.equal(z.grad, dz.to(torch.bfloat16))


def test_backward_rejects_wrong_gradient_dtype():
    """The ABI reads dout as FP32: another dtype is refused, not reinterpreted."""
    import torch

    from paper_2605_24207_amd import layer_bwd, layer_fwd

    rule = relgen.node_edge(agg="sum")
    gi = gpu_index(rule, bwd=True)
    layer = gpu_layer(rule, "f32")
    embs = distinct_embs(rule, "f32")
    W, b = to_dev(rule.W), to_dev(rule.b)
    out, pre, am = layer_fwd(gi, layer, embs, W, b)
    dz = torch.zeros_like(embs[0])
    with pytest.raises(TypeError, match="dout"):
        layer_bwd(gi, layer, [embs[0], embs[0]], W, b, pre, am, out.to(torch.bfloat16), [dz, dz],
                  torch.empty_like(W), torch.empty_like(b))

