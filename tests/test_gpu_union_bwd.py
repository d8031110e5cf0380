"""GPU parity of the union's backward (relnn_union_bwd, through the C ABI)
against the FP64 oracle's: every branch's W, b and embedding gradients and
the union rule's W_post, b_post, FP32 within 1e-5 and BF16 within 2e-2
(relative, Frobenius for weights, per row against the sum of the terms'
magnitudes for embeddings).  The forward's
decisions (the aggregate for ReLU after it, the MAX maximisers, ReLU of the
union rule's transform) are the kernel's.  Also: the union's MAX
maximisers against the oracle's, embeddings shared across branches, the
self-union, an empty branch and the autograd wrapper."""
import numpy as np
import pytest

import relgen
from oracle import relnn_oracle as orc
from tests.helpers import gpu_index, gpu_layer, oracle_inputs, rel_rows, to_dev
from tests.test_gpu_union import er_rules

pytestmark = pytest.mark.gpu

TOL = {"f32": 1e-5, "bf16": 2e-2}
# BF16 branch layers run their backward products on bf16 operands with
# FP32 accumulation (two operands rounded once each, at most 2^-9 apart
# relative): against the oracle on the bf16-rounded inputs the check allows
# 4 * 2^-9, as for the layer backward.
TOL_BF16_KERNEL = 4 * 2.0 ** -9


def fro(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)


def run(rules, agg, dtype, act_post="relu", post=None, seed=0):
    """Union forward then backward on the GPU.  Embedding arrays shared by
    atoms or by branches share one device tensor and one gradient buffer."""
    import torch

    from paper_2605_24207_amd import Union, union_bwd, union_fwd

    U = Union([gpu_index(r, bwd=True) for r in rules])
    layers = [gpu_layer(r, dtype) for r in rules]
    dev, grad = {}, {}
    for r in rules:
        for a in r.atoms:
            if id(a.emb) not in dev:
                dev[id(a.emb)] = to_dev(a.emb, dtype)
                grad[id(a.emb)] = torch.zeros(a.emb.shape, dtype=torch.float32, device="cuda")
    embs = [[dev[id(a.emb)] for a in r.atoms] for r in rules]
    demb = [[grad[id(a.emb)] for a in r.atoms] for r in rules]
    Ws = [to_dev(r.W, dtype) for r in rules]
    bs = [to_dev(r.b) for r in rules]
    W_post = b_post = dW_post = db_post = None
    h_out = rules[0].h
    if post is not None:
        W_post, b_post = to_dev(post[0]), to_dev(post[1])
        h_out = post[0].shape[1]
        dW_post = torch.full(tuple(post[0].shape), float("nan"), device="cuda")
        db_post = torch.full((h_out,), float("nan"), device="cuda")
    out, pre, am = union_fwd(U, layers, agg, act_post, embs, Ws, bs, W_post, b_post)
    dout = torch.from_numpy(np.random.default_rng(seed).standard_normal((U.G, h_out)).astype(np.float32)).cuda()
    dWs = [torch.full((r.K, r.h), float("nan"), device="cuda") for r in rules]
    dbs = [torch.full((r.h,), float("nan"), device="cuda") for r in rules]
    union_bwd(U, layers, agg, act_post, embs, Ws, bs, W_post, b_post, pre, am, dout, demb, dWs, dbs, dW_post,
              db_post)
    torch.cuda.synchronize()
    res = {"U": U, "out": out.cpu().numpy(), "pre": pre.cpu().numpy(), "dout": dout.cpu().numpy(),
           "am": None if am is None else am.cpu().numpy(),
           "demb": {k: g.cpu().numpy() for k, g in grad.items()},
           "dW": [d.cpu().numpy() for d in dWs], "db": [d.cpu().numpy() for d in dbs],
           "dW_post": None if dW_post is None else dW_post.cpu().numpy(),
           "db_post": None if db_post is None else db_post.cpu().numpy()}
    return res


def arg_pairs(rules, am):
    """The kernel's maximisers (positions in the concatenated tuple order)
    as (branch, position) pairs."""
    E = [orc.build_index(r).E for r in rules]
    base = np.concatenate([[0], np.cumsum(E)])
    br = np.searchsorted(base, am, side="right") - 1
    return np.stack([br, am - base[br]], axis=-1)


def oracle(rules, agg, res, dtype, act_post="relu", post=None, kdtype="f32"):
    """Oracle gradients on the FP32 master values or their bf16 roundings
    (dtype), with the per-tuple ReLU decisions of a BF16 kernel (kdtype)
    taken from the rounded values it holds."""
    branches, masks = [], []
    for r in rules:
        embs, W, b = oracle_inputs(r, dtype)
        idx = orc.build_index(r)
        branches.append((idx, embs, W, b, r.act_pre))
        if r.act_pre != "none" and kdtype == "bf16":         # act_pre' from the values the kernel holds
            ek, Wk, _ = oracle_inputs(r, "bf16")
            masks.append(orc.act_pre_mask(idx, ek, Wk, b))
        else:
            masks.append(None)
    arg = None if res["am"] is None else arg_pairs(rules, res["am"])
    Wp, bp = (None, None) if post is None else post
    post_mask = None if post is None else res["out"] > 0        # ReLU(u) > 0 exactly where u > 0
    grads, dWp, dbp = orc.union_bwd(branches, res["pre"], arg, res["dout"], agg, act_post, Wp, bp, masks, post_mask)
    # the magnitude of each embedding gradient's terms: the same chain with
    # |dout|, |W_post| and |W_i| and the same decisions (ReLU masks of the
    # signed values, the same maximisers)
    if post is not None and act_post == "relu":
        pm = post_mask
    else:
        pm = None
    abs_branches, abs_masks = [], []
    for (idx, embs, W, b, act), m in zip(branches, masks):
        if act != "none" and m is None:
            m = orc.act_pre_mask(idx, embs, W, b)
        abs_branches.append((idx, embs, np.abs(np.asarray(W, np.float64)), b, act))
        abs_masks.append(m)
    if post is None and act_post == "relu":                      # the mask of v itself, from the signed v
        dout_abs = np.abs(res["dout"]) * (res["pre"] > 0)
        ap = "none"
    else:
        dout_abs, ap = np.abs(res["dout"]), act_post
    mag_grads, _, _ = orc.union_bwd(abs_branches, res["pre"], arg, dout_abs, agg, ap,
                                    None if Wp is None else np.abs(np.asarray(Wp, np.float64)), bp, abs_masks, pm)
    demb, mag = {}, {}
    for r, (de, _, _), (dm, _, _) in zip(rules, grads, mag_grads):
        for a, g, m in zip(r.atoms, de, dm):
            demb[id(a.emb)] = demb.get(id(a.emb), 0) + g
            mag[id(a.emb)] = mag.get(id(a.emb), 0) + m
    return {"demb": demb, "mag": mag, "dW": [g[1] for g in grads], "db": [g[2] for g in grads],
            "dW_post": dWp, "db_post": dbp}


def compare(res, ref, tol):
    for got, want in zip(res["dW"], ref["dW"]):
        assert fro(got, want) <= tol, fro(got, want)
    for got, want in zip(res["db"], ref["db"]):
        assert fro(got, want) <= tol, fro(got, want)
    for k, want in ref["demb"].items():
        # per row, against the sum of the magnitudes of its terms: rows
        # whose terms cancel are held to the rounding their terms allow
        e = rel_rows(res["demb"][k], want, scale_ref=ref["mag"][k])
        assert e.max() <= tol, (e.max(), np.percentile(e, 99))
    if ref["dW_post"] is not None:
        assert fro(res["dW_post"], ref["dW_post"]) <= tol
        assert fro(res["db_post"], ref["db_post"]) <= tol


def check(rules, agg, dtype, act_post="relu", post=None):
    res = run(rules, agg, dtype, act_post, post)
    if dtype == "f32":
        compare(res, oracle(rules, agg, res, "f32", act_post, post), TOL["f32"])
    else:
        compare(res, oracle(rules, agg, res, "bf16", act_post, post, "bf16"), TOL_BF16_KERNEL)
        compare(res, oracle(rules, agg, res, "f32", act_post, post, "bf16"), TOL["bf16"])
    return res


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
@pytest.mark.parametrize("agg", ["mean", "sum", "max"])
def test_union_backward_two_bodies(agg, dtype):
    """Two bodies of Item(i) over User and Item embeddings that both read:
    the shared relations' gradients add the two branches' shares."""
    r1, r2 = er_rules(seed=7, n_buys=60_000)
    r2.act_pre = "relu"
    check([r1, r2], agg, dtype)


@pytest.mark.parametrize("agg,dtype", [("max", "f32"), ("mean", "f32"), ("mean", "bf16"), ("max", "bf16")])
def test_union_backward_three_branches_post_transform(agg, dtype):
    """Three bodies, then the union rule's transform 128 -> 96 and ReLU
    (FP32 W_post over bf16 branch layers in the BF16 cases)."""
    r1, r2 = er_rules(seed=8, n_buys=40_000)
    r3 = relgen.node_edge(seed=17, n_nodes=3000, n_edges=20_000, d=128, h=128, bias_std=0.1)
    rng = np.random.default_rng(4)
    post = (rng.standard_normal((128, 96)).astype(np.float32) / np.sqrt(128),
            rng.standard_normal(96).astype(np.float32))
    check([r1, r2, r3], agg, dtype, post=post)


def test_union_max_maximisers():
    """The union's MAX maximiser of each column is the first in (branch,
    position) order: against the oracle's where the maximum is unique
    beyond rounding, and a maximiser holding the maximum everywhere."""
    r1, r2 = er_rules(seed=9, n_buys=40_000)
    res = run([r1, r2], "max", "f32")
    branches = [(orc.build_index(r), *oracle_inputs(r, "f32"), r.act_pre) for r in (r1, r2)]
    _, _, o_pre, o_arg = orc.union_fwd(branches, "max", "relu")
    got = arg_pairs([r1, r2], res["am"])
    same = (got == o_arg).all(axis=-1)
    assert same.mean() > 0.999
    G, h = o_pre.shape
    for q, c in zip(*np.nonzero(~same)):
        idx, embs, W, b, act = branches[got[q, c, 0]]
        y = orc.transform(orc.gather_concat(idx, embs, [got[q, c, 1]]), W, b, act)[0, c]
        assert abs(y - o_pre[q, c]) <= 1e-5 * max(abs(o_pre[q, c]), 1.0)


def test_union_backward_self_union():
    """R united with itself: MEAN halves each copy's share; MAX routes
    everything to the first copy, so the second copy's weight gradient is
    zero."""
    rule = relgen.node_edge(seed=18, n_nodes=2000, n_edges=30_000, d=64, h=64, bias_std=0.2, act_pre="relu")
    check([rule, rule], "mean", "f32")
    res = check([rule, rule], "max", "f32")
    assert not np.any(res["dW"][1]) and not np.any(res["db"][1])


def test_union_backward_with_an_empty_branch():
    """A branch whose join is empty contributes no key, and its weight
    gradients are zero."""
    r1 = relgen.node_edge(seed=19, n_nodes=1500, n_edges=20_000, d=64, h=64, bias_std=0.2)
    r2 = relgen.node_edge(seed=20, n_nodes=1500, n_edges=0, d=64, h=64, bias_std=0.2)
    res = check([r1, r2], "sum", "f32")
    assert not np.any(res["dW"][1]) and not np.any(res["db"][1])


def test_union_autograd_matches_explicit_call():
    """UnionFn returns, bit for bit, the gradients of an explicit
    relnn_union_bwd call, for branches sharing an embedding tensor."""
    import torch

    from paper_2605_24207_amd import UnionFn

    r1, r2 = er_rules(seed=10, n_buys=30_000)
    rng = np.random.default_rng(5)
    post = (rng.standard_normal((128, 64)).astype(np.float32) / np.sqrt(128),
            rng.standard_normal(64).astype(np.float32))
    res = run([r1, r2], "mean", "f32", post=post)
    from paper_2605_24207_amd import Union

    U = Union([gpu_index(r, bwd=True) for r in (r1, r2)])
    dev = {}
    for r in (r1, r2):
        for a in r.atoms:
            dev.setdefault(id(a.emb), to_dev(a.emb).requires_grad_(True))
    Ws = [to_dev(r.W).requires_grad_(True) for r in (r1, r2)]
    bs = [to_dev(r.b).requires_grad_(True) for r in (r1, r2)]
    Wp, bp = to_dev(post[0]).requires_grad_(True), to_dev(post[1]).requires_grad_(True)
    params = []
    for r, W, b in zip((r1, r2), Ws, bs):
        params += [W, b] + [dev[id(a.emb)] for a in r.atoms]
    out = UnionFn.apply(U, [gpu_layer(r) for r in (r1, r2)], "mean", "relu", Wp, bp, *params)
    out.backward(torch.from_numpy(res["dout"]).cuda())
    np.testing.assert_array_equal(out.detach().cpu().numpy(), res["out"])
    for W, want in zip(Ws, res["dW"]):
        np.testing.assert_array_equal(W.grad.cpu().numpy(), want)
    for b, want in zip(bs, res["db"]):
        np.testing.assert_array_equal(b.grad.cpu().numpy(), want)
    np.testing.assert_array_equal(Wp.grad.cpu().numpy(), res["dW_post"])
    np.testing.assert_array_equal(bp.grad.cpu().numpy(), res["db_post"])
    for k, t in dev.items():
        np.testing.assert_array_equal(t.grad.cpu().numpy(), res["demb"][k])


def test_union_backward_errors():
    import torch

    from paper_2605_24207_amd import RelnnError, Union, union_bwd, union_fwd

    r1, r2 = er_rules(seed=11, n_buys=20_000)
    U = Union([gpu_index(r1), gpu_index(r2)])                # built without the backward's CSRs
    layers = [gpu_layer(r1), gpu_layer(r2)]
    embs = [[to_dev(a.emb) for a in r.atoms] for r in (r1, r2)]
    Ws = [to_dev(r.W) for r in (r1, r2)]
    out, pre, am = union_fwd(U, layers, "sum", "none", embs, Ws)
    demb = [[torch.zeros_like(e) for e in es] for es in embs]
    dWs = [torch.zeros_like(W) for W in Ws]
    with pytest.raises(RelnnError, match="INVALID"):
        union_bwd(U, layers, "sum", "none", embs, Ws, None, None, None, pre, am, torch.zeros_like(out), demb, dWs)


def test_union_backward_shared_weights_accumulate():
    """Two bodies with one W and b: the second branch adds its weight
    gradient into the first one's buffer (RELNN_DW_ACCUM), which then holds
    the sum of both branches' shares."""
    import torch

    from paper_2605_24207_amd import Union, union_bwd, union_fwd

    r1 = relgen.node_edge(seed=60, n_nodes=2000, n_edges=20_000, d=64, h=64, bias_std=0.2)
    r2 = relgen.node_edge(seed=61, n_nodes=2000, n_edges=15_000, d=64, h=64, bias_std=0.2)
    r2.W, r2.b = r1.W, r1.b
    r2.atoms = [relgen.Atom(a.col, r1.atoms[0].emb) for a in r2.atoms]   # one relation for all atoms
    U = Union([gpu_index(r, bwd=True) for r in (r1, r2)])
    z = to_dev(r1.atoms[0].emb)
    W, b = to_dev(r1.W), to_dev(r1.b)
    layers = [gpu_layer(r1), gpu_layer(r2)]
    out, pre, am = union_fwd(U, layers, "mean", "relu", [[z, z], [z, z]], [W, W], [b, b])
    dout = torch.from_numpy(np.random.default_rng(6).standard_normal(out.shape).astype(np.float32)).cuda()
    dz = torch.zeros_like(z)
    dW = torch.full(W.shape, float("nan"), device="cuda")
    db = torch.full(b.shape, float("nan"), device="cuda")
    union_bwd(U, layers, "mean", "relu", [[z, z], [z, z]], [W, W], [b, b], None, None, pre, am, dout,
              [[dz, dz], [dz, dz]], [dW, dW], [db, db], dw_accum=[False, True])
    torch.cuda.synchronize()
    branches = [(orc.build_index(r), [r1.atoms[0].emb] * 2, r1.W, r1.b, "none") for r in (r1, r2)]
    grads, _, _ = orc.union_bwd(branches, pre.cpu().numpy(), None, dout.cpu().numpy().astype(np.float64),
                                "mean", "relu")
    ref_dW = grads[0][1] + grads[1][1]
    ref_db = grads[0][2] + grads[1][2]
    ref_dz = sum(g for de, _, _ in grads for g in de)
    assert fro(dW.cpu().numpy(), ref_dW) <= TOL["f32"]
    assert fro(db.cpu().numpy(), ref_db) <= TOL["f32"]
    assert fro(dz.cpu().numpy(), ref_dz) <= TOL["f32"]
