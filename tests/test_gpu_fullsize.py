"""Parity at the full workload sizes, in the launch configuration bench.py
times (one launch over all joined tuples of a rule), checked on seeded
samples of the output that the oracle evaluates group by group or row by
row.  Sampled groups include one large group whose tiles span several
persistent blocks, so the carry fix-up is part of what is checked.

Workload 2: the ER schema (User 1M, Item 500k, Category 1k, Buys 20M with
item ~ Zipf 1.1), Item SUM (K = 384) and User MEAN (K = 256), FP32 and BF16.
Workload 3: the two-hop co-buy rule on the same graph, BF16, h = 256, MAX.
Workload 4: Node 2M x 128, Edge 10M (s ~ Zipf 1.2), the MAX layer forward
and the backward of both layers (SUM + ReLU and MAX), FP32 and BF16:
embedding-gradient rows of sampled nodes (the hottest source, about 1.9M
tuples, among them), db against its closed form, the dW rows of the atom
keyed by the group column in full and sampled dW columns of the other one.
Workload 5: the server at the benchmark's settings on the full ER graph.
"""
import copy

import numpy as np
import pytest

import relgen
from oracle import relnn_oracle as orc
from tests.helpers import distinct_embs, gpu_index, gpu_layer, oracle_inputs, rel_rows, to_dev

pytestmark = pytest.mark.gpu

TOL = {"f32": 1e-5, "bf16": 2e-2}


@pytest.fixture(scope="module")
def er():
    return relgen.er_graph()


@pytest.fixture(scope="module")
def power():
    return relgen.power_graph()


def sample_keys(keys, n_rand, big, seed):
    """n_rand random group keys that occur, plus the key whose group size is
    closest to ``big``."""
    cnt = np.bincount(keys)
    nz = np.nonzero(cnt)[0]
    rng = np.random.default_rng(seed)
    hot = nz[np.argmin(np.abs(cnt[nz] - big))]
    return np.unique(np.concatenate([rng.choice(nz, n_rand, replace=False), [hot]])), int(cnt[hot])


def restrict(rule, keys):
    """The same rule over the link rows of the sampled groups only."""
    sub = copy.copy(rule)
    sel = np.isin(rule.cols[rule.group_col], keys)
    sub.cols = [c[sel] for c in rule.cols]
    return sub


def gpu_full_fwd(rule, dtype, index, pushdown=False):
    import torch

    from paper_2605_24207_amd import layer_fwd

    out, pre, am = layer_fwd(index, gpu_layer(rule, dtype, pushdown=pushdown), distinct_embs(rule, dtype),
                             to_dev(rule.W, dtype), to_dev(rule.b))
    torch.cuda.synchronize()
    return out, pre, am


def check_sampled_forward(rule, dtype, keys, pushdown=False):
    import torch

    gi = gpu_index(rule)
    out, pre, am = gpu_full_fwd(rule, dtype, gi, pushdown)
    ex = gi.export()
    gk = ex["group_keys"].cpu().numpy()
    goff = ex["offsets"].cpu().numpy()
    sub = restrict(rule, keys)
    ref = orc.build_index(sub)
    np.testing.assert_array_equal(ref.group_keys, np.sort(keys))
    pos = np.searchsorted(gk, ref.group_keys)
    np.testing.assert_array_equal(gk[pos], ref.group_keys)
    # index: group sizes and the joined rows of every sampled group, bit-exact
    np.testing.assert_array_equal(goff[pos + 1] - goff[pos], np.diff(ref.offsets))
    rows = ex["tuple_rows"].cpu().numpy()
    for q, g in enumerate(pos):
        s, e = goff[g], goff[g + 1]
        for j in range(len(rule.atoms)):
            np.testing.assert_array_equal(rows[j][s:e], ref.rows[j][ref.offsets[q]:ref.offsets[q + 1]])
    # layer values
    idx_t = torch.from_numpy(pos.astype(np.int64)).to(pre.device)
    pre_g = pre.index_select(0, idx_t).float().cpu().numpy()
    out_g = out.index_select(0, idx_t).float().cpu().numpy()
    embs, W, b = oracle_inputs(rule, "f32")
    o_out, o_pre, o_am = orc.layer_fwd(ref, embs, W, b, rule.agg, rule.act_pre, rule.act_post)
    assert rel_rows(pre_g, o_pre).max() <= TOL[dtype]
    assert rel_rows(out_g, o_out, scale_ref=o_pre).max() <= TOL[dtype]
    am_ref, embs_k, W_k = o_am, embs, W
    if dtype == "bf16":          # the kernel's arithmetic alone, on the rounded inputs
        embs_k, W_k, _ = oracle_inputs(rule, "bf16")
        _, b_pre, b_am = orc.layer_fwd(ref, embs_k, W_k, b, rule.agg, rule.act_pre, rule.act_post)
        assert rel_rows(pre_g, b_pre).max() <= 1e-5 * np.sqrt(rule.K)
        am_ref = b_am
    if rule.agg == "max":        # maximiser position within its group
        am_g = am.index_select(0, idx_t).cpu().numpy().astype(np.int64) - goff[pos][:, None]
        am_r = am_ref - ref.offsets[:-1][:, None]
        diff = np.nonzero(am_g != am_r)
        for q, c in zip(*diff):
            x = orc.gather_concat(ref, embs_k, [ref.offsets[q] + am_g[q, c]])
            y = orc.transform(x, W_k, b, rule.act_pre)[0, c]
            assert abs(y - o_pre[q, c]) <= 4 * TOL[dtype] * max(1.0, abs(o_pre[q, c]))
        assert len(diff[0]) <= 0.01 * am_r.size + 1
    return gi, (out, pre, am)


@pytest.mark.parametrize("mode", ["fused", "pushdown"])
@pytest.mark.parametrize("dtype", ["f32", "bf16"])
@pytest.mark.parametrize("which", ["item", "user"])
def test_er_full_forward_sampled(er, which, dtype, mode):
    """300 sampled groups and one of about 60k tuples, with the transform
    evaluated per tuple (fused) or pushed below the join (node products)."""
    rule = relgen.er_item_rule(er) if which == "item" else relgen.er_user_rule(er)
    keys, hot = sample_keys(rule.cols[rule.group_col], 300, 60_000, seed=17)
    if which == "item":          # one group over many tiles and more than one block's range
        assert hot > 20_000
    check_sampled_forward(rule, dtype, keys, pushdown=mode == "pushdown")


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_er_full_forward_hottest_group(er, dtype):
    """The hottest Item group (about 2.5M of the 20M tuples, spread over
    many persistent blocks): its SUM crosses tens of thousands of tiles
    (Kahan-compensated inside a block) and dozens of block ranges (the carry
    fix-up).  Checked with a few random groups against the FP64 oracle."""
    rule = relgen.er_item_rule(er)
    gk = rule.cols[rule.group_col]
    cnt = np.bincount(gk)
    hot = int(np.argmax(cnt))
    assert cnt[hot] > 2_000_000
    rng = np.random.default_rng(31)
    keys = np.unique(np.concatenate([rng.choice(np.nonzero(cnt)[0], 20, replace=False), [hot]]))
    check_sampled_forward(rule, dtype, keys)


def test_power_full_max_forward_sampled(power):
    rule = relgen.power_rule(power, 1)
    keys, _ = sample_keys(rule.cols[rule.group_col], 300, 0, seed=19)
    check_sampled_forward(rule, "f32", keys)


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
@pytest.mark.parametrize("layer", [0, 1])
def test_power_full_backward(power, layer, dtype):
    """Workload-4 backward at full size (E = 10M), layer 1 (SUM, ReLU after
    the aggregate) or layer 2 (MAX), FP32 or BF16.  Checked against FP64
    sums over the FP32 master values, with the integer decisions (ReLU
    signs, maximisers) taken from the kernel's forward: the embedding-
    gradient rows of sampled nodes (the hottest source, about 1.9M tuples,
    and one of about 30k among them), db (closed form: sum_g w_g dA_g, w_g =
    |g| for SUM, 1 for MAX), the dW rows of the atom keyed by the group
    column in full and sampled dW columns of the other atom."""
    import torch

    from paper_2605_24207_amd import layer_bwd, layer_fwd

    tol = TOL[dtype]
    rule = relgen.power_rule(power, layer)
    gi = gpu_index(rule, bwd=True)
    lay = gpu_layer(rule, dtype)
    z = to_dev(rule.atoms[0].emb, dtype)
    W, b = to_dev(rule.W, dtype), to_dev(rule.b)
    out, pre, am = layer_fwd(gi, lay, [z, z], W, b)
    dout_np = np.random.default_rng(3).standard_normal((gi.G, rule.h)).astype(np.float32)
    dz = torch.zeros(z.shape, dtype=torch.float32, device="cuda")
    dW = torch.empty(W.shape, dtype=torch.float32, device="cuda")
    db = torch.empty_like(b)
    layer_bwd(gi, lay, [z, z], W, b, pre, am, to_dev(dout_np), [dz, dz], dW, db)
    torch.cuda.synchronize()

    ref = orc.build_index(rule)                   # full canonical order: positions match the kernel's
    ex = gi.export()
    np.testing.assert_array_equal(ex["offsets"].cpu().numpy(), ref.offsets)
    np.testing.assert_array_equal(ex["link_rows"].cpu().numpy(), ref.link_row)
    is_max = rule.agg == "max"
    am_np = am.cpu().numpy().astype(np.int64) if is_max else None
    dA = dout_np.astype(np.float64)
    if rule.act_post == "relu":
        dA = dA * (pre.cpu().numpy() > 0)         # the kernel's ReLU decisions
    cnt = np.diff(ref.offsets).astype(np.float64)
    wg = np.ones_like(cnt) if is_max else cnt
    rel = lambda a, r: np.linalg.norm(a - r) / max(np.linalg.norm(r), 1e-30)
    # db: every dA[g][c] reaches one tuple (MAX) or all |g| tuples (SUM)
    db_ref = (wg[:, None] * dA).sum(axis=0)
    assert rel(db.cpu().numpy(), db_ref) <= tol
    # dz rows of sampled nodes: the hottest source and one of about 30k
    deg = np.bincount(np.concatenate(rule.cols), minlength=rule.atoms[0].n_rows)
    nz = np.nonzero(deg)[0]
    rng = np.random.default_rng(23)
    hot = int(np.argmax(np.bincount(rule.cols[0])))
    mid = nz[np.argmin(np.abs(deg[nz] - 30_000))]
    nodes = np.unique(np.concatenate([rng.choice(nz, 150, replace=False), [hot, mid]]))
    assert deg[hot] > 1_000_000
    W64 = rule.W.astype(np.float64)
    d = rule.atoms[0].d
    dz_ref = np.zeros((len(nodes), d))
    sq = np.zeros(len(nodes))                    # sum of squared norms of the terms (error scale)
    for j in range(2):
        rows_j = ref.rows[j]
        tup = np.nonzero(np.isin(rows_j, nodes))[0]        # canonical positions joined to a sampled node
        g = ref.tuple_group[tup]
        dy = np.where(am_np[g] == tup[:, None], dA[g], 0.0) if is_max else dA[g]
        contrib = dy @ W64[j * d:(j + 1) * d].T
        at = np.searchsorted(nodes, rows_j[tup])
        np.add.at(dz_ref, at, contrib)
        np.add.at(sq, at, (contrib ** 2).sum(axis=1))
        del dy, contrib
    dz_g = dz.cpu().numpy()[nodes].astype(np.float64)
    scale = np.maximum(np.linalg.norm(dz_ref, axis=1), np.sqrt(sq))
    err = np.linalg.norm(dz_g - dz_ref, axis=1) / np.maximum(scale, 1e-30)
    assert err.max() <= tol, err.max()
    # dW rows of atom t (keyed by the group column: every tuple of g joins
    # the same row; the gradients of g add up to w_g dA_g) in full
    dW_np = dW.cpu().numpy().astype(np.float64)
    z64 = rule.atoms[0].emb.astype(np.float64)
    x_t = z64[ref.rows[1][ref.offsets[:-1]]]
    ref_t = x_t.T @ (wg[:, None] * dA)
    del x_t
    assert rel(dW_np[d:], ref_t) <= tol
    # rows of atom s on sampled output columns
    for c in np.random.default_rng(29).choice(rule.h, 3, replace=False):
        if is_max:                                # column c of g goes to the tuple the kernel chose
            col = z64[ref.rows[0][am_np[:, c]]].T @ dA[:, c]
        else:                                     # sum over tuples of z_s(tau) dA[g(tau), c]
            w = np.bincount(ref.rows[0], weights=dA[ref.tuple_group, c], minlength=z64.shape[0])
            col = z64.T @ w
        assert rel(dW_np[:d, c], col) <= tol


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_power_full_pushdown_forward_sampled(power, dtype):
    """Workload-4 layer 1 with the transform pushed below the join, at full
    size, on sampled groups."""
    rule = relgen.power_rule(power, 0)
    keys, _ = sample_keys(rule.cols[rule.group_col], 300, 0, seed=37)
    check_sampled_forward(rule, dtype, keys, pushdown=True)


def test_serve_full_graph_bench_settings(er):
    """Serving at the benchmark's settings on the full ER graph (Buys 20M):
    max_seeds 4096, max_slots 64, a 64 GiB budget; six requests submitted
    together, one of them 4096 seeds, FP32 and BF16, each against the FP64
    serving oracle on the FP32 master values (1e-5 and 2e-2 per row)."""
    from oracle import serve_oracle as so
    from tests.test_gpu_serve import make_server, rows_close

    adj = so.adjacency(er.buys_u, er.buys_i, er.item.shape[0], er.user.shape[0])
    rng = np.random.default_rng(41)
    reqs = [(rng.choice(er.item.shape[0], size=n, replace=False).astype(np.int32), int(rng.integers(0, 2**62)))
            for n in (4096, 1, 300, 2000, 17, 4096)]
    emb = (er.user, er.item, er.cat, er.belongs_cat)
    Wr = (er.W_user[0], er.W_item[0], er.W_item[1])
    refs = [so.evaluate(adj, emb, Wr, (None, None, None), s, rs, 15, 10) for s, rs in reqs]
    for dtype, tol in (("f32", 1e-5), ("bf16", 2e-2)):
        srv = make_server(er, dtype, max_seeds=4096, max_slots=64, budget_bytes=64 << 30)
        tickets = [srv.submit(s, rs) for s, rs in reqs]
        for (s, rs), t, (r_out, r_pres, r_tuples) in zip(reqs, tickets, refs):
            out, present, st = srv.wait(t, len(s))
            assert present.tolist() == r_pres.tolist()
            assert st["tuples"] == r_tuples
            assert rows_close(out, r_out, tol)
        srv.close()


def test_cobuy_full_precision_form(er):
    """Workload 3 at full size: Buys |x| Buys^T on item (at most 50 paths per
    item, about 9.8M paths), BF16 MFMA with FP32 accumulation, h = 256, MAX.
    The index is compared in full; the values on a 1% sample of the output
    rows, against the FP64 oracle."""
    import torch

    rule = relgen.cobuy_rule(er, d=256, h=256, cap=50, agg="max")
    gi = gpu_index(rule)
    ref = orc.build_index(rule)
    assert (gi.E, gi.G) == (ref.E, ref.G)
    ex = {k: v.cpu().numpy() for k, v in gi.export().items()}
    np.testing.assert_array_equal(ex["offsets"], ref.offsets)
    np.testing.assert_array_equal(ex["link_rows"], ref.link_row)
    for j in range(2):
        np.testing.assert_array_equal(ex["tuple_rows"][j], ref.rows[j])
    out, pre, am = gpu_full_fwd(rule, "bf16", gi)
    rng = np.random.default_rng(29)
    groups = np.sort(rng.choice(ref.G, ref.G // 100, replace=False))
    sel = torch.from_numpy(groups.astype(np.int64)).to(pre.device)
    pre_g = pre.index_select(0, sel).cpu().numpy()
    embs, W, b = oracle_inputs(rule, "f32")
    _, o_pre, _ = orc.layer_fwd(ref, embs, W, b, "max", groups=groups)
    assert rel_rows(pre_g, o_pre).max() <= TOL["bf16"]
    embs_k, W_k, _ = oracle_inputs(rule, "bf16")
    _, b_pre, b_am = orc.layer_fwd(ref, embs_k, W_k, b, "max", groups=groups)
    assert rel_rows(pre_g, b_pre).max() <= 1e-5 * np.sqrt(rule.K)
    am_g = am.index_select(0, sel).cpu().numpy().astype(np.int64)
    diff = np.nonzero(am_g != b_am)
    for q, c in zip(*diff):
        y = orc.transform(orc.gather_concat(ref, embs_k, [am_g[q, c]]), W_k, b, "none")[0, c]
        assert abs(y - b_pre[q, c]) <= 1e-5 * np.sqrt(rule.K) * max(1.0, abs(b_pre[q, c]))
    assert len(diff[0]) <= 0.01 * b_am.size + 1
