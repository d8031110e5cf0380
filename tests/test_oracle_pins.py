"""Pins of the FP64 oracle against things other than itself (CPU only).

Each test checks the oracle against a fact fixed by the paper's definitions
or by mathematics: a hand-worked example, a pure-Python nested-loop join,
dense closed forms, special cases that reduce to textbook operations,
permutation invariance, central finite differences and a torch-CPU FP64
composition of the paper's physical plan (Section 4.2).
"""
import json
import os

import numpy as np
import pytest

import relgen
from oracle import brute
from oracle import relnn_oracle as orc

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def tiny_rule(agg="sum", act_pre="none", act_post="relu"):
    with open(os.path.join(GOLD, "tiny_node_edge.json")) as f:
        g = json.load(f)
    z = np.array(g["node_z"], np.float32)
    rule = relgen.Rule(cols=[np.array(g["edge_s"], np.int32), np.array(g["edge_t"], np.int32)],
                       atoms=[relgen.Atom(0, z), relgen.Atom(1, z)], group_col=1,
                       W=np.array(g["W"], np.float32), b=np.array(g["b"], np.float32),
                       agg=agg, act_pre=act_pre, act_post=act_post)
    return rule, g


def run(rule, groups=None):
    idx = orc.build_index(rule)
    out, pre, am = orc.layer_fwd(idx, [a.emb for a in rule.atoms], rule.W, rule.b,
                                 rule.agg, rule.act_pre, rule.act_post, groups)
    return idx, out, pre, am


# --------------------------------------------------------------- golden
def test_golden_index():
    rule, g = tiny_rule()
    idx = orc.build_index(rule)
    assert idx.link_row.tolist() == g["canonical_link_rows"]
    assert idx.group_keys.tolist() == g["group_keys"]
    assert idx.offsets.tolist() == g["offsets"]


@pytest.mark.parametrize("agg,key", [("sum", "sum_pre"), ("mean", "mean_pre"), ("max", "max_pre")])
def test_golden_forward(agg, key):
    rule, g = tiny_rule(agg=agg, act_post="none")
    idx, out, pre, am = run(rule)
    np.testing.assert_allclose(pre, np.array(g[key]), rtol=0, atol=1e-15)
    if agg == "max":
        assert am.tolist() == g["max_argmax"]
    x = orc.gather_concat(idx, [rule.atoms[0].emb, rule.atoms[1].emb])
    y = orc.transform(x, rule.W, rule.b, "none")
    by_link = np.zeros_like(y)
    by_link[np.argsort(idx.link_row)] = y
    y_link = np.empty_like(y)
    y_link[idx.link_row] = y
    np.testing.assert_array_equal(y_link, np.array(g["per_tuple_y_by_link_row"], np.float64))


def test_golden_relu_and_grad():
    rule, g = tiny_rule(agg="sum", act_post="relu")
    idx, out, pre, am = run(rule)
    np.testing.assert_array_equal(out, np.array(g["sum_out_relu"], np.float64))
    demb, dW, db = orc.layer_bwd(idx, [a.emb for a in rule.atoms], rule.W, rule.b, pre, am,
                                 np.ones_like(out), "sum", "none", "relu")
    np.testing.assert_array_equal(dW, np.array(g["sum_relu_dW"], np.float64))
    np.testing.assert_array_equal(db, np.array(g["sum_relu_db"], np.float64))
    np.testing.assert_array_equal(demb[0] + demb[1], np.array(g["sum_relu_dz_total"], np.float64))


# --------------------------------------------------------------- brute force
def small_random_rule(seed, agg, keyed=False, chain=False, dangling=False,
                      act_pre="none", act_post="relu", n_link=40, h=3):
    rng = np.random.default_rng(seed)
    nA, nB, nC = 7, 5, 4
    dA, dB, dC = 2, 3, 2
    zA = rng.standard_normal((nA, dA)).astype(np.float32)
    zB = rng.standard_normal((nB, dB)).astype(np.float32)
    zC = rng.standard_normal((nC, dC)).astype(np.float32)
    hi = (nA + 2) if dangling else nA
    c0 = rng.integers(-1 if dangling else 0, hi, n_link).astype(np.int32)
    c1 = rng.integers(0, nB, n_link).astype(np.int32)
    keysA = keysB = None
    if keyed:
        keysA = rng.permutation(np.arange(100, 100 + 3 * nA, 3)).astype(np.int32)
        c0 = keysA[rng.integers(0, nA, n_link)].copy()
        if dangling:
            c0[::7] = 5
    atoms = [relgen.Atom(0, zA, keysA), relgen.Atom(1, zB, keysB)]
    chains = []
    if chain:
        vals = rng.integers(0, nC + (1 if dangling else 0), nB).astype(np.int32)
        chains = [relgen.Chain(src_col=1, vals=vals)]
        atoms.append(relgen.Atom(2, zC))
    K = sum(a.d for a in atoms)
    W = rng.standard_normal((K, h)).astype(np.float32)
    b = rng.standard_normal(h).astype(np.float32)
    return relgen.Rule(cols=[c0, c1], atoms=atoms, chains=chains, group_col=1, W=W, b=b,
                       agg=agg, act_pre=act_pre, act_post=act_post)


CASES = [dict(keyed=k, chain=c, dangling=d) for k in (False, True) for c in (False, True)
         for d in (False, True)]


@pytest.mark.parametrize("case", CASES)
def test_join_matches_nested_loop(case):
    rule = small_random_rule(3, "sum", **case)
    idx = orc.build_index(rule)
    bj = brute.join(rule)
    got = sorted((int(l),) + tuple(int(r[i]) for r in idx.rows) for i, l in enumerate(idx.link_row))
    exp = sorted((ell,) + rows for ell, rows, _ in bj)
    assert got == exp
    # canonical order: (head key, FK values in body order, link row) non-decreasing
    fk_cols = {ell: cols for ell, _, cols in bj}
    keys = [(fk_cols[int(l)][rule.group_col],) + tuple(fk_cols[int(l)][a.col] for a in rule.atoms) + (int(l),)
            for l in idx.link_row]
    assert keys == sorted(keys)
    assert idx.group_keys.tolist() == sorted({k[0] for k in keys})
    assert np.all(np.diff(idx.offsets) > 0)


@pytest.mark.parametrize("agg", ["sum", "mean", "max"])
@pytest.mark.parametrize("case", CASES[::3])
@pytest.mark.parametrize("acts", [("none", "relu"), ("relu", "none")])
def test_layer_matches_brute(agg, case, acts):
    rule = small_random_rule(11, agg, act_pre=acts[0], act_post=acts[1], **case)
    idx, out, pre, _ = run(rule)
    ref = brute.layer(rule)
    assert sorted(ref) == idx.group_keys.tolist()
    for q, g in enumerate(idx.group_keys.tolist()):
        np.testing.assert_allclose(pre[q], ref[g][0], rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(out[q], ref[g][1], rtol=1e-12, atol=1e-12)


def test_duplicate_key_raises():
    rule = small_random_rule(5, "sum", keyed=True)
    rule.atoms[0].keys[1] = rule.atoms[0].keys[0]
    with pytest.raises(orc.NotUnique):
        orc.build_index(rule)


# --------------------------------------------------------------- closed forms
def dense_parts(rule):
    n = rule.atoms[0].n_rows
    d = rule.atoms[0].d
    X = rule.atoms[0].emb.astype(np.float64)
    Ws = rule.W[:d].astype(np.float64)
    Wt = rule.W[d:].astype(np.float64)
    A = np.zeros((n, n))
    for s, t in zip(rule.cols[0].tolist(), rule.cols[1].tolist()):
        A[t, s] += 1.0                    # multiplicity of the edge (s, t)
    deg = A.sum(axis=1)
    return X, Ws, Wt, A, deg


def test_sum_closed_form():
    rule = relgen.node_edge(seed=7, n_nodes=60, n_edges=300, d=8, h=5, act_post="none",
                            bias_std=1.0)
    idx, out, pre, _ = run(rule)
    X, Ws, Wt, A, deg = dense_parts(rule)
    Z = A @ X @ Ws + np.diag(deg) @ X @ Wt + np.outer(deg, rule.b.astype(np.float64))
    present = np.nonzero(deg)[0]
    assert idx.group_keys.tolist() == present.tolist()
    np.testing.assert_allclose(pre, Z[present], rtol=1e-10, atol=1e-10)


def test_mean_closed_form():
    rule = relgen.node_edge(seed=8, n_nodes=60, n_edges=300, d=8, h=5, agg="mean",
                            act_post="none", bias_std=1.0)
    idx, out, pre, _ = run(rule)
    X, Ws, Wt, A, deg = dense_parts(rule)
    p = np.nonzero(deg)[0]
    Z = (A[p] / deg[p, None]) @ X @ Ws + X[p] @ Wt + rule.b.astype(np.float64)
    np.testing.assert_allclose(pre, Z, rtol=1e-10, atol=1e-10)


def test_max_properties():
    rule = relgen.node_edge(seed=9, n_nodes=50, n_edges=120, d=4, h=6, agg="max",
                            act_post="none", bias_std=1.0)
    idx, _, mx, am = run(rule)
    rule.agg = "mean"
    _, _, mean, _ = run(rule)
    assert np.all(mean <= mx + 1e-12)
    X, Ws, Wt, A, deg = dense_parts(rule)
    single = np.nonzero(np.diff(idx.offsets) == 1)[0]
    assert len(single) > 0
    for q in single:
        t = idx.group_keys[q]
        s = rule.cols[0][idx.link_row[idx.offsets[q]]]
        y = X[s] @ Ws + X[t] @ Wt + rule.b
        np.testing.assert_allclose(mx[q], y, rtol=1e-12, atol=1e-12)
        assert np.all(am[q] == idx.offsets[q])


def test_permutation_edges_reduce_to_mlp():
    rng = np.random.default_rng(4)
    n, d, h = 30, 6, 4
    pi = rng.permutation(n).astype(np.int32)
    z = rng.standard_normal((n, d)).astype(np.float32)
    W = rng.standard_normal((2 * d, h)).astype(np.float32)
    b = rng.standard_normal(h).astype(np.float32)
    rule = relgen.Rule(cols=[pi, np.arange(n, dtype=np.int32)], atoms=[relgen.Atom(0, z), relgen.Atom(1, z)],
                       group_col=1, W=W, b=b, agg="sum", act_post="relu")
    _, out, _, _ = run(rule)
    mlp = np.maximum(np.concatenate([z[pi], z], axis=1).astype(np.float64) @ W + b, 0)
    np.testing.assert_allclose(out, mlp, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("agg", ["sum", "mean", "max"])
def test_permutation_invariance(agg):
    rule = small_random_rule(21, agg, keyed=True, chain=True, n_link=60)
    _, out, pre, _ = run(rule)
    rng = np.random.default_rng(1)
    p = rng.permutation(rule.n_link)
    q = rng.permutation(rule.atoms[0].n_rows)
    rule2 = relgen.Rule(cols=[c[p] for c in rule.cols],
                        atoms=[relgen.Atom(0, rule.atoms[0].emb[q], rule.atoms[0].keys[q])] + rule.atoms[1:],
                        chains=rule.chains, group_col=rule.group_col, W=rule.W, b=rule.b, agg=agg,
                        act_post=rule.act_post)
    _, out2, pre2, _ = run(rule2)
    np.testing.assert_allclose(pre2, pre, rtol=1e-12, atol=1e-12)


def test_pandas_merge_groupby():
    pd = pytest.importorskip("pandas")
    rule = small_random_rule(31, "sum", keyed=True, chain=True, dangling=True, n_link=200)
    idx = orc.build_index(rule)
    L = pd.DataFrame({"c0": rule.cols[0], "c1": rule.cols[1], "ell": np.arange(rule.n_link)})
    A = pd.DataFrame({"c0": rule.atoms[0].keys, "rA": np.arange(rule.atoms[0].n_rows)})
    B = pd.DataFrame({"c1": np.arange(rule.atoms[1].n_rows), "rB": np.arange(rule.atoms[1].n_rows)})
    Ch = pd.DataFrame({"c1": np.arange(rule.chains[0].n_rows), "c2": rule.chains[0].vals})
    C = pd.DataFrame({"c2": np.arange(rule.atoms[2].n_rows), "rC": np.arange(rule.atoms[2].n_rows)})
    J = L.merge(Ch, on="c1").merge(A, on="c0").merge(B, on="c1").merge(C, on="c2")
    cnt = J.groupby("c1").size()
    assert cnt.index.tolist() == idx.group_keys.tolist()
    assert cnt.values.tolist() == np.diff(idx.offsets).tolist()
    assert sorted(J["ell"].tolist()) == sorted(idx.link_row.tolist())


# --------------------------------------------------------------- gradients
def total_loss(rule, embs, W, b, dout, idx):
    out, _, _ = orc.layer_fwd(idx, embs, W, b, rule.agg, rule.act_pre, rule.act_post)
    return float((out * dout).sum())


@pytest.mark.parametrize("agg", ["sum", "mean", "max"])
@pytest.mark.parametrize("act_pre", ["none", "relu"])
def test_grad_finite_differences(agg, act_pre):
    rule = small_random_rule(41, agg, chain=True, act_pre=act_pre, act_post="relu", n_link=30)
    idx = orc.build_index(rule)
    embs = [a.emb.astype(np.float64) for a in rule.atoms]
    W = rule.W.astype(np.float64)
    b = rule.b.astype(np.float64)
    out, pre, am = orc.layer_fwd(idx, embs, W, b, agg, act_pre, "relu")
    dout = np.random.default_rng(2).standard_normal(out.shape)
    demb, dW, db = orc.layer_bwd(idx, embs, W, b, pre, am, dout, agg, act_pre, "relu")
    eps = 1e-6

    def fd(arr, grad, pos):
        old = arr[pos]
        arr[pos] = old + eps
        lp = total_loss(rule, embs, W, b, dout, idx)
        out_p, pre_p, am_p = orc.layer_fwd(idx, embs, W, b, agg, act_pre, "relu")
        arr[pos] = old - eps
        lm = total_loss(rule, embs, W, b, dout, idx)
        out_m, pre_m, am_m = orc.layer_fwd(idx, embs, W, b, agg, act_pre, "relu")
        arr[pos] = old
        kinks = (np.any(np.sign(pre_p) != np.sign(pre_m)))
        if agg == "max":
            kinks = kinks or np.any(am_p != am_m)
        return (lp - lm) / (2 * eps), kinks

    rng = np.random.default_rng(3)
    checked = 0
    for arr, grad in [(embs[0], demb[0]), (embs[1], demb[1]), (embs[2], demb[2]), (W, dW), (b, db)]:
        for _ in range(8):
            pos = tuple(int(rng.integers(0, s)) for s in arr.shape)
            g_fd, kink = fd(arr, grad, pos)
            if kink:
                continue
            assert abs(g_fd - grad[pos]) <= 1e-6 * max(1.0, abs(grad[pos])), (pos, g_fd, grad[pos])
            checked += 1
    assert checked >= 20


def test_grad_closed_form_sum():
    rule = relgen.node_edge(seed=12, n_nodes=40, n_edges=200, d=5, h=3, act_post="none")
    idx, out, pre, am = run(rule)
    dout = np.random.default_rng(0).standard_normal(out.shape)
    demb, dW, db = orc.layer_bwd(idx, [rule.atoms[0].emb] * 2, rule.W, rule.b, pre, am, dout,
                                 "sum", "none", "none")
    X, Ws, Wt, A, deg = dense_parts(rule)
    dA = np.zeros((X.shape[0], dout.shape[1]))
    dA[idx.group_keys] = dout
    np.testing.assert_allclose(demb[0], A.T @ dA @ Ws.T, rtol=1e-10, atol=1e-10)
    np.testing.assert_allclose(demb[1], np.diag(deg) @ dA @ Wt.T, rtol=1e-10, atol=1e-10)
    np.testing.assert_allclose(dW, np.vstack([X.T @ A.T @ dA, X.T @ np.diag(deg) @ dA]), rtol=1e-10,
                               atol=1e-10)
    np.testing.assert_allclose(db, deg @ dA, rtol=1e-10, atol=1e-10)


@pytest.mark.parametrize("agg", ["sum", "mean", "max"])
def test_grad_torch_physical_plan(agg):
    """The paper's physical plan (Section 4.2): row indices -> index_select ->
    cat -> Linear -> scatter aggregate, differentiated by torch.autograd in
    FP64 on the CPU, must give the oracle's gradients."""
    torch = pytest.importorskip("torch")
    rule = small_random_rule(51, agg, chain=True, act_pre="relu", act_post="relu", n_link=50)
    idx = orc.build_index(rule)
    embs = [torch.tensor(a.emb, dtype=torch.float64, requires_grad=True) for a in rule.atoms]
    W = torch.tensor(rule.W, dtype=torch.float64, requires_grad=True)
    b = torch.tensor(rule.b, dtype=torch.float64, requires_grad=True)
    rows = [torch.tensor(r) for r in idx.rows]
    grp = torch.tensor(idx.tuple_group)
    x = torch.cat([torch.index_select(e, 0, r) for e, r in zip(embs, rows)], dim=1)
    y = torch.relu(x @ W + b)
    G, h = idx.G, W.shape[1]
    gi = grp[:, None].expand(-1, h)
    red = {"sum": "sum", "mean": "mean", "max": "amax"}[agg]
    agg_v = torch.zeros(G, h, dtype=torch.float64).scatter_reduce(0, gi, y, reduce=red, include_self=False)
    out = torch.relu(agg_v)
    dout = torch.tensor(np.random.default_rng(5).standard_normal((G, h)))
    (out * dout).sum().backward()
    o_out, o_pre, o_am = orc.layer_fwd(idx, [a.emb for a in rule.atoms], rule.W, rule.b, agg, "relu", "relu")
    np.testing.assert_allclose(out.detach().numpy(), o_out, rtol=1e-12, atol=1e-12)
    demb, dW, db = orc.layer_bwd(idx, [a.emb for a in rule.atoms], rule.W, rule.b, o_pre, o_am,
                                 dout.numpy(), agg, "relu", "relu")
    np.testing.assert_allclose(W.grad.numpy(), dW, rtol=1e-10, atol=1e-10)
    np.testing.assert_allclose(b.grad.numpy(), db, rtol=1e-10, atol=1e-10)
    for e, de in zip(embs, demb):
        np.testing.assert_allclose(e.grad.numpy(), de, rtol=1e-10, atol=1e-10)


# --------------------------------------------------------------- two-hop
def test_two_hop_full_cap_is_all_pairs():
    rng = np.random.default_rng(6)
    u = rng.integers(0, 6, 25).astype(np.int32)
    i = rng.integers(0, 4, 25).astype(np.int32)
    la, lb = orc.two_hop_paths([u, i], 1, cap=10_000)
    got = sorted(zip(la.tolist(), lb.tolist()))
    exp = sorted((a, c) for a in range(25) for c in range(25) if i[a] == i[c])
    assert got == exp


def test_two_hop_cap_order():
    u = np.array([5, 3, 9, 3, 7, 1], np.int32)
    i = np.array([2, 2, 2, 2, 8, 8], np.int32)
    la, lb = orc.two_hop_paths([u, i], 1, cap=5)
    # item 2: rows ordered by (user, row) = [1, 3, 0, 2]; item 8: [5, 4]
    assert list(zip(la.tolist(), lb.tolist())) == [
        (1, 3), (3, 0), (0, 2), (2, 1), (1, 0),       # successors, then shift 2
        (5, 4), (4, 5), (5, 5), (4, 4)]               # all 4 pairs of a 2-row group


def test_bf16_round():
    x = np.array([1.0, 1.00390625, 1.005859375, 1.0078125 + 2 ** -8, -2.5, 3.0e-3], np.float32)
    r = orc.bf16_round(x)
    # 1 + 2^-8 is a tie between 1 and 1 + 2^-7: to even -> 1; 1.005859375 = 1 + 3*2^-9 -> 1 + 2^-7
    assert r[0] == 1.0 and r[1] == 1.0 and r[2] == np.float32(1.0078125)
    assert r[3] == np.float32(1.015625) and r[4] == -2.5
    assert abs(r[5] - 3.0e-3) <= 3.0e-3 * 2 ** -8


def test_bwd_given_act_pre_mask_equals_computed():
    """Passing the act_pre' decisions computed from the same inputs changes
    nothing; flipping one decision changes only the gradients it feeds."""
    rule = relgen.node_edge(seed=3, n_nodes=40, n_edges=120, d=8, h=8, agg="sum", act_pre="relu",
                            act_post="none", bias_std=0.3)
    idx = orc.build_index(rule)
    embs = [a.emb for a in rule.atoms]
    _, pre, am = orc.layer_fwd(idx, embs, rule.W, rule.b, "sum", "relu", "none")
    dout = np.random.default_rng(0).standard_normal(pre.shape)
    base = orc.layer_bwd(idx, embs, rule.W, rule.b, pre, am, dout, "sum", "relu", "none")
    mask = orc.act_pre_mask(idx, embs, rule.W, rule.b)
    given = orc.layer_bwd(idx, embs, rule.W, rule.b, pre, am, dout, "sum", "relu", "none", pre_mask=mask)
    for a, b in zip(base[0] + [base[1], base[2]], given[0] + [given[1], given[2]]):
        np.testing.assert_array_equal(a, b)
    flipped = mask.copy()
    flipped[0, 0] = not flipped[0, 0]
    _, dW, db = orc.layer_bwd(idx, embs, rule.W, rule.b, pre, am, dout, "sum", "relu", "none", pre_mask=flipped)
    sign = 1.0 if flipped[0, 0] else -1.0
    np.testing.assert_allclose(db - base[2], sign * np.eye(8)[0] * dout[idx.tuple_group[0], 0], atol=1e-12)
    x0 = orc.gather_concat(idx, embs, [0])[0]
    np.testing.assert_allclose(dW - base[1], sign * np.outer(x0, np.eye(8)[0]) * dout[idx.tuple_group[0], 0],
                               atol=1e-12)


def _fd_check(loss, params, grads, coords, eps, decisions):
    """Central differences of ``loss`` at the listed coordinates; a
    coordinate whose +-eps probes change an integer decision (a ReLU sign or
    a MAX maximiser) is skipped.  Returns the number checked."""
    checked = 0
    for pi, pos in coords:
        arr = params[pi]
        old = arr[pos]
        arr[pos] = old + eps
        lp, dp = loss(), decisions()
        arr[pos] = old - eps
        lm, dm = loss(), decisions()
        arr[pos] = old
        if any(not np.array_equal(a, b) for a, b in zip(dp, dm)):
            continue
        g_fd = (lp - lm) / (2 * eps)
        g = grads[pi][pos]
        assert abs(g_fd - g) <= 1e-6 * max(1.0, abs(g)), (pi, pos, g_fd, g)
        checked += 1
    return checked


@pytest.mark.parametrize("layer", [0, 1])
def test_grad_finite_differences_power_law_instance(layer):
    """The differentiation workload's gradient instance: 2k nodes, 10k edges,
    s ~ Zipf(1.2), t uniform, width 128; layer 1 (SUM, ReLU after the
    aggregate) and layer 2 (MAX).  Central differences in FP64 of
    sum(out * dout) at sampled coordinates of z (the hottest source row
    among them), W and b against the analytic gradient."""
    p = relgen.power_graph(seed=5, n_nodes=2000, n_edges=10_000, d=128, h=128, bias_std=0.2)
    rule = relgen.power_rule(p, layer)
    idx = orc.build_index(rule)
    z = rule.atoms[0].emb.astype(np.float64)
    W = rule.W.astype(np.float64)
    b = rule.b.astype(np.float64)
    agg, post = rule.agg, rule.act_post
    out, pre, am = orc.layer_fwd(idx, [z, z], W, b, agg, "none", post)
    dout = np.random.default_rng(8).standard_normal(out.shape)
    demb, dW, db = orc.layer_bwd(idx, [z, z], W, b, pre, am, dout, agg, "none", post)
    dz = demb[0] + demb[1]                      # both atoms read Node

    def loss():
        o, _, _ = orc.layer_fwd(idx, [z, z], W, b, agg, "none", post)
        return float((o * dout).sum())

    def decisions():
        _, pr, a = orc.layer_fwd(idx, [z, z], W, b, agg, "none", post)
        return (np.sign(pr),) if agg != "max" else (np.sign(pr), a)

    rng = np.random.default_rng(9)
    deg = np.bincount(p.s, minlength=2000)
    hot = int(np.argmax(deg))
    coords = [(0, (hot, int(c))) for c in rng.integers(0, 128, 4)]
    coords += [(0, (int(rng.integers(0, 2000)), int(rng.integers(0, 128)))) for _ in range(6)]
    coords += [(1, (int(rng.integers(0, 256)), int(rng.integers(0, 128)))) for _ in range(8)]
    coords += [(2, (int(rng.integers(0, 128)),)) for _ in range(4)]
    n = _fd_check(loss, [z, W, b], [dz, dW, db], coords, 1e-6, decisions)
    assert deg[hot] > 100 and n >= 16, (deg[hot], n)


def test_grad_finite_differences_power_law_two_layer_mse():
    """The two-layer net of the differentiation workload on its gradient
    instance, MSE against N(0, 1) targets: central differences of the loss
    through both layers (the chain the autograd wrapper drives) against the
    chained analytic gradients."""
    p = relgen.power_graph(seed=6, n_nodes=2000, n_edges=10_000, d=128, h=128, bias_std=0.2)
    z = p.z.astype(np.float64)
    W1, W2 = p.W[0].astype(np.float64), p.W[1].astype(np.float64)
    b1, b2 = p.b[0].astype(np.float64), p.b[1].astype(np.float64)
    r1 = relgen.power_rule(p, 0)
    i1 = orc.build_index(r1)
    o1 = orc.layer_fwd(i1, [z, z], W1, b1, "sum", "none", "relu")[0]
    r2 = relgen.power_rule(p, 1, z=o1, z_keys=i1.group_keys.astype(np.int32))
    i2 = orc.build_index(r2)
    tg = p.target[i2.group_keys].astype(np.float64)

    def forward():
        o1, pre1, am1 = orc.layer_fwd(i1, [z, z], W1, b1, "sum", "none", "relu")
        o2, pre2, am2 = orc.layer_fwd(i2, [o1, o1], W2, b2, "max", "none", "none")
        return o1, pre1, am1, o2, pre2, am2

    def loss():
        o2 = forward()[3]
        return float(((o2 - tg) ** 2).mean())

    def decisions():
        _, pre1, _, _, pre2, am2 = forward()
        return np.sign(pre1), am2

    o1, pre1, am1, o2, pre2, am2 = forward()
    dout2 = 2.0 * (o2 - tg) / o2.size
    d2, dW2, db2 = orc.layer_bwd(i2, [o1, o1], W2, b2, pre2, am2, dout2, "max", "none", "none")
    d1, dW1, db1 = orc.layer_bwd(i1, [z, z], W1, b1, pre1, am1, d2[0] + d2[1], "sum", "none", "relu")
    rng = np.random.default_rng(10)
    coords = [(0, (int(rng.integers(0, 2000)), int(rng.integers(0, 128)))) for _ in range(6)]
    coords += [(1, (int(rng.integers(0, 256)), int(rng.integers(0, 128)))) for _ in range(4)]
    coords += [(2, (int(rng.integers(0, 256)), int(rng.integers(0, 128)))) for _ in range(4)]
    coords += [(3, (int(rng.integers(0, 128)),)), (4, (int(rng.integers(0, 128)),))]
    n = _fd_check(loss, [z, W1, W2, b1, b2], [d1[0] + d1[1], dW1, dW2, db1, db2], coords, 1e-6, decisions)
    assert n >= 12, n
