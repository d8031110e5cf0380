"""Pins of the oracle's selection and general joins (CPU only).

The filter expression of a rule (Section 3.1: a conjunction of predicates
e1 theta e2 over content variables and constants) and joins of further link
relations (Section 2.2: natural joins on shared variables, many-to-many and
cyclic, as in the DHN triangle rule of Section 5.2) are checked against a
pure-Python nested loop over all row combinations, and against dense closed
forms: a triangle match anchored at n is a closed walk n -> v -> w -> n, so
with a constant transform the SUM over them is the diagonal of A^3 (A the
multiplicity matrix of Edge), and with a Linear one each term is a product of
A, A^2 and the embeddings.
"""
import copy

import numpy as np
import pytest

import relgen
from oracle import brute
from oracle import relnn_oracle as orc


def run(rule):
    idx = orc.build_index(rule)
    out, pre, am = orc.layer_fwd(idx, [a.emb for a in rule.atoms], rule.W, rule.b, rule.agg, rule.act_pre,
                                 rule.act_post)
    return idx, out, pre, am


def canonical_from_brute(rule):
    """(head key, atom rows, link row) of every joined tuple of the nested
    loop, sorted by (head key, FK values of the atoms, source rows): the
    canonical order.  The link row of a tuple is the position of its source
    rows (link row, row of each further relation) in the lexicographic order
    of all joined link tuples."""
    pos = {src: p for p, (src, _) in enumerate(brute._link_tuples(rule))}
    items = []
    for src, rows, cols in brute.join(rule):
        src = src if isinstance(src, tuple) else (src,)
        items.append(((cols[rule.group_col],) + tuple(cols[a.col] for a in rule.atoms) + src,
                      (cols[rule.group_col],) + rows + (pos[src],)))
    return [v for _, v in sorted(items)]


def oracle_tuples(idx):
    return [(int(idx.gkey[i]),) + tuple(int(r[i]) for r in idx.rows) + (int(idx.link_row[i]),)
            for i in range(idx.E)]


def tiny_edge_rule(seed, n=9, m=30, d=3, h=2, agg="sum"):
    rng = np.random.default_rng(seed)
    s = rng.integers(0, n, m).astype(np.int32)
    t = rng.integers(0, n, m).astype(np.int32)
    z = rng.standard_normal((n, d)).astype(np.float32)
    W = rng.standard_normal((2 * d, h)).astype(np.float32)
    b = rng.standard_normal(h).astype(np.float32)
    return relgen.Rule(cols=[s, t], atoms=[relgen.Atom(0, z), relgen.Atom(1, z)], group_col=1, W=W, b=b, agg=agg,
                       act_post="none")


PRED_CASES = [
    [relgen.Pred(a=0, op="lt", b=1)],                                          # s < t
    [relgen.Pred(a=0, op="ne", b=1)],                                          # no self-loops
    [relgen.Pred(a=0, op="ge", b=1, mul_a=2, mul_b=-1, add=-3)],               # 2 s - t - 3 >= 0
    [relgen.Pred(a=1, op="eq", add=-4)],                                       # t = 4
    [relgen.Pred(a=0, op="le", add=-5), relgen.Pred(a=1, op="gt", add=-2)],   # s <= 5 and t > 2
]


@pytest.mark.parametrize("case", range(len(PRED_CASES)))
@pytest.mark.parametrize("agg", ["sum", "mean", "max"])
def test_selection_matches_nested_loop(case, agg):
    rule = tiny_edge_rule(3 + case, agg=agg)
    rule.preds = PRED_CASES[case]
    idx, out, pre, _ = run(rule)
    got = oracle_tuples(idx)
    assert got == canonical_from_brute(rule)
    ref = brute.layer(rule)
    assert sorted(ref) == idx.group_keys.tolist()
    for q, g in enumerate(idx.group_keys.tolist()):
        np.testing.assert_allclose(pre[q], ref[g][0], rtol=1e-12, atol=1e-12)


def test_selection_closed_form():
    """SUM with the filter s < t is the SUM closed form on the filtered
    multiplicity matrix A[t, s] [s < t]."""
    rule = relgen.node_edge(seed=12, n_nodes=50, n_edges=400, d=6, h=4, act_post="none", bias_std=1.0)
    rule.preds = [relgen.Pred(a=0, op="lt", b=1)]
    idx, out, pre, _ = run(rule)
    d = rule.atoms[0].d
    X = rule.atoms[0].emb.astype(np.float64)
    A = np.zeros((50, 50))
    for s, t in zip(rule.cols[0].tolist(), rule.cols[1].tolist()):
        if s < t:
            A[t, s] += 1.0
    deg = A.sum(axis=1)
    Z = A @ X @ rule.W[:d].astype(np.float64) + np.diag(deg) @ X @ rule.W[d:].astype(np.float64) + \
        np.outer(deg, rule.b.astype(np.float64))
    p = np.nonzero(deg)[0]
    assert idx.group_keys.tolist() == p.tolist()
    np.testing.assert_allclose(pre, Z[p], rtol=1e-10, atol=1e-10)


def many_to_many_rule(seed, agg="sum"):
    """Co-purchase without a cap: Buys(u, i) joined with Buys(u2, i) on the
    item (many-to-many), grouped by u; atoms User(u) and User(u2)."""
    rng = np.random.default_rng(seed)
    nu, ni, m, d, h = 8, 5, 25, 3, 2
    bu = rng.integers(0, nu, m).astype(np.int32)
    bi = rng.integers(0, ni, m).astype(np.int32)
    z = rng.standard_normal((nu, d)).astype(np.float32)
    W = rng.standard_normal((2 * d, h)).astype(np.float32)
    b = rng.standard_normal(h).astype(np.float32)
    step = relgen.Step(cols=[bu.copy(), bi.copy()], on=[1], key=[1])
    return relgen.Rule(cols=[bu, bi], atoms=[relgen.Atom(0, z), relgen.Atom(2, z)], group_col=0, W=W, b=b,
                       agg=agg, act_post="none", steps=[step])


@pytest.mark.parametrize("agg", ["sum", "max"])
def test_many_to_many_join_matches_nested_loop(agg):
    rule = many_to_many_rule(4, agg)
    idx, out, pre, _ = run(rule)
    got = oracle_tuples(idx)
    assert got == canonical_from_brute(rule)
    # bag semantics: the number of pairs per item is (buyers of the item)^2
    cnt = np.bincount(rule.cols[1], minlength=5)
    assert idx.E == int((cnt ** 2).sum())
    ref = brute.layer(rule)
    for q, g in enumerate(idx.group_keys.tolist()):
        np.testing.assert_allclose(pre[q], ref[g][0], rtol=1e-12, atol=1e-12)


def test_triangle_join_matches_nested_loop():
    rule = relgen.triangle_rule(seed=3, n_graphs=2, n_nodes=7, avg_degree=4, d=2, h=2)
    rule.preds = [relgen.Pred(a=2, op="lt", b=5)]          # v < w as well
    idx, out, pre, _ = run(rule)
    got = oracle_tuples(idx)
    assert idx.E > 0 and got == canonical_from_brute(rule)
    ref = brute.layer(rule)
    for q, g in enumerate(idx.group_keys.tolist()):
        np.testing.assert_allclose(pre[q], ref[g][0], rtol=1e-12, atol=1e-12)


def adjacency(rule, n):
    A = np.zeros((n, n))
    for s, t in zip(rule.cols[1].tolist(), rule.cols[2].tolist()):
        A[s, t] += 1.0
    return A


def test_triangle_count_is_diagonal_of_A_cubed():
    """With tau = 1 (W = 0, b = 1) the SUM over triangle matches anchored at
    n counts the closed walks n -> v -> w -> n: (A^3)[n, n]."""
    rule = relgen.triangle_rule(seed=5, n_graphs=30, n_nodes=12, avg_degree=5, d=4, h=1, act_post="none")
    rule.W = np.zeros_like(rule.W)
    rule.b = np.ones(1, np.float32)
    idx, out, pre, _ = run(rule)
    n = rule.atoms[0].n_rows
    A = adjacency(rule, n)
    c = np.diag(A @ A @ A)
    p = np.nonzero(c)[0]
    assert idx.group_keys.tolist() == p.tolist()
    np.testing.assert_allclose(pre[:, 0], c[p], rtol=0, atol=1e-9)


def test_triangle_linear_closed_form():
    """SUM over triangles of Lin(h_n (+) h_v (+) h_w) = c_n h_n W1 +
    ((A o (A^2)^T) H W2)[n] + ((A^2 o A^T) H W3)[n] + c_n b, c = diag(A^3)."""
    rule = relgen.triangle_rule(seed=6, n_graphs=25, n_nodes=12, avg_degree=5, d=5, h=3, act_post="none",
                                bias_std=1.0)
    idx, out, pre, _ = run(rule)
    n, d = rule.atoms[0].n_rows, rule.atoms[0].d
    A = adjacency(rule, n)
    A2 = A @ A
    c = np.diag(A2 @ A)
    H = rule.atoms[0].emb.astype(np.float64)
    W = rule.W.astype(np.float64)
    Z = (c[:, None] * H) @ W[:d] + (A * A2.T) @ H @ W[d:2 * d] + (A2 * A.T) @ H @ W[2 * d:] + \
        np.outer(c, rule.b.astype(np.float64))
    p = np.nonzero(c)[0]
    assert idx.group_keys.tolist() == p.tolist()
    np.testing.assert_allclose(pre, Z[p], rtol=1e-10, atol=1e-10)


def test_step_with_no_match_and_filter_rejecting_all():
    rule = many_to_many_rule(5)
    rule.steps[0].cols[1] = rule.steps[0].cols[1] + 100        # no item matches
    assert orc.build_index(rule).E == 0
    rule = tiny_edge_rule(6)
    rule.preds = [relgen.Pred(a=0, op="lt", add=0)]            # s < 0: nothing passes
    idx = orc.build_index(rule)
    assert idx.E == 0 and idx.G == 0


def test_filter_applies_to_derived_columns():
    """A predicate on an FK-chain column (Buys.item -> BelongsTo.cat)."""
    rng = np.random.default_rng(9)
    n_item, m = 6, 40
    bu = rng.integers(0, 5, m).astype(np.int32)
    bi = rng.integers(0, n_item, m).astype(np.int32)
    cat = rng.integers(0, 3, n_item).astype(np.int32)
    zu = rng.standard_normal((5, 2)).astype(np.float32)
    zc = rng.standard_normal((3, 2)).astype(np.float32)
    rule = relgen.Rule(cols=[bu, bi], atoms=[relgen.Atom(0, zu), relgen.Atom(2, zc)], group_col=1,
                       W=rng.standard_normal((4, 2)).astype(np.float32), b=np.zeros(2, np.float32),
                       chains=[relgen.Chain(src_col=1, vals=cat)], preds=[relgen.Pred(a=2, op="ne", add=-1)])
    idx, out, pre, _ = run(rule)
    got = oracle_tuples(idx)
    assert got == canonical_from_brute(rule)
    assert all(int(r) != 1 for r in idx.rows[1])
    plain = copy.copy(rule)
    plain.preds = []
    assert orc.build_index(plain).E > idx.E
