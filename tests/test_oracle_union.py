"""Pins of the oracle's k-ary projected union and union rules (CPU only).

The projected union (Section 2.2) unifies the head keys of k relations and
aggregates, once, the multiset of every tuple with a key, whichever
relation it comes from; MEAN is not decomposable and must not be a mean of
the relations' means.  A union rule (Section 3.1) applies its transform
after the union.  Checked against a pure-Python nested loop, against
k = 1 (the projection of a join rule), a relation united with itself, a
hand-counted MEAN across two relations and the closed form of the
transform after the union.
"""
import numpy as np
import pytest

import relgen
from oracle import brute
from oracle import relnn_oracle as orc


def branch_rule(seed, n_link, n_keys=6, agg="sum", act_pre="none", h=3):
    rng = np.random.default_rng(seed)
    nA, dA, dB = 7, 2, 3
    zA = rng.standard_normal((nA, dA)).astype(np.float32)
    zB = rng.standard_normal((n_keys, dB)).astype(np.float32)
    c0 = rng.integers(0, nA, n_link).astype(np.int32)
    c1 = rng.integers(0, n_keys, n_link).astype(np.int32)
    W = rng.standard_normal((dA + dB, h)).astype(np.float32)
    b = rng.standard_normal(h).astype(np.float32)
    return relgen.Rule(cols=[c0, c1], atoms=[relgen.Atom(0, zA), relgen.Atom(1, zB)], group_col=1, W=W, b=b,
                       agg=agg, act_pre=act_pre)


def branch(rule):
    return (orc.build_index(rule), [a.emb for a in rule.atoms], rule.W, rule.b, rule.act_pre)


@pytest.mark.parametrize("agg", ["sum", "mean", "max"])
@pytest.mark.parametrize("k", [2, 3])
def test_union_matches_nested_loop(agg, k):
    rules = [branch_rule(10 + i, n_link=8 + 5 * i, n_keys=5 + i, act_pre="relu" if i == 1 else "none")
             for i in range(k)]
    rng = np.random.default_rng(1)
    Wp, bp = rng.standard_normal((3, 4)), rng.standard_normal(4)
    bs = [branch(r) for r in rules]
    keys, out, pre, arg = orc.union_fwd(bs, agg, "relu", Wp, bp)
    ref = brute.union_layer(rules, agg, "relu", Wp, bp)
    assert keys.tolist() == sorted(ref)
    for q, key in enumerate(keys.tolist()):
        np.testing.assert_allclose(pre[q], ref[key][0], rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(out[q], ref[key][1], rtol=1e-12, atol=1e-12)
    if agg == "max":                 # the maximiser named by (branch, position) holds the maximum
        for q in range(len(keys)):
            for c in range(pre.shape[1]):
                bi, p = arg[q, c]
                idx, embs, W, b, act = bs[bi]
                assert idx.gkey[p] == keys[q]
                y = orc.transform(orc.gather_concat(idx, embs, [p]), W, b, act)[0, c]
                assert y == pre[q, c]


@pytest.mark.parametrize("agg", ["sum", "mean", "max"])
def test_union_of_one_is_the_projection(agg):
    rule = branch_rule(3, n_link=30, agg=agg)
    idx = orc.build_index(rule)
    o_out, o_pre, o_am = orc.layer_fwd(idx, [a.emb for a in rule.atoms], rule.W, rule.b, agg, "none", "relu")
    keys, out, pre, arg = orc.union_fwd([branch(rule)], agg, "relu")
    assert keys.tolist() == idx.group_keys.tolist()
    np.testing.assert_allclose(pre, o_pre, rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(out, o_out, rtol=1e-13, atol=1e-13)
    if agg == "max":
        assert (arg[..., 0] == 0).all() and (arg[..., 1] == o_am).all()


def test_self_union():
    """R united with itself: every multiset doubles, so SUM doubles and MEAN
    and MAX stay; MAX's maximiser is in the first copy."""
    rule = branch_rule(4, n_link=25)
    b = branch(rule)
    _, _, s1, _ = orc.union_fwd([b], "sum")
    _, _, s2, _ = orc.union_fwd([b, b], "sum")
    np.testing.assert_allclose(s2, 2 * s1, rtol=1e-13)
    _, _, m1, _ = orc.union_fwd([b], "mean")
    _, _, m2, _ = orc.union_fwd([b, b], "mean")
    np.testing.assert_allclose(m2, m1, rtol=1e-13)
    _, _, x2, a2 = orc.union_fwd([b, b], "max")
    _, _, x1, _ = orc.union_fwd([b], "max")
    np.testing.assert_allclose(x2, x1, rtol=0)
    assert (a2[..., 0] == 0).all()


def test_mean_is_applied_once_across_relations():
    """Key 0 has one tuple (y = 1) in R1 and three (y = 2, 3, 4) in R2, with
    W = identity on a one-column embedding: the union's MEAN is 10 / 4 =
    2.5, not the mean of the means (1 + 3) / 2 = 2."""
    def rel(values):
        z = np.array([[v] for v in values], np.float32)
        return relgen.Rule(cols=[np.arange(len(values), dtype=np.int32), np.zeros(len(values), np.int32)],
                           atoms=[relgen.Atom(0, z)], group_col=1, W=np.ones((1, 1), np.float32),
                           b=np.zeros(1, np.float32))
    keys, out, pre, _ = orc.union_fwd([branch(rel([1.0])), branch(rel([2.0, 3.0, 4.0]))], "mean")
    assert keys.tolist() == [0] and pre[0, 0] == 2.5
    keys, out, pre, _ = orc.union_fwd([branch(rel([1.0])), branch(rel([2.0, 3.0, 4.0]))], "sum")
    assert pre[0, 0] == 10.0


def test_keys_are_the_union_of_the_branches():
    r1 = branch_rule(5, n_link=6, n_keys=4)
    r2 = branch_rule(6, n_link=6, n_keys=12)
    r2.cols[1] = r2.cols[1] % 9 + 3              # keys 3..11 (all present in its atom), overlapping 3
    keys, _, _, _ = orc.union_fwd([branch(r1), branch(r2)], "sum")
    expect = sorted(set(r1.cols[1].tolist()) | set(r2.cols[1].tolist()))
    assert keys.tolist() == expect


def test_union_rule_transform_after_the_union():
    """tau after the union: out = act(agg W_post + b_post), once per key."""
    rules = [branch_rule(7, 12), branch_rule(8, 15)]
    rng = np.random.default_rng(2)
    Wp, bp = rng.standard_normal((3, 2)), rng.standard_normal(2)
    keys, out, pre, _ = orc.union_fwd([branch(r) for r in rules], "mean", "none", Wp, bp)
    np.testing.assert_allclose(out, pre @ Wp + bp, rtol=1e-13)


# ---------------------------------------------------------------------------
# backward
# ---------------------------------------------------------------------------
def _union_loss(rules, arrays, agg, act_post, Wp, bp, dout):
    """sum(out * dout) of the union of ``rules`` whose parameters are taken
    from ``arrays`` = [zA_0, zB_0, W_0, b_0, zA_1, ...]."""
    bs = []
    for i, r in enumerate(rules):
        zA, zB, W, b = arrays[4 * i: 4 * i + 4]
        bs.append((orc.build_index(r), [zA, zB], W, b, r.act_pre))
    _, out, _, _ = orc.union_fwd(bs, agg, act_post, Wp, bp)
    return float((out * dout).sum())


@pytest.mark.parametrize("agg", ["sum", "mean", "max"])
@pytest.mark.parametrize("post", [False, True])
def test_union_backward_finite_differences(agg, post):
    """Every gradient of the union (both branches' embeddings, W and b, and
    the union rule's W_post and b_post) against FP64 central differences of
    sum(out * dout), with ReLU inside the second branch and after the
    union."""
    rules = [branch_rule(20, n_link=14, n_keys=5), branch_rule(21, n_link=11, n_keys=7, act_pre="relu")]
    rng = np.random.default_rng(3)
    arrays = []
    for r in rules:
        arrays += [r.atoms[0].emb.astype(np.float64), r.atoms[1].emb.astype(np.float64),
                   r.W.astype(np.float64), r.b.astype(np.float64)]
    Wp = rng.standard_normal((3, 4)) if post else None
    bp = rng.standard_normal(4) if post else None
    bs = [(orc.build_index(r), arrays[4 * i: 4 * i + 2], arrays[4 * i + 2], arrays[4 * i + 3], r.act_pre)
          for i, r in enumerate(rules)]
    keys, out, pre, arg = orc.union_fwd(bs, agg, "relu", Wp, bp)
    dout = rng.standard_normal(out.shape)
    grads, dWp, dbp = orc.union_bwd(bs, pre, arg, dout, agg, "relu", Wp, bp)
    flat = []
    for demb, dW, db in grads:
        flat += [demb[0], demb[1], dW, db]
    params = arrays + ([Wp, bp] if post else [])
    flat += [dWp, dbp] if post else []
    for a_i, (arr, gr) in enumerate(zip(params, flat)):
        fd = np.zeros_like(arr)
        for pos in np.ndindex(*arr.shape):
            def f(delta):
                ps = [p.copy() for p in params]
                ps[a_i][pos] += delta
                return _union_loss(rules, ps[:8], agg, "relu", ps[8] if post else None, ps[9] if post else None,
                                   dout)
            fd[pos] = (f(1e-6) - f(-1e-6)) / 2e-6
        np.testing.assert_allclose(gr, fd, rtol=1e-5, atol=1e-6, err_msg=f"parameter {a_i}")


@pytest.mark.parametrize("agg", ["sum", "mean", "max"])
def test_union_backward_of_one_is_the_layer_backward(agg):
    """k = 1: the union is the projection of one join rule, so its backward
    is that layer's."""
    rule = branch_rule(3, n_link=30, agg=agg, act_pre="relu")
    idx = orc.build_index(rule)
    embs = [a.emb for a in rule.atoms]
    o_out, o_pre, o_am = orc.layer_fwd(idx, embs, rule.W, rule.b, agg, "relu", "relu")
    keys, out, pre, arg = orc.union_fwd([branch(rule)], agg, "relu")
    dout = np.random.default_rng(4).standard_normal(out.shape)
    grads, dWp, dbp = orc.union_bwd([branch(rule)], pre, arg, dout, agg, "relu")
    demb, dW, db = orc.layer_bwd(idx, embs, rule.W, rule.b, o_pre, o_am, dout, agg, "relu", "relu")
    assert dWp is None and dbp is None
    np.testing.assert_allclose(grads[0][1], dW, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(grads[0][2], db, rtol=1e-12, atol=1e-12)
    for a, b in zip(grads[0][0], demb):
        np.testing.assert_allclose(a, b, rtol=1e-12, atol=1e-12)


def test_self_union_backward():
    """R united with itself: each copy's tuples get the single rule's
    gradient (SUM), half of it (MEAN: every multiset doubles), or all of it
    in the first copy and none in the second (MAX: the first maximiser)."""
    rule = branch_rule(4, n_link=25, act_pre="relu")
    b = branch(rule)
    rng = np.random.default_rng(5)
    for agg, parts in (("sum", (1.0, 1.0)), ("mean", (0.5, 0.5)), ("max", (1.0, 0.0))):
        _, out1, pre1, arg1 = orc.union_fwd([b], agg, "relu")
        _, out2, pre2, arg2 = orc.union_fwd([b, b], agg, "relu")
        dout = rng.standard_normal(out1.shape)
        g1, _, _ = orc.union_bwd([b], pre1, arg1, dout, agg, "relu")
        g2, _, _ = orc.union_bwd([b, b], pre2, arg2, dout, agg, "relu")
        for copy, f in enumerate(parts):
            np.testing.assert_allclose(g2[copy][1], f * g1[0][1], rtol=1e-12, atol=1e-12)
            np.testing.assert_allclose(g2[copy][2], f * g1[0][2], rtol=1e-12, atol=1e-12)
            for a, c in zip(g2[copy][0], g1[0][0]):
                np.testing.assert_allclose(a, f * c, rtol=1e-12, atol=1e-12)


def test_union_backward_mean_counts_every_relation():
    """The hand-counted MEAN across two relations (one tuple with y = 1 in
    R1, three in R2; W = identity on one column): out = 10 / 4, so every
    one of the four embeddings has gradient dout / 4 and W gets
    dout * (1 + 2 + 3 + 4) / 4 split by branch (1 / 4 and 9 / 4)."""
    def rel(values):
        z = np.array([[v] for v in values], np.float32)
        return relgen.Rule(cols=[np.arange(len(values), dtype=np.int32), np.zeros(len(values), np.int32)],
                           atoms=[relgen.Atom(0, z)], group_col=1, W=np.ones((1, 1), np.float32),
                           b=np.zeros(1, np.float32))
    bs = [branch(rel([1.0])), branch(rel([2.0, 3.0, 4.0]))]
    keys, out, pre, arg = orc.union_fwd(bs, "mean")
    grads, _, _ = orc.union_bwd(bs, pre, arg, np.array([[2.0]]), "mean")
    np.testing.assert_allclose(grads[0][0][0], [[0.5]], rtol=0)
    np.testing.assert_allclose(grads[1][0][0], [[0.5], [0.5], [0.5]], rtol=0)
    np.testing.assert_allclose(grads[0][1], [[0.5]], rtol=0)
    np.testing.assert_allclose(grads[1][1], [[4.5]], rtol=0)
    np.testing.assert_allclose(grads[0][2] + grads[1][2], [2.0], rtol=0)
