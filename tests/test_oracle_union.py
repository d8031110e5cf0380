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
