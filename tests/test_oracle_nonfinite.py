"""Non-finite values in the oracle's SUM and MEAN (CPU).

Section 2.2 defines the aggregate of a group over that group's tuples only,
so an infinite or NaN embedding value may reach only the groups whose tuples
read it.  The oracle is checked against the nested-loop brute force (plain
Python float arithmetic, IEEE-754) on an instance with +Inf, -Inf and NaN
planted in three embedding rows: the same non-finite entries, the finite
ones within 1e-12, and every group that reads none of the planted rows
finite.
"""
import numpy as np
import pytest

import relgen
from oracle import brute
from oracle import relnn_oracle as orc

BAD = {5: (2, np.inf), 9: (1, -np.inf), 17: (0, np.nan)}


def planted_rule(agg, seed=21):
    rule = relgen.node_edge(seed=seed, n_nodes=50, n_edges=400, d=6, h=4, agg=agg, act_post="none",
                            bias_std=0.5)
    z = rule.atoms[0].emb.copy()
    for r, (c, v) in BAD.items():
        z[r, c] = v
    for a in rule.atoms:
        a.emb = z
    return rule


def same_nonfinite(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return (np.array_equal(np.isnan(a), np.isnan(b)) and np.array_equal(np.isposinf(a), np.isposinf(b))
            and np.array_equal(np.isneginf(a), np.isneginf(b)))


@pytest.mark.parametrize("agg", ["sum", "mean"])
def test_nonfinite_matches_nested_loop_and_stays_in_its_groups(agg):
    rule = planted_rule(agg)
    idx = orc.build_index(rule)
    with np.errstate(invalid="ignore", over="ignore"):
        _, pre, _ = orc.layer_fwd(idx, [a.emb for a in rule.atoms], rule.W, rule.b, agg, "none", "none")
    ref = brute.layer(rule)
    assert sorted(ref) == idx.group_keys.tolist()
    exp = np.array([ref[g][0] for g in idx.group_keys.tolist()])
    assert same_nonfinite(pre, exp)
    fin = np.isfinite(exp)
    np.testing.assert_allclose(pre[fin], exp[fin], rtol=1e-12, atol=1e-12)
    # confinement: a group is non-finite only if one of its tuples reads a planted row
    bad_rows = np.array(sorted(BAD))
    touched = np.zeros(idx.G, bool)
    for q in range(idx.G):
        s, e = idx.offsets[q], idx.offsets[q + 1]
        touched[q] = any(np.isin(idx.rows[j][s:e], bad_rows).any() for j in range(len(rule.atoms)))
    assert touched.any() and not touched.all()
    assert np.isfinite(pre[~touched]).all()
    assert not np.isfinite(pre[touched]).all(axis=1).any()     # every touched group has a non-finite entry
    # each kind occurs
    assert np.isnan(pre).any() and np.isposinf(pre).any() and np.isneginf(pre).any()
