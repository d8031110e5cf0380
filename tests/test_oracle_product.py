"""Pins of the oracle's product transform (CPU only): tau = z_1 * ... * z_k
elementwise (Section 1's q*k and a*v, Section 5.4's gated mean z_e*z_w).
Checked against the nested-loop brute force and against the closed form
of SUM over an edge relation: sum_s A[t, s] z_s * z_t = (A Z)[t] * Z[t],
and MEAN divided by the in-degree."""
import numpy as np
import pytest

import relgen
from oracle import brute
from oracle import relnn_oracle as orc


def prod_rule(seed, agg, act_pre="none", n=40, m=200, d=6):
    rule = relgen.node_edge(seed=seed, n_nodes=n, n_edges=m, d=d, h=d, agg=agg, act_pre=act_pre, act_post="relu")
    return rule


@pytest.mark.parametrize("agg", ["sum", "mean", "max"])
@pytest.mark.parametrize("act_pre", ["none", "relu"])
def test_product_matches_nested_loop(agg, act_pre):
    rule = prod_rule(2, agg, act_pre, n=9, m=30, d=3)
    idx = orc.build_index(rule)
    out, pre, am = orc.layer_fwd(idx, [a.emb for a in rule.atoms], None, None, agg, act_pre, "relu", tf="product")
    ref = brute.layer(rule, tf="product")
    assert sorted(ref) == idx.group_keys.tolist()
    for q, g in enumerate(idx.group_keys.tolist()):
        np.testing.assert_allclose(pre[q], ref[g][0], rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(out[q], ref[g][1], rtol=1e-12, atol=1e-12)


def test_product_closed_forms():
    rule = prod_rule(3, "sum", n=50, m=400)
    idx = orc.build_index(rule)
    Z = rule.atoms[0].emb.astype(np.float64)
    A = np.zeros((50, 50))
    for s, t in zip(rule.cols[0].tolist(), rule.cols[1].tolist()):
        A[t, s] += 1.0
    deg = A.sum(axis=1)
    p = np.nonzero(deg)[0]
    _, pre, _ = orc.layer_fwd(idx, [Z, Z], None, None, "sum", tf="product")
    np.testing.assert_allclose(pre, ((A @ Z) * Z)[p], rtol=1e-12, atol=1e-12)
    _, pre, _ = orc.layer_fwd(idx, [Z, Z], None, None, "mean", tf="product")
    np.testing.assert_allclose(pre, ((A @ Z) * Z / deg[:, None])[p], rtol=1e-12, atol=1e-12)
