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


def _loss(rule, embs, agg, act_pre, dout):
    idx = orc.build_index(rule)
    out, _, _ = orc.layer_fwd(idx, embs, None, None, agg, act_pre, "relu", tf="product")
    return float((out * dout).sum())


@pytest.mark.parametrize("agg", ["sum", "mean", "max"])
@pytest.mark.parametrize("act_pre", ["none", "relu"])
def test_product_backward_finite_differences(agg, act_pre):
    """The product transform's gradients against FP64 central differences of
    sum(out * dout), for two atoms on distinct relations and for a self-join
    (one relation read by both atoms: the entries add)."""
    rng = np.random.default_rng(5)
    rule = prod_rule(4, agg, act_pre, n=9, m=40, d=3)
    Zs = rng.standard_normal((9, 3))
    Zt = rng.standard_normal((9, 3))
    idx = orc.build_index(rule)
    dout = rng.standard_normal((idx.G, 3))
    for embs, shared in (([Zs, Zt], False), ([Zs, Zs], True)):
        out, pre, am = orc.layer_fwd(idx, embs, None, None, agg, act_pre, "relu", tf="product")
        demb = orc.product_bwd(idx, embs, pre, am, dout, agg, act_pre, "relu")
        grads = [demb[0] + demb[1]] if shared else demb
        arrays = [Zs] if shared else [Zs, Zt]
        for a_i, (arr, gr) in enumerate(zip(arrays, grads)):
            fd = np.zeros_like(arr)
            for r in range(arr.shape[0]):
                for c in range(arr.shape[1]):
                    def f(delta):
                        x = arr.copy()
                        x[r, c] += delta
                        e = [x, x] if shared else ([x, embs[1]] if a_i == 0 else [embs[0], x])
                        return _loss(rule, e, agg, act_pre, dout)
                    fd[r, c] = (f(1e-6) - f(-1e-6)) / 2e-6
            np.testing.assert_allclose(gr, fd, rtol=1e-5, atol=1e-6)


def test_product_backward_closed_form():
    """SUM over an edge relation with distinct relations Zs, Zt and no
    activations: out[t] = (A Zs)[t] * Zt[t], so dZs = A^T (dout * Zt) and
    dZt = dout * (A Zs) on the targets that occur."""
    rng = np.random.default_rng(6)
    rule = relgen.node_edge(seed=7, n_nodes=30, n_edges=200, d=4, h=4, agg="sum", act_post="none")
    Zs = rng.standard_normal((30, 4))
    Zt = rng.standard_normal((30, 4))
    idx = orc.build_index(rule)
    dout = rng.standard_normal((idx.G, 4))
    out, pre, am = orc.layer_fwd(idx, [Zs, Zt], None, None, "sum", "none", "none", tf="product")
    dzs, dzt = orc.product_bwd(idx, [Zs, Zt], pre, am, dout, "sum", "none", "none")
    A = np.zeros((30, 30))
    for s, t in zip(rule.cols[0].tolist(), rule.cols[1].tolist()):
        A[t, s] += 1.0
    D = np.zeros((30, 4))
    D[idx.group_keys] = dout
    np.testing.assert_allclose(dzs, A.T @ (D * Zt), rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(dzt, D * (A @ Zs), rtol=1e-12, atol=1e-12)
