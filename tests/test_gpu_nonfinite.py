"""Non-finite values stay in their own group (GPU, SUM and MEAN).

The fused kernels sum the runs of a tile on the matrix cores, multiplying
every tuple value of the tile by 0 or 1; an infinite or NaN value must not
leak into the other groups of its tile.  +Inf, -Inf and NaN are planted in
three embedding rows (a hot node among them, so long groups and tiles cut
by unit boundaries are covered); the GPU's pre-activation aggregate must
have exactly the oracle's non-finite entries (NaN, +Inf and -Inf in the
same places) and match it within 1e-5 (FP32) / 2e-2 (BF16) on every finite
row, for the fused kernel (narrow and wide tiles), the plain pipeline and
the pushdown.
"""
import numpy as np
import pytest

import relgen
from oracle import relnn_oracle as orc
from tests.helpers import gpu_fwd, rel_rows

pytestmark = pytest.mark.gpu

TOL = {"f32": 1e-5, "bf16": 2e-2}


def plant(rule, rows):
    """Plant +Inf, -Inf, NaN at (row, column) in the rule's embedding
    relations (atoms sharing one array keep sharing it)."""
    seen = {}
    for a in rule.atoms:
        if id(a.emb) not in seen:
            z = a.emb.copy()
            for (r, c), v in zip(rows, (np.inf, -np.inf, np.nan)):
                if r < len(z):
                    z[r, c % z.shape[1]] = v
            seen[id(a.emb)] = z
        a.emb = seen[id(a.emb)]
    return rule


def node_rule(agg):
    rule = relgen.node_edge(seed=41, n_nodes=4000, n_edges=80_000, d=64, h=64, agg=agg, act_post="none",
                            bias_std=0.3, src_zipf=1.2)
    return plant(rule, [(0, 3), (77, 10), (1234, 20)])             # node 0 is the hottest source


def er_rule(agg):
    g = relgen.er_graph(seed=8, n_user=6000, n_item=3000, n_cat=40, n_buys=80_000, n_layers=1)
    rule = relgen.er_item_rule(g)
    rule.agg, rule.act_post = agg, "none"
    return plant(rule, [(0, 5), (11, 50), (23, 100)])


def check(rule, dtype, **kw):
    res = gpu_fwd(rule, dtype, **kw)
    with np.errstate(invalid="ignore", over="ignore"):
        _, _, o_pre, _ = orc_fwd(rule, dtype)
    got = res["pre"].astype(np.float64)
    assert np.array_equal(np.isnan(got), np.isnan(o_pre))
    assert np.array_equal(np.isposinf(got), np.isposinf(o_pre))
    assert np.array_equal(np.isneginf(got), np.isneginf(o_pre))
    bad = ~np.isfinite(o_pre).all(axis=1)
    assert 0 < bad.sum() < 0.2 * len(bad)
    assert rel_rows(got[~bad], o_pre[~bad]).max() <= TOL[dtype]


def orc_fwd(rule, dtype):
    idx = orc.build_index(rule)
    r = (lambda a: orc.bf16_round(a)) if dtype == "bf16" else (lambda a: a)
    embs = [r(a.emb) for a in rule.atoms]
    out, pre, am = orc.layer_fwd(idx, embs, r(rule.W), rule.b, rule.agg, rule.act_pre, rule.act_post)
    return idx, out, pre, am


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
@pytest.mark.parametrize("agg", ["sum", "mean"])
def test_fused_nonfinite_confined(agg, dtype):
    check(node_rule(agg), dtype)
    check(er_rule(agg), dtype)


@pytest.mark.parametrize("mode", ["plain", "pushdown"])
def test_unfused_nonfinite_confined(mode):
    for dtype in ("f32", "bf16"):
        check(node_rule("sum"), dtype, **{mode: True})
