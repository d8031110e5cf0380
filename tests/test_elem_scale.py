"""The element-wise condition scale of the GPU tests (CPU): rounding the
inputs to bf16 moves every output element of the FP64 oracle by at most
2^-8 of its scale, for SUM, MEAN and MAX, with and without ReLU; and the
scale is exact for a one-term case."""
import numpy as np
import pytest

import relgen
from oracle import relnn_oracle as orc
from tests.helpers import elem_err, elem_scale, oracle_fwd


@pytest.mark.parametrize("agg", ["sum", "mean", "max"])
@pytest.mark.parametrize("act_pre", ["none", "relu"])
def test_bf16_rounding_within_scale(agg, act_pre):
    rule = relgen.node_edge(seed=7, n_nodes=300, n_edges=3000, d=16, h=8, agg=agg, act_pre=act_pre, bias_std=0.5)
    idx, _, pre, _ = oracle_fwd(rule, "f32")
    _, _, pre_b, _ = oracle_fwd(rule, "bf16", idx=idx)
    e = elem_err(pre_b, pre, elem_scale(rule, idx, "f32"))
    assert 1e-4 < e <= 2.0 ** -8


def test_scale_of_single_term():
    """One tuple per group, one nonzero input and weight: the scale is |x w|."""
    rule = relgen.node_edge(seed=8, n_nodes=20, n_edges=20, d=2, h=1, agg="sum")
    rule.cols = [np.arange(20, dtype=np.int32), np.arange(20, dtype=np.int32)]
    z = np.zeros((20, 2), np.float32)
    z[:, 0] = np.arange(20) - 10
    for a in rule.atoms:
        a.emb = z
    rule.W = np.array([[3.0], [0.0], [-2.0], [0.0]], np.float32)
    idx = orc.build_index(rule)
    sc = elem_scale(rule, idx)
    np.testing.assert_allclose(sc[:, 0], 5.0 * np.abs(np.arange(20) - 10))
