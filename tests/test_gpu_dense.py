"""GPU checks of the dense output layout (relnn_out_dense, through the C
ABI): rows addressed by the head key with a presence byte.  The set of keys
that occur is checked bit for bit against the oracle's, each present row
against the compact output it copies (bit for bit) and against the oracle
(FP32 bound), absent rows are zero; the union's keys; no key; a key
outside the dense range is refused."""
import numpy as np
import pytest

import relgen
from oracle import relnn_oracle as orc
from tests.helpers import distinct_embs, gpu_index, gpu_layer, oracle_fwd, rel_rows, to_dev

pytestmark = pytest.mark.gpu


def layer_out(rule):
    import torch

    from paper_2605_24207_amd import layer_fwd

    gi = gpu_index(rule)
    out, pre, _ = layer_fwd(gi, gpu_layer(rule), distinct_embs(rule), to_dev(rule.W), to_dev(rule.b))
    torch.cuda.synchronize()
    return gi, out


@pytest.mark.parametrize("agg", ["sum", "max"])
def test_dense_layer_output(agg):
    """3000 nodes, 2000 edges: most targets have no tuple."""
    from paper_2605_24207_amd import out_dense

    rule = relgen.node_edge(seed=50, n_nodes=3000, n_edges=2000, d=32, h=32, agg=agg, bias_std=0.3)
    gi, out = layer_out(rule)
    keys = gi.export()["group_keys"]
    dense, present = out_dense(keys, out, 3000)
    dense, present = dense.cpu().numpy(), present.cpu().numpy()
    idx, o_out, _, _ = oracle_fwd(rule)
    np.testing.assert_array_equal(np.nonzero(present)[0], idx.group_keys)
    assert set(np.unique(present).tolist()) <= {0, 1}
    np.testing.assert_array_equal(dense[idx.group_keys], out.cpu().numpy())
    assert rel_rows(dense[idx.group_keys], o_out, scale_ref=np.maximum(np.abs(o_out), 1e-3)).max() <= 1e-5
    absent = np.setdiff1d(np.arange(3000), idx.group_keys)
    assert len(absent) > 1000 and not np.any(dense[absent])


def test_dense_union_output():
    import torch

    from paper_2605_24207_amd import Union, out_dense, union_fwd

    r1 = relgen.node_edge(seed=51, n_nodes=2000, n_edges=1500, d=32, h=32, bias_std=0.3)
    r2 = relgen.node_edge(seed=52, n_nodes=2000, n_edges=1500, d=32, h=32, bias_std=0.3)
    U = Union([gpu_index(r1), gpu_index(r2)])
    out, _, _ = union_fwd(U, [gpu_layer(r1), gpu_layer(r2)], "mean", "relu", [distinct_embs(r1), distinct_embs(r2)],
                          [to_dev(r1.W), to_dev(r2.W)], [to_dev(r1.b), to_dev(r2.b)])
    keys = U.export()["keys"]
    dense, present = out_dense(keys, out, 2000)
    torch.cuda.synchronize()
    k = keys.cpu().numpy()
    expect = np.union1d(orc.build_index(r1).group_keys, orc.build_index(r2).group_keys)
    np.testing.assert_array_equal(k, expect)
    np.testing.assert_array_equal(np.nonzero(present.cpu().numpy())[0], expect)
    np.testing.assert_array_equal(dense.cpu().numpy()[k], out.cpu().numpy())


def test_dense_without_keys_and_without_presence():
    import torch

    from paper_2605_24207_amd import out_dense

    dense, present = out_dense(torch.zeros(0, dtype=torch.int32, device="cuda"),
                               torch.zeros(0, 16, device="cuda"), 100)
    assert not dense.cpu().numpy().any() and not present.cpu().numpy().any()
    rule = relgen.node_edge(seed=53, n_nodes=500, n_edges=800, d=32, h=32)
    gi, out = layer_out(rule)
    dense, present = out_dense(gi.export()["group_keys"], out, 500, want_present=False)
    assert present is None and dense.shape == (500, 32)


def test_dense_key_out_of_range_is_refused():
    from paper_2605_24207_amd import RelnnError, out_dense

    rule = relgen.node_edge(seed=54, n_nodes=500, n_edges=3000, d=32, h=32)
    gi, out = layer_out(rule)
    keys = gi.export()["group_keys"]
    n = int(keys[-1].item())                      # the largest key needs n + 1 rows
    with pytest.raises(RelnnError, match="RANGE"):
        out_dense(keys, out, n)
