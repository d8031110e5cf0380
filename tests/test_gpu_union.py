"""GPU parity of the k-ary projected union and union rules (through the C
ABI): the union's keys and member counts bit for bit, its aggregate and
output against the FP64 oracle within 1e-5 (FP32) and 2e-2 (BF16 branch
transforms).  Cases: MEAN across two relations with overlapping and
disjoint keys (MEAN applied once over the whole multiset), SUM and MAX, a
relation united with itself, three branches with different body shapes,
the union rule's transform after the union, and k = 1 against the layer.
"""
import numpy as np
import pytest

import relgen
from oracle import relnn_oracle as orc
from tests.helpers import distinct_embs, gpu_index, gpu_layer, oracle_inputs, rel_rows, to_dev

pytestmark = pytest.mark.gpu

TOL = {"f32": 1e-5, "bf16": 2e-2}


def er_rules(seed=3, n_user=6000, n_item=3000, n_buys=80_000):
    """Two bodies of one head Item(i): Buys(u, i) with User, Item, Category
    (K = 384), and Views(u, i) with User, Item (K = 256) on other rows."""
    g = relgen.er_graph(seed=seed, n_user=n_user, n_item=n_item, n_cat=40, n_buys=n_buys, n_layers=1)
    r1 = relgen.er_item_rule(g)
    r2 = relgen.er_user_rule(g)
    r2.group_col = 1                               # grouped by item: a second body of Item(i)
    half = n_buys // 2
    r1.cols = [c[:half].copy() for c in r1.cols]
    r2.cols = [c[half:].copy() for c in r2.cols]
    r2.cols[1] = (r2.cols[1] % (n_item // 2)).astype(np.int32)  # the second body reaches half the items
    return r1, r2


def run_union(rules, agg, dtype, act_post="relu", post=None):
    from paper_2605_24207_amd import Union, union_fwd

    idx = [gpu_index(r) for r in rules]
    U = Union(idx)
    layers = [gpu_layer(r, dtype) for r in rules]
    embs = [distinct_embs(r, dtype) for r in rules]
    Ws = [to_dev(r.W, dtype) for r in rules]
    bs = [to_dev(r.b) for r in rules]
    W_post = b_post = None
    if post is not None:
        W_post, b_post = to_dev(post[0]), to_dev(post[1])
    out, pre, am = union_fwd(U, layers, agg, act_post, embs, Ws, bs, W_post, b_post)
    ex = U.export()
    return U, ex["keys"].cpu().numpy(), ex["counts"].cpu().numpy(), out.cpu().numpy(), pre.cpu().numpy()


def oracle_union(rules, agg, act_post="relu", post=None, dtype="f32"):
    branches = []
    for r in rules:
        embs, W, b = oracle_inputs(r, dtype)
        branches.append((orc.build_index(r), embs, W, b, r.act_pre))
    Wp, bp = (None, None) if post is None else post
    keys, out, pre, _ = orc.union_fwd(branches, agg, act_post, Wp, bp)
    cnt = np.zeros(len(keys), np.int64)
    for br in branches:
        idx = br[0]
        pos = np.searchsorted(keys, idx.group_keys)
        cnt[pos] += np.diff(idx.offsets)
    return keys, cnt, out, pre


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
@pytest.mark.parametrize("agg", ["mean", "sum", "max"])
def test_union_of_two_bodies(agg, dtype):
    rules = er_rules()
    U, keys, cnt, out, pre = run_union(rules, agg, dtype)
    r_keys, r_cnt, r_out, r_pre = oracle_union(rules, agg)
    np.testing.assert_array_equal(keys, r_keys)
    np.testing.assert_array_equal(cnt, r_cnt)
    assert rel_rows(pre, r_pre).max() <= TOL[dtype]
    assert rel_rows(out, r_out, scale_ref=r_pre).max() <= TOL[dtype]
    if dtype == "bf16":                           # the kernels' arithmetic on the rounded inputs
        _, _, _, b_pre = oracle_union(rules, agg, dtype="bf16")
        assert rel_rows(pre, b_pre).max() <= 1e-5 * np.sqrt(384)


def test_mean_across_relations_is_not_a_mean_of_means():
    """Keys reached by both bodies with different member counts: the union's
    MEAN must differ from the mean of the two bodies' means, and equal the
    oracle's single MEAN."""
    rules = er_rules(seed=4)
    U, keys, cnt, out, pre = run_union(rules, "mean", "f32", act_post="none")
    _, _, _, r_pre = oracle_union(rules, "mean", act_post="none")
    assert rel_rows(pre, r_pre).max() <= 1e-5
    i1, i2 = orc.build_index(rules[0]), orc.build_index(rules[1])
    both = np.intersect1d(i1.group_keys, i2.group_keys)
    assert len(both) > 100
    _, _, p1, _ = orc.union_fwd([(i1, *oracle_inputs(rules[0], "f32"), "none")], "mean")
    _, _, p2, _ = orc.union_fwd([(i2, *oracle_inputs(rules[1], "f32"), "none")], "mean")
    mm = 0.5 * (p1[np.searchsorted(i1.group_keys, both)] + p2[np.searchsorted(i2.group_keys, both)])
    got = pre[np.searchsorted(keys, both)]
    assert np.median(rel_rows(got, mm)) > 1e-2


def test_self_union_and_k1():
    from paper_2605_24207_amd import layer_fwd

    rule = relgen.node_edge(seed=15, n_nodes=2000, n_edges=30_000, d=64, h=64, agg="sum", bias_std=0.2)
    _, k1, c1, o1, p1 = run_union([rule], "sum", "f32")
    gi = gpu_index(rule)
    out, pre, _ = layer_fwd(gi, gpu_layer(rule, "f32"), distinct_embs(rule), to_dev(rule.W), to_dev(rule.b))
    assert np.array_equal(k1, gi.export()["group_keys"].cpu().numpy())
    np.testing.assert_array_equal(p1, pre.cpu().numpy())      # same kernels, same order: bit for bit
    _, k2, c2, o2, p2 = run_union([rule, rule], "sum", "f32")
    np.testing.assert_array_equal(k2, k1)
    np.testing.assert_array_equal(c2, 2 * c1)
    np.testing.assert_array_equal(p2, 2 * p1)                  # x + x is exact
    _, _, _, _, m2 = run_union([rule, rule], "mean", "f32")
    _, _, _, _, m1 = run_union([rule], "mean", "f32")
    assert rel_rows(m2, m1).max() <= 1e-6


def test_three_branches_union_rule_transform():
    """Three bodies (the two ER bodies and a node-edge rule on the item ids)
    with MAX, then the union rule's transform tau(v) = v W_post + b_post and
    ReLU, once per key."""
    r1, r2 = er_rules(seed=5)
    r3 = relgen.node_edge(seed=16, n_nodes=3000, n_edges=20_000, d=128, h=128, agg="max", bias_std=0.1)
    rng = np.random.default_rng(3)
    post = (rng.standard_normal((128, 96)).astype(np.float32) / np.sqrt(128),
            rng.standard_normal(96).astype(np.float32))
    for agg in ("max", "mean"):
        U, keys, cnt, out, pre = run_union([r1, r2, r3], agg, "f32", post=post)
        r_keys, r_cnt, r_out, r_pre = oracle_union([r1, r2, r3], agg, post=post)
        np.testing.assert_array_equal(keys, r_keys)
        np.testing.assert_array_equal(cnt, r_cnt)
        assert rel_rows(pre, r_pre).max() <= 1e-5
        lin = r_pre @ post[0].astype(np.float64) + post[1]
        assert rel_rows(out, r_out, scale_ref=lin).max() <= 1e-5


def test_union_errors():
    from paper_2605_24207_amd import RelnnError, Union, union_fwd

    r1, r2 = er_rules(seed=6, n_buys=20_000)
    U = Union([gpu_index(r1), gpu_index(r2)])
    bad = relgen.node_edge(seed=1, d=32, h=32)                 # another width
    with pytest.raises(RelnnError, match="INVALID"):
        union_fwd(U, [gpu_layer(r1), gpu_layer(bad)], "sum", "none",
                  [distinct_embs(r1), distinct_embs(bad)], [to_dev(r1.W), to_dev(bad.W)])
