"""GPU parity of the index build and the forward layer against the FP64
oracle (through the C ABI).  Index results bit-exact; FP32 within 1e-5 and
BF16 within 2e-2 per-row relative error against the oracle on the FP32
master values; BF16 also against the oracle on bf16-rounded inputs."""
import numpy as np
import pytest

import relgen
from oracle import relnn_oracle as orc
from tests.helpers import (distinct_embs, elem_err, elem_scale, gpu_fwd, gpu_index, gpu_layer, oracle_fwd,
                           oracle_inputs, rel_rows, to_dev)

pytestmark = pytest.mark.gpu

TOL = {"f32": 1e-5, "bf16": 2e-2}
# element-wise, relative to the element's condition scale (elem_scale): FP32
# rounding stays near sqrt(K) 2^-24 of it; bf16 rounding of x and W moves
# each product by at most 2^-8 of its magnitude
ELEM_TOL = {"f32": 1e-5, "bf16": 6e-3}


def er_small(seed=3, n_user=3000, n_item=1500, n_cat=20, n_buys=60_000, d=128, h=128):
    return relgen.er_graph(seed=seed, n_user=n_user, n_item=n_item, n_cat=n_cat, n_buys=n_buys, d=d,
                           h=h, n_layers=1)


def random_rule(seed, agg="sum", keyed=True, chain=True, dangling=True, n_link=3000, d=(8, 16, 8), h=32):
    rng = np.random.default_rng(seed)
    nA, nB, nC = 300, 200, 50
    zA = rng.standard_normal((nA, d[0])).astype(np.float32)
    zB = rng.standard_normal((nB, d[1])).astype(np.float32)
    zC = rng.standard_normal((nC, d[2])).astype(np.float32)
    keysA = rng.permutation(np.arange(-5000, 5000, 7)[:nA]).astype(np.int32) if keyed else None
    c0 = (keysA[rng.integers(0, nA, n_link)] if keyed else rng.integers(0, nA, n_link)).astype(np.int32)
    c1 = rng.integers(-3 if dangling else 0, nB + (3 if dangling else 0), n_link).astype(np.int32)
    if dangling and keyed:
        c0[::11] = 12345
    atoms = [relgen.Atom(0, zA, keysA), relgen.Atom(1, zB)]
    chains = []
    if chain:
        chains = [relgen.Chain(src_col=1, vals=rng.integers(0, nC + (2 if dangling else 0), nB).astype(np.int32))]
        atoms.append(relgen.Atom(2, zC))
    K = sum(a.d for a in atoms)
    W = (rng.standard_normal((K, h)) / np.sqrt(K)).astype(np.float32)
    b = rng.standard_normal(h).astype(np.float32)
    return relgen.Rule(cols=[c0, c1], atoms=atoms, chains=chains, group_col=1, W=W, b=b, agg=agg,
                       act_post="relu")


def index_rules():
    hot = relgen.node_edge(seed=5, n_nodes=500, n_edges=20_000)
    hot.cols[1][: 15_000] = 7                       # one group spans many tiles
    allbad = relgen.node_edge(seed=6, n_nodes=100, n_edges=300)
    allbad.cols[0][:] = 1000                       # every FK dangles: E = 0
    return {
        "node_edge": relgen.node_edge(),
        "random_keyed_chain": random_rule(1),
        "random_dense": random_rule(2, keyed=False, chain=False, dangling=False),
        "hot_segment": hot,
        "all_dangling": allbad,
        "er_item": relgen.er_item_rule(er_small()),
        "er_user": relgen.er_user_rule(er_small()),
    }


@pytest.mark.parametrize("name", list(index_rules()))
def test_index_bit_exact(name):
    rule = index_rules()[name]
    gi = gpu_index(rule)
    ref = orc.build_index(rule)
    assert (gi.E, gi.G) == (ref.E, ref.G)
    ex = {k: v.cpu().numpy() for k, v in gi.export().items()}
    np.testing.assert_array_equal(ex["group_keys"], ref.group_keys)
    np.testing.assert_array_equal(ex["offsets"], ref.offsets)
    np.testing.assert_array_equal(ex["link_rows"], ref.link_row)
    for j in range(len(rule.atoms)):
        np.testing.assert_array_equal(ex["tuple_rows"][j], ref.rows[j])


def test_duplicate_key_is_rejected():
    from paper_2605_24207_amd import RelnnError

    rule = random_rule(4)
    rule.atoms[0].keys[3] = rule.atoms[0].keys[4]
    with pytest.raises(RelnnError, match="NOT_UNIQUE"):
        gpu_index(rule)


def check_fwd(rule, dtype, plain=False, pushdown=False):
    res = gpu_fwd(rule, dtype, plain, pushdown=pushdown)
    idx, out, pre, am = oracle_fwd(rule, "f32")
    assert res["out"].shape == out.shape
    e_pre = rel_rows(res["pre"], pre)
    e_out = rel_rows(res["out"], out, scale_ref=pre)
    assert e_pre.max() <= TOL[dtype], (e_pre.max(), np.percentile(e_pre, 99))
    assert e_out.max() <= TOL[dtype]
    # element by element, against the condition scale of each output element
    assert elem_err(res["pre"], pre, elem_scale(rule, idx, dtype)) <= ELEM_TOL[dtype]
    am_ref = am
    if dtype == "bf16":   # kernel arithmetic alone, on the rounded inputs
        _, out_b, pre_b, am_b = oracle_fwd(rule, "bf16", idx=idx)
        assert rel_rows(res["pre"], pre_b).max() <= 1e-5 * np.sqrt(rule.K)
        am_ref = am_b     # the argmax is decided on the values the kernel sees
    if rule.agg == "max":
        embs, W, b = oracle_inputs(rule, dtype)
        am_g = res["argmax"]
        diff = np.nonzero(am_g != am_ref)
        for g, c in zip(*diff):
            y = orc.transform(orc.gather_concat(idx, embs, [am_g[g, c]]), W, b, rule.act_pre)[0, c]
            assert abs(y - pre[g, c]) <= 4 * TOL[dtype] * max(1.0, abs(pre[g, c]))
        assert len(diff[0]) <= 0.01 * am_ref.size + 1
    return res


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
@pytest.mark.parametrize("agg", ["sum", "mean", "max"])
@pytest.mark.parametrize("plain", [False, True])
def test_fwd_node_edge(dtype, agg, plain):
    check_fwd(relgen.node_edge(agg=agg, bias_std=0.5), dtype, plain)


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
@pytest.mark.parametrize("agg", ["sum", "max"])
def test_fwd_wide_256(dtype, agg):
    check_fwd(relgen.node_edge(d=256, h=256, agg=agg, w_std=1 / 32), dtype)


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
@pytest.mark.parametrize("which", ["item", "user"])
def test_fwd_er_rules(dtype, which):
    g = er_small()
    rule = relgen.er_item_rule(g) if which == "item" else relgen.er_user_rule(g)
    check_fwd(rule, dtype)


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
@pytest.mark.parametrize("agg", ["sum", "mean", "max"])
def test_fwd_hot_segment_and_ragged_tail(dtype, agg):
    rule = relgen.node_edge(seed=9, n_nodes=700, n_edges=40_003, agg=agg, act_pre="relu", bias_std=0.3)
    rule.cols[1][:30_000] = 11          # a group of 30k tuples spanning ~470 tiles
    check_fwd(rule, dtype)


@pytest.mark.parametrize("agg", ["sum", "max"])
def test_fwd_random_keyed_chains(agg):
    check_fwd(random_rule(7, agg=agg), "f32")


@pytest.mark.parametrize("d,h", [((8, 16, 8), 48),          # K 32 in a 64-wide tile (pad), 3 column waves
                                 ((24, 40, 64), 80),        # K 128, 5 column waves
                                 ((64, 72, 64), 112),       # K 200 in a 256-wide tile, 7 column waves
                                 ((96, 104, 96), 128),      # K 296 in a 384-wide tile
                                 ((16, 16, 8), 64),         # BF16: two 32-column waves
                                 ((40, 40, 48), 96),        # BF16: three 32-column waves
                                 ((96, 104, 96), 256),      # two 128-column chunks per tuple range
                                 ((200, 200, 64), 384)])    # BF16: K 464 in a 512-wide tile, three chunks
@pytest.mark.parametrize("agg", ["sum", "mean", "max"])
@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_fwd_tile_shapes_and_long_ranges(d, h, agg, dtype):
    """~4k tiles (many per block, so the load ring wraps many times) over
    widths that leave a zero pad in the LDS tile and odd column-wave counts."""
    check_fwd(random_rule(21, agg=agg, n_link=150_000, d=d, h=h), dtype)


@pytest.mark.parametrize("h", [256, 384])
@pytest.mark.parametrize("agg", ["sum", "mean", "max"])
@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_fwd_column_chunks_few_tiles(h, agg, dtype):
    """Fewer tuple ranges than one round of XCDs: the column-chunked grid has
    blocks with no range, which must leave at once."""
    check_fwd(random_rule(33, agg=agg, n_link=150, d=(96, 104, 96), h=h), dtype)


@pytest.mark.parametrize("case", ["hot_ragged", "long_ranges", "chunks_512"])
@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_fwd_max_without_argmax(case, dtype):
    """MAX asked for values only: the same values and outputs, bit for bit,
    as with the maximiser positions, across tiles, blocks and column chunks."""
    import torch

    from paper_2605_24207_amd import layer_fwd

    if case == "hot_ragged":
        rule = relgen.node_edge(seed=9, n_nodes=700, n_edges=40_003, agg="max", act_pre="relu", bias_std=0.3)
        rule.cols[1][:30_000] = 11
    elif case == "long_ranges":
        rule = random_rule(21, agg="max", n_link=150_000, d=(96, 104, 96), h=128)
    else:
        rule = random_rule(22, agg="max", n_link=60_000, d=(200, 200, 64), h=256)
    gi = gpu_index(rule)
    layer = gpu_layer(rule, dtype)
    embs, W, b = distinct_embs(rule, dtype), to_dev(rule.W, dtype), to_dev(rule.b)
    out1, pre1, am1 = layer_fwd(gi, layer, embs, W, b)
    out2, pre2, am2 = layer_fwd(gi, layer, embs, W, b, want_argmax=False)
    torch.cuda.synchronize()
    assert am1 is not None and am2 is None
    assert torch.equal(pre1, pre2) and torch.equal(out1, out2)
    _, o_out, o_pre, _ = oracle_fwd(rule, "f32")
    tol = TOL[dtype]
    assert rel_rows(pre2.cpu().numpy(), o_pre).max() <= tol


@pytest.mark.parametrize("case", ["one_tuple", "one_group"])
@pytest.mark.parametrize("agg", ["sum", "mean", "max"])
@pytest.mark.parametrize("dtype", ["f32", "bf16"])
@pytest.mark.parametrize("h", [32, 256])
def test_fwd_degenerate_sizes(case, agg, dtype, h):
    """A join of one tuple, and one group holding every tuple of many blocks'
    ranges (the whole output is one carried group)."""
    n_edges = 1 if case == "one_tuple" else 20_000
    rule = relgen.node_edge(seed=31, n_nodes=300, n_edges=n_edges, d=32, h=h, agg=agg, bias_std=0.3)
    if case == "one_group":
        rule.cols[1][:] = 5
    res = check_fwd(rule, dtype)
    assert res["out"].shape[0] == 1


def test_fwd_empty_join():
    rule = index_rules()["all_dangling"]
    res = gpu_fwd(rule, "f32")
    assert res["out"].shape == (0, rule.h)


def test_plain_and_fused_agree():
    """Same FP32 arithmetic in a different k order: agreement to rounding."""
    rule = relgen.node_edge(seed=10, n_nodes=400, n_edges=9000, bias_std=0.1)
    a = gpu_fwd(rule, "f32", plain=False)
    b = gpu_fwd(rule, "f32", plain=True)
    assert rel_rows(a["pre"], b["pre"]).max() <= 2e-6


def test_deterministic_and_permutation_invariant():
    rule = relgen.node_edge(seed=12, n_nodes=300, n_edges=12_000, bias_std=0.1)
    a = gpu_fwd(rule, "f32")
    b = gpu_fwd(rule, "f32")
    np.testing.assert_array_equal(a["pre"], b["pre"])
    p = np.random.default_rng(0).permutation(rule.n_link)
    rule.cols = [c[p] for c in rule.cols]
    c = gpu_fwd(rule, "f32")
    np.testing.assert_array_equal(a["pre"], c["pre"])


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
@pytest.mark.parametrize("agg", ["sum", "max"])
@pytest.mark.parametrize("plain", [False, True])
def test_workspace_is_not_overrun(dtype, agg, plain):
    """Kernels stay inside the workspace relnn_workspace_size reports: a
    sentinel region right after it must survive the call."""
    import torch

    from paper_2605_24207_amd import layer_fwd, workspace_size
    from tests.helpers import distinct_embs, gpu_layer, to_dev

    rule = relgen.node_edge(seed=13, n_nodes=700, n_edges=20_000, agg=agg)
    idx = gpu_index(rule)
    layer = gpu_layer(rule, dtype, plain)
    n = workspace_size(idx, layer)
    buf = torch.full((n + 65536,), 0xAB, dtype=torch.uint8, device="cuda")
    layer_fwd(idx, layer, distinct_embs(rule, dtype), to_dev(rule.W, dtype), to_dev(rule.b), ws=buf[:n])
    torch.cuda.synchronize()
    assert bool((buf[n:] == 0xAB).all())


@pytest.mark.parametrize("d,h", [(64, 64), (256, 256)])
@pytest.mark.parametrize("agg", ["sum", "max"])
@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_two_hop_cobuy(d, h, agg, dtype):
    """Buys |x| Buys^T on item, at most 50 paths per item, grouped by the
    first buyer: index bit-exact and layer within the bound."""
    g = relgen.er_graph(seed=8, n_user=3000, n_item=600, n_cat=10, n_buys=20_000, n_layers=1)
    rule = relgen.cobuy_rule(g, d=d, h=h, cap=50, agg=agg)
    gi = gpu_index(rule)
    ref = orc.build_index(rule)
    assert (gi.E, gi.G) == (ref.E, ref.G)
    ex = {k: v.cpu().numpy() for k, v in gi.export().items()}
    np.testing.assert_array_equal(ex["link_rows"], ref.link_row)
    np.testing.assert_array_equal(ex["offsets"], ref.offsets)
    for j in range(2):
        np.testing.assert_array_equal(ex["tuple_rows"][j], ref.rows[j])
    check_fwd(rule, dtype)


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
@pytest.mark.parametrize("agg", ["sum", "mean", "max"])
def test_pushdown_node_edge(dtype, agg):
    """Transform pushed below the join: same layer, same oracle bound."""
    check_fwd(relgen.node_edge(agg=agg, bias_std=0.5), dtype, pushdown=True)


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
@pytest.mark.parametrize("which", ["item", "user"])
def test_pushdown_er_rules(dtype, which):
    """The ER rules have atoms keyed by the head key (Item and Category in
    the Item rule, User in the User rule): their terms enter once per group."""
    g = er_small()
    g.b_item[0] = np.random.default_rng(1).standard_normal(128).astype(np.float32)
    g.b_user[0] = np.random.default_rng(2).standard_normal(128).astype(np.float32)
    rule = relgen.er_item_rule(g) if which == "item" else relgen.er_user_rule(g)
    check_fwd(rule, dtype, pushdown=True)


@pytest.mark.parametrize("agg", ["sum", "mean", "max"])
def test_pushdown_hot_segment(agg):
    rule = relgen.node_edge(seed=9, n_nodes=700, n_edges=40_003, agg=agg, bias_std=0.3)
    rule.cols[1][:30_000] = 11
    check_fwd(rule, "f32", pushdown=True)


def test_pushdown_rejects_nonaffine_transform():
    from paper_2605_24207_amd import RelnnError

    rule = relgen.node_edge(act_pre="relu")
    with pytest.raises(RelnnError, match="INVALID"):
        gpu_fwd(rule, "f32", pushdown=True)
