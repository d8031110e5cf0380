"""Parity of the widened rows at the sizes bench.py times, in its launch
configuration, on seeded samples of the output that the oracle evaluates.

* Attention: 2M targets (Zipf 1.1), 4M sources, 20M tuples, d = dv = 128,
  8 heads, FP32 and BF16 inputs: out and lse of sampled targets (a group of
  about 200k tuples among them, spread over many waves' ranges); dQ of the
  sampled targets; dK and dV of sampled sources, whose sums run over every
  group that joins them.
* Union: Item(i) over two bodies on the halves of Buys 20M (the Item rule,
  K = 384, and the User rule's body grouped by item, K = 256), MEAN once;
  its backward on sampled User, Item and Category rows.
* Product: Item(i; mean(relu(z_u * z_i * z_c))) over Buys 20M; its
  backward on sampled User, Item (one of about 50k tuples) and Category
  rows.
* Triangle: the DHN triangle rule over 20k graphs of 40 nodes; the graphs are
  disjoint, so the oracle evaluates a sample of whole graphs.

The oracle sees compact copies of the relations (the rows the sample
reaches), so its inputs stay small while the GPU runs at full size.
"""
import copy

import numpy as np
import pytest

import relgen
from oracle import relnn_oracle as orc
from tests.helpers import distinct_embs, gpu_index, gpu_layer, oracle_inputs, rel_rows, to_dev
from tests.test_gpu_attention import cond_err, grad_scales
from tests.test_oracle_attention import attn_rule

pytestmark = pytest.mark.gpu

TOL = {"f32": 1e-5, "bf16": 2e-2}


def near_size_key(keys, size, rng):
    cnt = np.bincount(keys)
    nz = np.nonzero(cnt)[0]
    return nz[np.argmin(np.abs(cnt[nz] - size))], cnt


# ---------------------------------------------------------------- attention
@pytest.fixture(scope="module")
def attn_data():
    rng = np.random.default_rng(7)
    n_t, n_s, E, d = 2_000_000, 4_000_000, 20_000_000, 128
    tgt = relgen.zipf_ids(rng, E, n_t, 1.1).astype(np.int32)
    src = rng.integers(0, n_s, E).astype(np.int32)
    r2 = np.random.default_rng(8)
    Q = r2.standard_normal((n_t, d), dtype=np.float32)
    K = r2.standard_normal((n_s, d), dtype=np.float32)
    V = r2.standard_normal((n_s, d), dtype=np.float32)
    return tgt, src, Q, K, V


def compact_attn(tgt, src, Q, K, V, sel):
    """The attention rule over the selected tuples, with Q, K and V reduced
    to the rows they reach; returns the rule, the compact arrays and the
    original ids of their rows."""
    t, s = tgt[sel], src[sel]
    uq, tc = np.unique(t, return_inverse=True)
    us, sc = np.unique(s, return_inverse=True)
    Qc, Kc, Vc = Q[uq], K[us], V[us]
    return attn_rule(tc, sc, Qc, Kc, Vc), Qc, Kc, Vc, uq, us


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_attention_full_size(attn_data, dtype):
    import torch

    from paper_2605_24207_amd import Index, attn_bwd, attn_fwd

    tgt, src, Q, K, V = attn_data
    heads, scale = 8, 0.25
    n_t, n_s = Q.shape[0], K.shape[0]
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    cv = (lambda x: x.to(torch.bfloat16)) if dtype == "bf16" else (lambda x: x)
    ix = Index([t(tgt), t(src)], [(n_t, 0, None), (n_s, 1, None), (n_s, 1, None)], 0, bwd=True)
    q, k, v = cv(t(Q)), cv(t(K)), cv(t(V))
    out, lse = attn_fwd(ix, q, k, v, heads, scale)
    dout = np.random.default_rng(9).standard_normal((ix.G, 128), dtype=np.float32)
    dq, dk, dv = (torch.zeros(x.shape, dtype=torch.float32, device="cuda") for x in (q, k, v))
    attn_bwd(ix, q, k, v, heads, scale, out, lse, t(dout), dq, dk, dv)
    torch.cuda.synchronize()
    gk = ix.export()["group_keys"].cpu().numpy()
    out, lse = out.cpu().numpy(), lse.cpu().numpy()
    r = (lambda a: orc.bf16_round(a)) if dtype == "bf16" else (lambda a: a)
    rng = np.random.default_rng(11)

    # targets: random ones plus one of about 200k tuples
    big, cnt = near_size_key(tgt, 200_000, rng)
    assert cnt[big] > 100_000
    keys = np.unique(np.concatenate([rng.choice(np.nonzero(cnt)[0], 60, replace=False), [big]]))
    rule, Qc, Kc, Vc, uq, us = compact_attn(tgt, src, Q, K, V, np.isin(tgt, keys))
    idx = orc.build_index(rule)
    rows = np.searchsorted(gk, uq[idx.group_keys])
    o_out, o_lse = orc.attention_fwd(idx, Qc, Kc, Vc, heads, scale)
    assert rel_rows(out[rows], o_out).max() <= TOL[dtype]
    assert np.abs(lse[rows] - o_lse).max() <= TOL[dtype] * max(1.0, np.abs(o_lse).max())
    if dtype == "bf16":                              # the kernel's arithmetic on the rounded inputs
        b_out, _ = orc.attention_fwd(idx, r(Qc), r(Kc), r(Vc), heads, scale)
        assert rel_rows(out[rows], b_out).max() <= 1e-4
    o_dq, _, _ = orc.attention_bwd(idx, Qc, Kc, Vc, heads, scale, dout[rows])
    c_dq, _, _ = grad_scales(idx, Qc, Kc, Vc, heads, scale, dout[rows])
    assert cond_err(dq.cpu().numpy()[uq], o_dq, c_dq).max() <= TOL[dtype]

    # sources: their dK and dV sum over every group that joins them; take
    # sources whose groups stay below 300k tuples (the oracle's size)
    order = np.argsort(src, kind="stable")
    ss = src[order]
    cand = rng.choice(n_s, 400, replace=False)
    lo, hi = np.searchsorted(ss, cand), np.searchsorted(ss, cand, side="right")
    ok = [c for c, a, b in zip(cand, lo, hi) if b > a and cnt[tgt[order[a:b]]].max() <= 300_000]
    S = np.sort(np.array(ok[:40]))
    groups = np.unique(tgt[np.isin(src, S)])
    rule, Qc, Kc, Vc, uq, us = compact_attn(tgt, src, Q, K, V, np.isin(tgt, groups))
    idx = orc.build_index(rule)
    rows = np.searchsorted(gk, uq[idx.group_keys])
    _, o_dk, o_dv = orc.attention_bwd(idx, Qc, Kc, Vc, heads, scale, dout[rows])
    _, c_dk, c_dv = grad_scales(idx, Qc, Kc, Vc, heads, scale, dout[rows])
    pos = np.searchsorted(us, S)
    assert np.array_equal(us[pos], S)
    assert cond_err(dk.cpu().numpy()[S], o_dk[pos], c_dk[pos]).max() <= TOL[dtype]
    assert cond_err(dv.cpu().numpy()[S], o_dv[pos], c_dv[pos]).max() <= TOL[dtype]


# ---------------------------------------------------------------- ER rows
@pytest.fixture(scope="module")
def er():
    return relgen.er_graph(n_layers=1)


def restrict(rule, keys):
    sub = copy.copy(rule)
    sel = np.isin(rule.cols[rule.group_col], keys)
    sub.cols = [c[sel] for c in rule.cols]
    return sub


def item_keys(g, seed):
    rng = np.random.default_rng(seed)
    big, cnt = near_size_key(g.buys_i, 50_000, rng)
    return np.unique(np.concatenate([rng.choice(np.nonzero(cnt)[0], 80, replace=False), [big]]))


def test_union_full_size(er):
    import torch

    from paper_2605_24207_amd import Union, union_fwd

    g = er
    half = len(g.buys_u) // 2
    r1 = relgen.er_item_rule(g)
    r2 = relgen.er_user_rule(g)
    r2.group_col = 1                                        # the User body grouped by item
    r1.cols = [c[:half] for c in r1.cols]
    r2.cols = [c[half:] for c in r2.cols]
    idx = [gpu_index(r) for r in (r1, r2)]
    U = Union(idx)
    out, pre, _ = union_fwd(U, [gpu_layer(r1), gpu_layer(r2)], "mean", "relu", [distinct_embs(r1), distinct_embs(r2)],
                         [to_dev(r1.W), to_dev(r2.W)], [to_dev(r1.b), to_dev(r2.b)])
    torch.cuda.synchronize()
    keys_all = U.export()["keys"].cpu().numpy()
    keys = item_keys(g, 12)
    branches = []
    for r in (r1, r2):
        sub = restrict(r, keys)
        embs, W, b = oracle_inputs(sub, "f32")
        branches.append((orc.build_index(sub), embs, W, b, sub.act_pre))
    o_keys, o_out, o_pre, _ = orc.union_fwd(branches, "mean", "relu")
    np.testing.assert_array_equal(o_keys, np.sort(keys))
    rows = np.searchsorted(keys_all, o_keys)
    assert np.array_equal(keys_all[rows], o_keys)
    assert rel_rows(pre.cpu().numpy()[rows], o_pre).max() <= TOL["f32"]
    assert rel_rows(out.cpu().numpy()[rows], o_out, scale_ref=o_pre).max() <= TOL["f32"]


def test_product_full_size(er):
    import torch

    from paper_2605_24207_amd import Layer, layer_fwd

    g = er
    rule = relgen.er_item_rule(g)
    rule.agg, rule.act_pre, rule.act_post = "mean", "relu", "none"
    gi = gpu_index(rule)
    L = Layer([128, 128, 128], 128, "f32", "mean", "relu", "none", transform="product")
    out, pre, _ = layer_fwd(gi, L, distinct_embs(rule), None)
    torch.cuda.synchronize()
    gk = gi.export()["group_keys"].cpu().numpy()
    keys = item_keys(g, 13)
    sub = restrict(rule, keys)
    idx = orc.build_index(sub)
    _, o_pre, _ = orc.layer_fwd(idx, [a.emb for a in sub.atoms], None, None, "mean", "relu", "none", tf="product")
    rows = np.searchsorted(gk, idx.group_keys)
    assert rel_rows(pre.cpu().numpy()[rows], o_pre).max() <= TOL["f32"]


# ---------------------------------------------------------------- triangle
def test_triangle_full_size():
    import torch

    from paper_2605_24207_amd import layer_fwd

    n_graphs, n_nodes = 20_000, 40
    rule = relgen.triangle_rule(n_graphs=n_graphs, n_nodes=n_nodes, avg_degree=6, d=64, h=64, bias_std=0.2)
    gi = gpu_index(rule)
    out, pre, _ = layer_fwd(gi, gpu_layer(rule), distinct_embs(rule), to_dev(rule.W), to_dev(rule.b))
    torch.cuda.synchronize()
    gk = gi.export()["group_keys"].cpu().numpy()
    # whole graphs: every column of the link and step relations carries the graph id
    rng = np.random.default_rng(14)
    graphs = np.sort(rng.choice(n_graphs, 40, replace=False))
    sub = copy.deepcopy(rule)
    sel = np.isin(rule.cols[0], graphs)
    sub.cols = [c[sel] for c in rule.cols]
    for st in sub.steps:
        ssel = np.isin(st.cols[0], graphs)
        st.cols = [c[ssel] for c in st.cols]
    idx = orc.build_index(sub)
    assert idx.E > 100
    embs, W, b = oracle_inputs(sub, "f32")
    o_out, o_pre, _ = orc.layer_fwd(idx, embs, W, b, sub.agg, sub.act_pre, sub.act_post)
    rows = np.searchsorted(gk, idx.group_keys)
    assert np.array_equal(gk[rows], idx.group_keys)
    assert rel_rows(pre.cpu().numpy()[rows], o_pre).max() <= TOL["f32"]
    assert rel_rows(out.cpu().numpy()[rows], o_out, scale_ref=o_pre).max() <= TOL["f32"]


# ------------------------------------------------- backward of the next rows
def sample_rows(g, rng):
    """Sampled rows of each ER relation: users and categories at random,
    items at random plus the one nearest 50k tuples."""
    users = np.sort(rng.choice(g.user.shape[0], 60, replace=False))
    big, cnt = near_size_key(g.buys_i, 50_000, rng)
    items = np.unique(np.concatenate([rng.choice(np.nonzero(cnt)[0], 60, replace=False), [big]]))
    cats = np.sort(rng.choice(g.cat.shape[0], 2, replace=False))
    return users, items, cats


def touching(rule, g, which, rows):
    """The rule restricted to the tuples that join one of ``rows`` of the
    given relation (0 user, 1 item, 2 category)."""
    r_of = {0: rule.cols[0], 1: rule.cols[1], 2: g.belongs_cat[rule.cols[1]]}[which]
    sub = copy.copy(rule)
    sel = np.isin(r_of, rows)
    sub.cols = [c[sel] for c in rule.cols]
    return sub


def test_product_backward_full_size(er):
    """Item(i; mean(relu(z_u * z_i * z_c))) over Buys 20M: the gradients of
    sampled User, Item and Category rows (the hot Item's row sums 50k
    tuples; a Category's about 20k) against the oracle.  A sampled row's
    gradient involves only the tuples that join it, each routed its group's
    gradient over the group's full member count, so the oracle runs SUM over
    those tuples with dout divided by the full counts (the definition of
    MEAN's routing)."""
    import torch

    from paper_2605_24207_amd import Layer, layer_bwd, layer_fwd

    g = er
    rule = relgen.er_item_rule(g)
    rule.agg, rule.act_pre, rule.act_post = "mean", "relu", "none"
    gi = gpu_index(rule, bwd=True)
    L = Layer([128, 128, 128], 128, "f32", "mean", "relu", "none", transform="product")
    embs = distinct_embs(rule)
    out, _, _ = layer_fwd(gi, L, embs, None)
    dout = torch.from_numpy(np.random.default_rng(15).standard_normal((gi.G, 128)).astype(np.float32)).cuda()
    demb = [torch.zeros(e.shape, device="cuda") for e in embs]
    layer_bwd(gi, L, embs, None, None, None, None, dout, demb, None)
    torch.cuda.synchronize()
    ex = gi.export()
    gk = ex["group_keys"].cpu().numpy()
    cnt = np.diff(ex["offsets"].cpu().numpy()).astype(np.float64)
    dout = dout.cpu().numpy().astype(np.float64)
    o_embs = [a.emb for a in rule.atoms]
    for which, rows in enumerate(sample_rows(g, np.random.default_rng(16))):
        sub = touching(rule, g, which, rows)
        idx = orc.build_index(sub)
        q = np.searchsorted(gk, idx.group_keys)
        assert np.array_equal(gk[q], idx.group_keys)
        d = dout[q] / cnt[q][:, None]
        zero = np.zeros_like(d)
        ref = orc.product_bwd(idx, o_embs, zero, None, d, "sum", "relu", "none")[which][rows]
        mask = orc.product(idx, o_embs, slice(None), "none") > 0
        mag = orc.product_bwd(idx, [np.abs(e) for e in o_embs], zero, None, np.abs(d), "sum", "relu", "none",
                              pre_mask=mask)[which][rows]
        got = demb[which].cpu().numpy()[rows]
        assert rel_rows(got, ref, scale_ref=mag).max() <= TOL["f32"], which


def test_union_backward_full_size(er):
    """The union of two bodies of Item(i) over the halves of Buys 20M, MEAN
    once, ReLU after: the gradients of sampled User, Item and Category rows
    (their tuples in both bodies) against the oracle's union backward.  The
    union's ReLU is taken from the kernel's aggregate and the MEAN over the
    union's full member counts, so the oracle runs SUM over the tuples that
    join a sampled row with the gradient so divided."""
    import torch

    from paper_2605_24207_amd import Union, union_bwd, union_fwd

    g = er
    half = len(g.buys_u) // 2
    r1 = relgen.er_item_rule(g)
    r2 = relgen.er_user_rule(g)
    r2.group_col = 1
    r1.cols = [c[:half] for c in r1.cols]
    r2.cols = [c[half:] for c in r2.cols]
    U = Union([gpu_index(r, bwd=True) for r in (r1, r2)])
    dev = {id(a): to_dev(a) for a in (g.user, g.item, g.cat)}
    embs = [[dev[id(a.emb)] for a in r.atoms] for r in (r1, r2)]
    grad = {k: torch.zeros(t.shape, device="cuda") for k, t in dev.items()}
    demb = [[grad[id(a.emb)] for a in r.atoms] for r in (r1, r2)]
    layers = [gpu_layer(r1), gpu_layer(r2)]
    Ws, bs = [to_dev(r1.W), to_dev(r2.W)], [to_dev(r1.b), to_dev(r2.b)]
    out, pre, _ = union_fwd(U, layers, "mean", "relu", embs, Ws, bs)
    dout = torch.from_numpy(np.random.default_rng(17).standard_normal((U.G, 128)).astype(np.float32)).cuda()
    dWs = [torch.empty(r.K, 128, device="cuda") for r in (r1, r2)]
    union_bwd(U, layers, "mean", "relu", embs, Ws, bs, None, None, pre, None, dout, demb, dWs)
    torch.cuda.synchronize()
    ex = U.export()
    keys_all = ex["keys"].cpu().numpy()
    members = ex["counts"].cpu().numpy().astype(np.float64)
    dV = dout.cpu().numpy().astype(np.float64) * (pre.cpu().numpy() > 0)
    for which, rows in enumerate(sample_rows(g, np.random.default_rng(18))):
        branches, abs_branches = [], []
        for r in (r1, r2):
            sub = touching(r, g, which, rows)
            embs_o, W, b = oracle_inputs(sub, "f32")
            branches.append((orc.build_index(sub), embs_o, W, b, sub.act_pre))
            abs_branches.append((branches[-1][0], embs_o, np.abs(W.astype(np.float64)), b, sub.act_pre))
        keys = np.array(sorted(set().union(*[set(br[0].group_keys.tolist()) for br in branches])), np.int64)
        q = np.searchsorted(keys_all, keys)
        assert np.array_equal(keys_all[q], keys)
        d = dV[q] / members[q][:, None]
        zero = np.zeros_like(d)
        grads, _, _ = orc.union_bwd(branches, zero, None, d, "sum", "none")
        mags, _, _ = orc.union_bwd(abs_branches, zero, None, np.abs(d), "sum", "none")
        target = (g.user, g.item, g.cat)[which]
        ref, mag = 0, 0
        for r, (de, _, _), (dm, _, _) in zip((r1, r2), grads, mags):
            for a, x, m in zip(r.atoms, de, dm):
                if a.emb is target:
                    ref, mag = ref + x[rows], mag + m[rows]
        got = grad[id(target)].cpu().numpy()[rows]
        assert rel_rows(got, ref, scale_ref=mag).max() <= TOL["f32"], which
