"""GPU parity of segmented softmax attention (through the C ABI) against the
FP64 oracle: out and lse per group within 1e-5 (FP32) and 2e-2 (BF16 inputs)
relative per row, and the gradients of Q, K and V likewise.  Cases: several
head splits, unequal key and value widths, a hot target whose tuples span
many waves' ranges (the carried softmax states merged by the fix-up),
one-tuple groups, and K and V read from one relation (one gradient
buffer)."""
import numpy as np
import pytest

from oracle import relnn_oracle as orc
from tests.helpers import gpu_index, rel_rows
from tests.test_oracle_attention import attn_rule

pytestmark = pytest.mark.gpu

TOL = {"f32": 1e-5, "bf16": 2e-2}


def workload(seed, n_t=3000, n_s=5000, m=120_000, d=64, dv=64, hot=0, same_kv=False):
    """Targets t with Zipf-skewed degrees (HGT-like in-neighbourhoods), one
    hot target of `hot` extra tuples, and a few one-tuple targets."""
    rng = np.random.default_rng(seed)
    w = np.arange(1, n_t + 1, dtype=np.float64) ** -0.8
    t = rng.choice(n_t - 3, size=m - 3 - hot, p=w[:n_t - 3] / w[:n_t - 3].sum())
    t = np.concatenate([t, np.full(hot, 7), np.arange(n_t - 3, n_t)])
    s = rng.integers(0, n_s, len(t))
    Q = rng.standard_normal((n_t, d)).astype(np.float32)
    K = rng.standard_normal((n_s, d)).astype(np.float32)
    V = K[:, :dv].copy() if same_kv else rng.standard_normal((n_s, dv)).astype(np.float32)
    if same_kv:
        assert d == dv
        V = K
    return attn_rule(t, s, Q, K, V), Q, K, V


def dev(a, dtype):
    import torch

    x = torch.from_numpy(np.ascontiguousarray(a)).cuda()
    return x.to(torch.bfloat16) if dtype == "bf16" else x


def run(rule, Q, K, V, heads, scale, dtype, same_kv=False, bwd=True):
    import torch

    from paper_2605_24207_amd import attn_bwd, attn_fwd

    gi = gpu_index(rule, bwd=bwd)
    q, k = dev(Q, dtype), dev(K, dtype)
    v = k if same_kv else dev(V, dtype)
    out, lse = attn_fwd(gi, q, k, v, heads, scale)
    res = {"gi": gi, "out": out.cpu().numpy(), "lse": lse.cpu().numpy()}
    if bwd:
        dout = np.random.default_rng(9).standard_normal((gi.G, V.shape[1])).astype(np.float32)
        dq = torch.zeros(q.shape, dtype=torch.float32, device="cuda")
        dk = torch.zeros(k.shape, dtype=torch.float32, device="cuda")
        dv = dk if same_kv else torch.zeros(v.shape, dtype=torch.float32, device="cuda")
        attn_bwd(gi, q, k, v, heads, scale, out, lse, torch.from_numpy(dout).cuda(), dq, dk, dv)
        torch.cuda.synchronize()
        res.update(dout=dout, dq=dq.cpu().numpy(), dk=dk.cpu().numpy(), dv=dv.cpu().numpy())
    return res


def grad_scales(idx, Q, K, V, heads, scale, dout):
    """Condition scales of the gradient rows: the same sums as the backward
    with every term replaced by its magnitude (|ds| bounded by a (|dp| +
    sum a |dp|)).  A gradient that cancels to zero (a one-tuple group's dq)
    is judged against the size of the terms that cancelled, not against 0."""
    Q, K, V, dout = (np.asarray(a, np.float64) for a in (Q, K, V, dout))
    d, dv = K.shape[1], V.shape[1]
    sq, sk, sv = np.zeros_like(Q), np.zeros_like(K), np.zeros_like(V)
    for g in range(idx.G):
        s0, e0 = int(idx.offsets[g]), int(idx.offsets[g + 1])
        n = e0 - s0
        rq, rk, rv = idx.rows[0][s0:e0], idx.rows[1][s0:e0], idx.rows[2][s0:e0]
        S = scale * (Q[rq] * K[rk]).reshape(n, heads, -1).sum(axis=2)
        ex = np.exp(S - S.max(axis=0))
        a = ex / ex.sum(axis=0)
        do = np.abs(dout[g]).reshape(heads, dv // heads)
        dp = (np.abs(V[rv]).reshape(n, heads, -1) * do[None]).sum(axis=2)
        ds = a * (dp + (a * dp).sum(axis=0))
        np.add.at(sv, rv, (a[:, :, None] * do[None]).reshape(n, dv))
        np.add.at(sq, rq, (abs(scale) * ds[:, :, None] * np.abs(K[rk]).reshape(n, heads, -1)).reshape(n, d))
        np.add.at(sk, rk, (abs(scale) * ds[:, :, None] * np.abs(Q[rq]).reshape(n, heads, -1)).reshape(n, d))
    return sq, sk, sv


def cond_err(g, r, c):
    g, r = np.asarray(g, np.float64), np.asarray(r, np.float64)
    return np.linalg.norm(g - r, axis=1) / np.maximum(np.linalg.norm(c, axis=1), 1e-30)


def check(rule, Q, K, V, heads, scale, dtype, same_kv=False):
    res = run(rule, Q, K, V, heads, scale, dtype, same_kv)
    idx = orc.build_index(rule)
    out, lse = orc.attention_fwd(idx, Q, K, V, heads, scale)
    tol = TOL[dtype]
    assert rel_rows(res["out"], out).max() <= tol
    assert np.abs(res["lse"] - lse).max() <= tol * max(1.0, np.abs(lse).max())
    dq, dk, dv = orc.attention_bwd(idx, Q, K, V, heads, scale, res["dout"])
    cq, ck, cv = grad_scales(idx, Q, K, V, heads, scale, res["dout"])
    if same_kv:
        dk, ck = dk + dv, ck + cv
        dv, cv = dk, ck
    for j, (got, ref, c) in enumerate(((res["dq"], dq, cq), (res["dk"], dk, ck), (res["dv"], dv, cv))):
        used = np.zeros(len(ref), bool)            # rows some tuple joins
        used[np.unique(idx.rows[j])] = True
        if same_kv and j > 0:
            used[np.unique(idx.rows[1])] = True
        assert cond_err(got[used], ref[used], c[used]).max() <= tol
        assert np.abs(got[~used]).max(initial=0.0) == 0.0
    if dtype == "bf16":                  # the kernels' arithmetic on the bf16-rounded inputs
        r = lambda a: orc.bf16_round(a)
        o2, _ = orc.attention_fwd(idx, r(Q), r(K), r(V), heads, scale)
        assert rel_rows(res["out"], o2).max() <= 1e-4
    return res


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
@pytest.mark.parametrize("heads", [1, 2, 8])
def test_attention_heads(heads, dtype):
    rule, Q, K, V = workload(1)
    check(rule, Q, K, V, heads, 1.0 / np.sqrt(64 / heads), dtype)


def test_attention_unequal_widths():
    rule, Q, K, V = workload(2, d=128, dv=32)
    check(rule, Q, K, V, 4, 1.0 / np.sqrt(32), "f32")


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_attention_hot_target_over_many_ranges(dtype):
    """One target with 300k tuples: its softmax state is carried across many
    waves' ranges and merged in range order."""
    rule, Q, K, V = workload(3, m=420_000, hot=300_000)
    res = check(rule, Q, K, V, 2, 0.25, dtype)
    assert res["gi"].E > 400_000


def test_attention_keys_and_values_from_one_relation():
    rule, Q, K, V = workload(4, same_kv=True)
    check(rule, Q, K, V, 4, 0.3, "f32", same_kv=True)


def test_attention_query_not_keyed_by_the_group():
    """Q joined on its own column (not the group key): a Q row meets several
    groups, so dQ goes through the gather-sum over Q's rows instead of the
    weights pass."""
    rng = np.random.default_rng(12)
    n_t, n_s, n_q, m, d = 2000, 3000, 500, 80_000, 32
    t = rng.integers(0, n_t, m).astype(np.int32)
    s = rng.integers(0, n_s, m).astype(np.int32)
    x = rng.integers(0, n_q, m).astype(np.int32)
    Q = rng.standard_normal((n_q, d)).astype(np.float32)
    K = rng.standard_normal((n_s, d)).astype(np.float32)
    V = rng.standard_normal((n_s, d)).astype(np.float32)
    import relgen

    rule = relgen.Rule(cols=[t, s, x], atoms=[relgen.Atom(2, Q), relgen.Atom(1, K), relgen.Atom(1, V)],
                       group_col=0, W=np.zeros((1, 1), np.float32), b=np.zeros(1, np.float32))
    for dtype in ("f32", "bf16"):
        check(rule, Q, K, V, 4, 0.35, dtype)


def test_attention_deterministic():
    rule, Q, K, V = workload(5, m=200_000, hot=100_000)
    a = run(rule, Q, K, V, 2, 0.5, "f32")
    b = run(rule, Q, K, V, 2, 0.5, "f32")
    for key in ("out", "lse", "dq", "dk", "dv"):
        np.testing.assert_array_equal(a[key], b[key])


def test_attention_errors():
    from paper_2605_24207_amd import RelnnError, attn_fwd

    rule, Q, K, V = workload(6, m=1000)
    gi = gpu_index(rule)
    q, k, v = dev(Q, "f32"), dev(K, "f32"), dev(V, "f32")
    with pytest.raises(RelnnError, match="INVALID"):           # heads do not divide d
        attn_fwd(gi, q, k, v, 3, 1.0)
    with pytest.raises(RelnnError, match="UNSUPPORTED"):       # head width not a power of two
        attn_fwd(gi, q[:, :48].contiguous(), k[:, :48].contiguous(), v, 4, 1.0)
