"""Pins of the oracle's segmented softmax attention (CPU only).

Attention as rules (Section 1's Score / Attention example, Section 5.2's
HGT head): a score per joined tuple and head from the product q*k summed
over the head's features, a softmax over the tuples of each group, and the
weighted sum of values sum(a*v).  Pinned by a hand-worked example
(tests/golden/attention_tiny.json), by the invariance of softmax to a shift
of all scores of a group, by special cases (a one-tuple group returns its
value, a zero scale averages the values), by torch's own softmax and
autograd in FP64 on the CPU, and by central finite differences.
"""
import json
import os

import numpy as np
import pytest

import relgen
from oracle import relnn_oracle as orc

GOLD = os.path.join(os.path.dirname(__file__), "golden", "attention_tiny.json")


def attn_rule(t, s, Q, K, V):
    """Link (t, s); atoms Q on t, K on s, V on s; grouped by t."""
    t = np.asarray(t, np.int32)
    s = np.asarray(s, np.int32)
    return relgen.Rule(cols=[t, s], atoms=[relgen.Atom(0, np.asarray(Q, np.float32)),
                                           relgen.Atom(1, np.asarray(K, np.float32)),
                                           relgen.Atom(1, np.asarray(V, np.float32))],
                       group_col=0, W=np.zeros((1, 1), np.float32), b=np.zeros(1, np.float32))


def golden():
    with open(GOLD) as f:
        g = json.load(f)
    rule = attn_rule(g["link_t"], g["link_s"], g["Q"], g["K"], g["V"])
    return g, orc.build_index(rule), np.array(g["Q"]), np.array(g["K"]), np.array(g["V"])


def test_golden_forward():
    g, idx, Q, K, V = golden()
    for heads, key in ((1, "heads1"), (2, "heads2")):
        out, lse = orc.attention_fwd(idx, Q, K, V, heads, 1.0)
        np.testing.assert_allclose(out, g[key]["out"], rtol=0, atol=1e-14)
        np.testing.assert_allclose(lse, g[key]["lse"], rtol=0, atol=1e-14)


def test_golden_backward():
    g, idx, Q, K, V = golden()
    dq, dk, dv = orc.attention_bwd(idx, Q, K, V, 1, 1.0, np.array(g["heads1"]["dout"]))
    np.testing.assert_allclose(dq, g["heads1"]["dQ"], rtol=0, atol=1e-14)
    np.testing.assert_allclose(dk, g["heads1"]["dK"], rtol=0, atol=1e-14)
    np.testing.assert_allclose(dv, g["heads1"]["dV"], rtol=0, atol=1e-14)


def random_attn(seed, n_t=30, n_s=40, m=300, d=8, dv=6, heads=2, hot=None):
    """Groups of about m / (n_t - 3) tuples, the last three with one tuple each."""
    rng = np.random.default_rng(seed)
    t = np.concatenate([rng.integers(0, n_t - 3, m - 3), np.arange(n_t - 3, n_t)])
    s = rng.integers(0, n_s, m)
    if hot is not None:
        t[:hot] = 3
    Q = rng.standard_normal((n_t, d))
    K = rng.standard_normal((n_s, d))
    V = rng.standard_normal((n_s, dv))
    return attn_rule(t, s, Q, K, V), Q, K, V


def test_shift_invariance():
    """Moving every key by the same vector delta adds scale <q_h, delta_h> to
    every score of a group and head: the softmax, hence the output, does not
    change; lse moves by exactly that amount."""
    rule, Q, K, V = random_attn(1)
    idx = orc.build_index(rule)
    out, lse = orc.attention_fwd(idx, Q, K, V, 2, 0.7)
    delta = np.random.default_rng(2).standard_normal(8)
    out2, lse2 = orc.attention_fwd(idx, Q, K + delta, V, 2, 0.7)
    np.testing.assert_allclose(out2, out, rtol=1e-12, atol=1e-12)
    qd = 0.7 * (Q[idx.group_keys] * delta).reshape(-1, 2, 4).sum(axis=2)
    np.testing.assert_allclose(lse2, lse + qd, rtol=1e-12, atol=1e-12)


def test_special_cases():
    rule, Q, K, V = random_attn(3)
    idx = orc.build_index(rule)
    out, lse = orc.attention_fwd(idx, Q, K, V, 2, 0.0)          # scale 0: uniform weights, the mean
    for g in range(idx.G):
        s0, e0 = idx.offsets[g], idx.offsets[g + 1]
        np.testing.assert_allclose(out[g], V[idx.rows[2][s0:e0]].mean(axis=0), rtol=1e-12)
        np.testing.assert_allclose(lse[g], np.log(e0 - s0), rtol=1e-12)
    one = [g for g in range(idx.G) if idx.offsets[g + 1] - idx.offsets[g] == 1]
    out, lse = orc.attention_fwd(idx, Q, K, V, 2, 1.3)
    assert one
    for g in one:                                              # one tuple: weight 1, its value
        np.testing.assert_allclose(out[g], V[idx.rows[2][idx.offsets[g]]], rtol=1e-14)


def torch_attention(idx, Q, K, V, heads, scale):
    """The same computation written with torch's softmax on FP64 CPU
    tensors, one group at a time (a library special case)."""
    import torch

    outs = []
    for g in range(idx.G):
        s0, e0 = int(idx.offsets[g]), int(idx.offsets[g + 1])
        rq = torch.from_numpy(np.asarray(idx.rows[0][s0:e0]))
        rk = torch.from_numpy(np.asarray(idx.rows[1][s0:e0]))
        rv = torch.from_numpy(np.asarray(idx.rows[2][s0:e0]))
        n = e0 - s0
        S = scale * (Q[rq] * K[rk]).reshape(n, heads, -1).sum(dim=2)
        a = torch.softmax(S, dim=0)
        outs.append((a[:, :, None] * V[rv].reshape(n, heads, -1)).sum(dim=0).reshape(-1))
    return torch.stack(outs)


def test_matches_torch_softmax_and_autograd():
    import torch

    rule, Q, K, V = random_attn(4, hot=60)
    idx = orc.build_index(rule)
    out, lse = orc.attention_fwd(idx, Q, K, V, 2, 0.8)
    tQ, tK, tV = (torch.tensor(a, dtype=torch.float64, requires_grad=True) for a in (Q, K, V))
    ref = torch_attention(idx, tQ, tK, tV, 2, 0.8)
    np.testing.assert_allclose(out, ref.detach().numpy(), rtol=1e-12, atol=1e-12)
    dout = np.random.default_rng(5).standard_normal(out.shape)
    (ref * torch.from_numpy(dout)).sum().backward()
    dq, dk, dv = orc.attention_bwd(idx, Q, K, V, 2, 0.8, dout)
    np.testing.assert_allclose(dq, tQ.grad.numpy(), rtol=1e-11, atol=1e-11)
    np.testing.assert_allclose(dk, tK.grad.numpy(), rtol=1e-11, atol=1e-11)
    np.testing.assert_allclose(dv, tV.grad.numpy(), rtol=1e-11, atol=1e-11)


def test_finite_differences():
    rule, Q, K, V = random_attn(6, m=120)
    idx = orc.build_index(rule)
    dout = np.random.default_rng(7).standard_normal((idx.G, 6))
    grads = orc.attention_bwd(idx, Q, K, V, 2, 0.9, dout)
    rng = np.random.default_rng(8)
    eps = 1e-6
    for arr, gr in zip((Q, K, V), grads):
        for _ in range(6):
            pos = tuple(int(rng.integers(0, n)) for n in arr.shape)
            old = arr[pos]
            arr[pos] = old + eps
            lp = float((orc.attention_fwd(idx, Q, K, V, 2, 0.9)[0] * dout).sum())
            arr[pos] = old - eps
            lm = float((orc.attention_fwd(idx, Q, K, V, 2, 0.9)[0] * dout).sum())
            arr[pos] = old
            assert abs((lp - lm) / (2 * eps) - gr[pos]) <= 1e-6 * max(1.0, abs(gr[pos]))
