"""Glue between relgen rules, the oracle and the GPU binding (tests only)."""
from __future__ import annotations

import numpy as np

from oracle import relnn_oracle as orc


def gpu_index(rule, bwd=False, device="cuda"):
    import torch

    from paper_2605_24207_amd import Index

    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).to(device)
    cols = [t(c) for c in rule.cols]
    atoms = [(a.n_rows, a.col, None if a.keys is None else t(a.keys)) for a in rule.atoms]
    chains = [(c.src_col, t(c.vals), None if c.keys is None else t(c.keys)) for c in rule.chains]
    two = None if rule.two_hop_mid < 0 else (rule.two_hop_mid, rule.two_hop_cap)
    steps = [([t(c) for c in st.cols], st.on, st.key) for st in rule.steps]
    preds = [(p.a, p.op, p.b, p.mul_a, p.mul_b, p.add) for p in rule.preds]
    return Index(cols, atoms, rule.group_col, chains=chains, two_hop=two, bwd=bwd, steps=steps, preds=preds)


def gpu_layer(rule, dtype="f32", plain=False, pushdown=False):
    from paper_2605_24207_amd import Layer

    return Layer([a.d for a in rule.atoms], rule.h, dtype=dtype, agg=rule.agg, act_pre=rule.act_pre,
                 act_post=rule.act_post, plain=plain, pushdown=pushdown)


def to_dev(a, dtype="f32", device="cuda"):
    import torch

    x = torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(device)
    return x.to(torch.bfloat16) if dtype == "bf16" else x


def distinct_embs(rule, dtype="f32"):
    """Device copies of the atoms' embeddings; atoms sharing one numpy array
    share one device tensor (self-joins)."""
    seen = {}
    out = []
    for a in rule.atoms:
        k = id(a.emb)
        if k not in seen:
            seen[k] = to_dev(a.emb, dtype)
        out.append(seen[k])
    return out


def gpu_fwd(rule, dtype="f32", plain=False, index=None, pushdown=False):
    import torch

    from paper_2605_24207_amd import layer_fwd

    idx = gpu_index(rule) if index is None else index
    layer = gpu_layer(rule, dtype, plain, pushdown)
    embs = distinct_embs(rule, dtype)
    W = to_dev(rule.W, dtype)
    b = to_dev(rule.b)
    out, pre, am = layer_fwd(idx, layer, embs, W, b)
    torch.cuda.synchronize()
    res = {"out": out.cpu().numpy(), "pre": pre.cpu().numpy(),
           "argmax": None if am is None else am.cpu().numpy(), "index": idx}
    return res


def oracle_inputs(rule, dtype="f32"):
    """Embeddings, W and b as the oracle sees them: the FP32 master values,
    or their bf16 roundings for the kernel-arithmetic check."""
    r = (lambda a: orc.bf16_round(a)) if dtype == "bf16" else (lambda a: a)
    return [r(a.emb) for a in rule.atoms], r(rule.W), rule.b


def oracle_fwd(rule, dtype="f32", groups=None, idx=None):
    idx = orc.build_index(rule) if idx is None else idx
    embs, W, b = oracle_inputs(rule, dtype)
    out, pre, am = orc.layer_fwd(idx, embs, W, b, rule.agg, rule.act_pre, rule.act_post, groups)
    return idx, out, pre, am


def elem_scale(rule, idx, dtype="f32", chunk=8192):
    """Per group and column, the condition scale of the aggregate: the
    aggregate over the group's tuples (SUM: sum, MEAN: mean, MAX: max) of
    |x| |W| + |b|, the sum of the magnitudes of the terms of each tuple's
    value.  A rounding error of relative size u in every product and sum
    moves an output element by at most about u times this, cancellation
    included, so element-wise bounds are stated against it."""
    embs, W, b = oracle_inputs(rule, dtype)
    aW = np.abs(np.asarray(W, np.float64))
    ab = np.abs(np.asarray(b, np.float64))
    t = np.empty((idx.E, aW.shape[1]))
    for s in range(0, idx.E, chunk):
        e = min(idx.E, s + chunk)
        t[s:e] = np.abs(orc.gather_concat(idx, embs, slice(s, e))) @ aW + ab
    if idx.E == 0:
        return np.zeros((0, aW.shape[1]))
    starts = np.asarray(idx.offsets[:-1], np.int64)
    if rule.agg == "max":
        return np.maximum.reduceat(t, starts, axis=0)
    agg = np.add.reduceat(t, starts, axis=0)
    if rule.agg == "mean":
        agg /= np.diff(idx.offsets)[:, None]
    return agg


def elem_err(z, ref, scale):
    """Largest |z - ref| / scale over the elements (scale from elem_scale)."""
    z = np.asarray(z, np.float64)
    return float((np.abs(z - np.asarray(ref, np.float64)) / np.maximum(scale, 1e-30)).max(initial=0.0))


def rel_rows(z, ref, scale_ref=None):
    z = np.asarray(z, np.float64)
    ref = np.asarray(ref, np.float64)
    den = np.linalg.norm(ref if scale_ref is None else np.asarray(scale_ref, np.float64), axis=-1)
    den = np.maximum(den, 1e-30)
    return np.linalg.norm(z - ref, axis=-1) / den


def check_argmax(am_gpu, am_ref, pre_ref, y_of_pos, tol):
    """MAX: where the oracle's maximiser is unique beyond ``tol`` the
    positions must agree; elsewhere the GPU's choice must be a valid
    maximiser within ``tol``.  y_of_pos(pos, col) -> oracle value."""
    bad = 0
    G, h = am_ref.shape
    for g in range(G):
        for c in range(h):
            if am_gpu[g, c] == am_ref[g, c]:
                continue
            v = y_of_pos(am_gpu[g, c], c)
            if abs(v - pre_ref[g, c]) > tol * max(1.0, abs(pre_ref[g, c])):
                bad += 1
    return bad
