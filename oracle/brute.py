"""Pure-Python brute force for tiny inputs.  TEST INFRASTRUCTURE ONLY.

Enumerates every combination of a link row with one row of every body atom
and keeps those whose keys agree (the natural join of Section 2.2, written as
a nested loop over all row combinations), then applies the transform and the
multiset aggregate of Section 2.2 with plain Python floats.  It shares no
code with ``relnn_oracle`` and exists to pin it.
"""
from __future__ import annotations

import itertools


def _key(keys, r):
    return r if keys is None else int(keys[r])


def join(rule):
    """List of (link_row, (r_1..r_k), columns) for every joined tuple, in
    link-row order; no index or hashing, a full nested loop."""
    base = [[int(v) for v in c] for c in rule.cols]
    n_link = len(base[0])
    if rule.two_hop_mid >= 0:
        raise NotImplementedError("use join_two_hop")
    out = []
    for ell in range(n_link):
        cols = [c[ell] for c in base]
        ok = True
        for ch in rule.chains:
            hits = [r for r in range(ch.n_rows) if _key(ch.keys, r) == cols[ch.src_col]]
            if not hits:
                ok = False
                cols.append(None)
            else:
                cols.append(int(ch.vals[hits[0]]))
        if not ok:
            continue
        cand = []
        for a in rule.atoms:
            cand.append([r for r in range(a.n_rows) if _key(a.keys, r) == cols[a.col]])
        for combo in itertools.product(*cand):
            out.append((ell, tuple(combo), tuple(cols)))
    return out


def layer(rule, embs=None, W=None, b=None):
    """dict head key -> (pre-activation aggregate as a list, output list)."""
    embs = [a.emb for a in rule.atoms] if embs is None else embs
    W = rule.W if W is None else W
    b = rule.b if b is None else b
    K, h = len(W), len(W[0])
    groups = {}
    for ell, rows, cols in join(rule):
        x = []
        for e, r in zip(embs, rows):
            x.extend(float(v) for v in e[r])
        y = []
        for c in range(h):
            acc = float(b[c])
            for q in range(K):
                acc += x[q] * float(W[q][c])
            if rule.act_pre == "relu":
                acc = max(acc, 0.0)
            y.append(acc)
        groups.setdefault(cols[rule.group_col], []).append(y)
    res = {}
    for g, ys in groups.items():
        if rule.agg == "sum":
            a = [sum(col) for col in zip(*ys)]
        elif rule.agg == "mean":
            a = [sum(col) / len(ys) for col in zip(*ys)]
        else:
            a = [max(col) for col in zip(*ys)]
        o = [max(v, 0.0) for v in a] if rule.act_post == "relu" else list(a)
        res[g] = (a, o)
    return res
