"""Pure-Python brute force for tiny inputs.  TEST INFRASTRUCTURE ONLY.

Enumerates every combination of a link row, a row of every further link
relation and a row of every body atom, and keeps those whose keys agree (the
natural join of Section 2.2, written as a nested loop over all row
combinations) and that satisfy every filter predicate (the selection of
Section 3.1), then applies the transform and the multiset aggregate of
Section 2.2 with plain Python floats.  It shares no
code with ``relnn_oracle`` and exists to pin it.
"""
from __future__ import annotations

import itertools


def _key(keys, r):
    return r if keys is None else int(keys[r])


_OPS = {"eq": lambda v: v == 0, "ne": lambda v: v != 0, "lt": lambda v: v < 0, "le": lambda v: v <= 0,
        "gt": lambda v: v > 0, "ge": lambda v: v >= 0}


def _holds(p, cols):
    v = p.add
    if p.a >= 0:
        v += p.mul_a * cols[p.a]
    if p.b >= 0:
        v += p.mul_b * cols[p.b]
    return _OPS[p.op](v)


def _link_tuples(rule):
    """(source rows, columns) of every tuple of the link relation joined with
    the further link relations: a nested loop over all row combinations,
    kept where the join columns agree."""
    base = [[int(v) for v in c] for c in rule.cols]
    cur = [((ell,), [c[ell] for c in base]) for ell in range(len(base[0]))]
    for st in getattr(rule, "steps", ()):
        S = [[int(v) for v in c] for c in st.cols]
        nxt = []
        for src, cols in cur:
            for r in range(len(S[0])):
                if all(cols[o] == S[k][r] for o, k in zip(st.on, st.key)):
                    nxt.append((src + (r,), cols + [c[r] for c in S]))
        cur = nxt
    return cur


def join(rule):
    """List of (source rows, (r_1..r_k), columns) for every joined tuple, in
    source-row order (link row, then the row of each further link relation);
    no index or hashing, a full nested loop."""
    if rule.two_hop_mid >= 0:
        raise NotImplementedError("two-hop paths are pinned separately")
    out = []
    for ell, cols in _link_tuples(rule):
        cols = list(cols)
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
        if not all(_holds(p, cols) for p in getattr(rule, "preds", ())):
            continue
        cand = []
        for a in rule.atoms:
            cand.append([r for r in range(a.n_rows) if _key(a.keys, r) == cols[a.col]])
        for combo in itertools.product(*cand):
            out.append((ell if len(ell) > 1 else ell[0], tuple(combo), tuple(cols)))
    return out


def layer(rule, embs=None, W=None, b=None, tf="linear"):
    """dict head key -> (pre-activation aggregate as a list, output list).
    tf = "product": the transform is the elementwise product of the atoms'
    embedding rows."""
    embs = [a.emb for a in rule.atoms] if embs is None else embs
    W = rule.W if W is None else W
    b = rule.b if b is None else b
    K, h = len(W), len(W[0])
    groups = {}
    for ell, rows, cols in join(rule):
        if tf == "product":
            hp = len(embs[0][rows[0]])
            y = []
            for c in range(hp):
                acc = 1.0
                for e, r in zip(embs, rows):
                    acc *= float(e[r][c])
                y.append(max(acc, 0.0) if rule.act_pre == "relu" else acc)
            groups.setdefault(cols[rule.group_col], []).append(y)
            continue
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


def tuple_values(rule, embs=None, W=None, b=None):
    """(head key, transformed embedding as a list) of every joined tuple of
    the nested loop, in source-row order."""
    embs = [a.emb for a in rule.atoms] if embs is None else embs
    W = rule.W if W is None else W
    b = rule.b if b is None else b
    K, h = len(W), len(W[0])
    out = []
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
        out.append((cols[rule.group_col], y))
    return out


def union_layer(rules, agg, act_post="none", W_post=None, b_post=None):
    """dict head key -> (aggregate, output) of the projected union of the
    rules' joined and transformed tuples: every tuple of every rule with
    the key is one member of the key's multiset, aggregated once."""
    members = {}
    for rule in rules:
        for key, y in tuple_values(rule):
            members.setdefault(key, []).append(y)
    res = {}
    for key, ys in members.items():
        if agg == "sum":
            a = [sum(col) for col in zip(*ys)]
        elif agg == "mean":
            a = [sum(col) / len(ys) for col in zip(*ys)]
        else:
            a = [max(col) for col in zip(*ys)]
        v = list(a)
        if W_post is not None:
            v = [sum(a[i] * float(W_post[i][c]) for i in range(len(a))) + (0.0 if b_post is None else float(b_post[c]))
                 for c in range(len(W_post[0]))]
        o = [max(x, 0.0) for x in v] if act_post == "relu" else v
        res[key] = (a, o)
    return res
