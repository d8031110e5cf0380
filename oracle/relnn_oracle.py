"""FP64 CPU oracle for one relational layer.  TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module.  The HIP library never calls it and
shares no code with it; the two meet only at the seeded inputs of ``relgen``.

What it computes, and where the paper defines it:

* join (Section 2.2, "Join"): natural join of the link relation (and of
  further link relations joined on shared columns: many-to-many and cyclic
  joins) with each body atom on the atom's key; the embedding of a joined
  tuple is the concatenation of the contributing embeddings in body-atom
  order;
* selection (Section 2.2 "Other operators", Section 3.1 filter expression):
  the joined tuples that satisfy the conjunction of the filter predicates;
* transformation (Section 2.2, "Transformation"): tau applied independently
  to every joined tuple, here tau = act_pre(Linear(Concat(...)));
* projected union with k = 1 (Section 2.2, "Projected union"): the output
  content is the *set* of distinct head keys; each output tuple aggregates
  the *multiset* B_t of joined tuples that project onto it, with
  alpha in {sum, mean, max}, applied once;
* the join rule (Section 3.1) composes these as union(T(join(...))); an
  activation after the aggregate follows the union-rule form, where T comes
  after the union (Section 3.1);
* training (Section 2.3) needs gradients with respect to both the
  per-tuple embeddings and the transform weights: ``layer_bwd``.

Readings where the paper is silent (each is listed with its reason in the
design notes of the repository): bag semantics for link rows; absent output
for empty groups; canonical tuple order (group key, FK values of the atoms
in body order, link row); MAX ties go to the earliest canonical tuple and
its gradient goes only there; ReLU'(0) = 0; W is [K, h] with y = x W + b.

Parity is pinned by tests/test_oracle_pins.py: brute-force enumeration,
dense closed forms, a hand-worked golden example, permutation invariance,
finite differences and a torch-CPU FP64 composition of the paper's physical
plan (Section 4.2).  The two-hop path cap and the neighbourhood sampler are
readings of ours with no counterpart in the paper: "parity unpinned" by the
paper, pinned only by brute force and by their own invariants.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np


class NotUnique(ValueError):
    """A keyed atom has a duplicate primary key (FK -> PK join required)."""


# ---------------------------------------------------------------------------
# join
# ---------------------------------------------------------------------------
def lookup_rows(n_rows: int, keys: Optional[np.ndarray], values: np.ndarray) -> np.ndarray:
    """Row of the relation whose key equals each value; -1 if none (a
    dangling foreign key, which drops the joined tuple: inner join)."""
    values = np.asarray(values, dtype=np.int64)
    if keys is None:
        ok = (values >= 0) & (values < n_rows)
        return np.where(ok, values, -1)
    pos = {}
    for r, k in enumerate(np.asarray(keys).tolist()):
        if k in pos:
            raise NotUnique(f"duplicate key {k}")
        pos[k] = r
    return np.array([pos.get(v, -1) for v in values.tolist()], dtype=np.int64)


def two_hop_paths(cols: Sequence[np.ndarray], mid: int, cap: int):
    """Self-join of the link relation on column ``mid`` (Buys |x| Buys^T).

    For every mid key m (ascending) the link rows with that key are ordered
    by their other columns, then by link row: B_m = [b_0 .. b_{n-1}].  Path
    number p (0 <= p < min(cap, n*n)) pairs b_i with b_j where
    i = p mod n and j = (i + 1 + p div n) mod n, which walks all n*n ordered
    pairs, starting with each row's successor.  Returns the two link-row
    arrays, in path order."""
    n_link = len(cols[0])
    others = [np.asarray(c, np.int64) for q, c in enumerate(cols) if q != mid]
    order = np.lexsort([np.arange(n_link)] + others[::-1] + [np.asarray(cols[mid], np.int64)])
    midv = np.asarray(cols[mid], np.int64)[order]
    la, lb = [], []
    start = 0
    while start < n_link:
        end = start
        while end < n_link and midv[end] == midv[start]:
            end += 1
        n = end - start
        for p in range(min(cap, n * n)):
            i = p % n
            j = (i + 1 + p // n) % n
            la.append(order[start + i])
            lb.append(order[start + j])
        start = end
    return np.array(la, np.int64), np.array(lb, np.int64)


def join_step(cols: List[np.ndarray], step) -> List[np.ndarray]:
    """Natural join of the tuples so far with a further link relation S (the
    join of Section 2.2 applied once more, bag semantics): every pair of a
    tuple and a row r of S with cols[on[q]] == S.cols[key[q]][r] for all q
    is a tuple.  The result has the columns so far followed by those of S,
    ordered by (position so far, row of S).  Many-to-many and cyclic joins
    (a column pair that closes a cycle) are both this step."""
    S = [np.asarray(c, np.int64) for c in step.cols]
    rows_of = {}
    for r in range(step.n_rows):                 # an index nested loop: key -> rows of S
        rows_of.setdefault(tuple(int(S[k][r]) for k in step.key), []).append(r)
    src, srow = [], []
    for i in range(len(cols[0]) if cols else 0):
        for r in rows_of.get(tuple(int(cols[o][i]) for o in step.on), ()):
            src.append(i)
            srow.append(r)
    src = np.array(src, np.int64)
    srow = np.array(srow, np.int64)
    return [c[src] for c in cols] + [c[srow] for c in S]


_CMP = {"eq": np.equal, "ne": np.not_equal, "lt": np.less, "le": np.less_equal,
        "gt": np.greater, "ge": np.greater_equal}


def selection(cols: List[np.ndarray], preds) -> np.ndarray:
    """The selection of a filter expression (Section 3.1): the conjunction of
    its atomic predicates e1 theta e2, each written as mul_a * col[a] +
    mul_b * col[b] + add theta 0 in integer arithmetic."""
    n = len(cols[0]) if cols else 0
    keep = np.ones(n, dtype=bool)
    for p in preds:
        v = np.full(n, p.add, np.int64)
        if p.a >= 0:
            v = v + p.mul_a * np.asarray(cols[p.a], np.int64)
        if p.b >= 0:
            v = v + p.mul_b * np.asarray(cols[p.b], np.int64)
        keep &= _CMP[p.op](v, 0)
    return keep


@dataclass
class Index:
    """Join result in canonical order plus the group structure."""
    link_row: np.ndarray      # [E] link row (or path number) of each tuple
    rows: List[np.ndarray]    # k x [E] row of atom j joined to each tuple
    gkey: np.ndarray          # [E] head key of each tuple
    group_keys: np.ndarray    # [G] distinct head keys, ascending
    offsets: np.ndarray       # [G+1] segment bounds in the tuple list
    tuple_group: np.ndarray   # [E] segment number of each tuple

    @property
    def E(self) -> int:
        return int(self.link_row.shape[0])

    @property
    def G(self) -> int:
        return int(self.group_keys.shape[0])


def build_index(rule) -> Index:
    """Join the link relation with the body atoms and group by the head key."""
    cols = [np.asarray(c, np.int64) for c in rule.cols]
    if rule.two_hop_mid >= 0:
        la, lb = two_hop_paths(rule.cols, rule.two_hop_mid, rule.two_hop_cap)
        cols = [c[la] for c in cols] + [c[lb] for c in cols]
    for st in getattr(rule, "steps", ()):        # further link relations, in order
        cols = join_step(cols, st)
    n_link = len(cols[0])
    valid = np.ones(n_link, dtype=bool)
    for ch in rule.chains:                       # derived columns, in order
        r = lookup_rows(ch.n_rows, ch.keys, cols[ch.src_col])
        valid &= r >= 0
        cols.append(np.where(r >= 0, np.asarray(ch.vals, np.int64)[np.maximum(r, 0)], 0))
    valid &= selection(cols, getattr(rule, "preds", ()))
    rows = []
    for a in rule.atoms:
        r = lookup_rows(a.n_rows, a.keys, cols[a.col])
        valid &= r >= 0
        rows.append(r)
    ell = np.nonzero(valid)[0]
    g = cols[rule.group_col][ell]
    fk = [cols[a.col][ell] for a in rule.atoms]
    # canonical order: head key, then FK values of the atoms, then link row
    order = np.lexsort([ell] + fk[::-1] + [g])
    ell, g = ell[order], g[order]
    rows = [r[ell] for r in rows]
    head = np.ones(len(ell), dtype=bool)
    head[1:] = g[1:] != g[:-1]
    starts = np.nonzero(head)[0]
    offsets = np.append(starts, len(ell)).astype(np.int64)
    tuple_group = np.cumsum(head) - 1
    return Index(link_row=ell, rows=rows, gkey=g, group_keys=g[starts],
                 offsets=offsets, tuple_group=tuple_group)


# ---------------------------------------------------------------------------
# transform + aggregate
# ---------------------------------------------------------------------------
def bf16_round(x: np.ndarray) -> np.ndarray:
    """float32 -> bfloat16 (round to nearest, ties to even), returned as the
    float32 value it represents; infinities and the quiet NaN are kept."""
    b = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lsb = (b >> 16) & 1
    b = (b + 0x7FFF + lsb) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32)


def _act(name: str, v: np.ndarray) -> np.ndarray:
    if name == "none":
        return v
    if name == "relu":
        return np.maximum(v, 0.0)
    raise ValueError(name)


def _act_grad(name: str, v: np.ndarray) -> np.ndarray:
    if name == "none":
        return np.ones_like(v)
    if name == "relu":
        return (v > 0).astype(np.float64)          # ReLU'(0) = 0
    raise ValueError(name)


def gather_concat(idx: Index, embs: Sequence[np.ndarray], sel=slice(None)) -> np.ndarray:
    """x_tau = z_1[r_1] (+) ... (+) z_k[r_k] in body-atom order, FP64."""
    parts = [np.asarray(e)[r[sel]].astype(np.float64) for e, r in zip(embs, idx.rows)]
    return np.concatenate(parts, axis=1)


def act_pre_mask(idx: Index, embs, W, b) -> np.ndarray:
    """[E, h] decisions x W + b > 0 of every joined tuple (ReLU'(0) = 0)."""
    return gather_concat(idx, embs) @ np.asarray(W, np.float64) + np.asarray(b, np.float64) > 0


def transform(x: np.ndarray, W: np.ndarray, b: np.ndarray, act_pre: str) -> np.ndarray:
    return _act(act_pre, x @ np.asarray(W, np.float64) + np.asarray(b, np.float64))


def _groups(idx: Index, groups):
    return np.arange(idx.G) if groups is None else np.asarray(groups, np.int64)


def product(idx: Index, embs, sel, act_pre: str) -> np.ndarray:
    """The product transform: act_pre(z_1[r_1] * ... * z_k[r_k]), elementwise
    (the Score rule's q*k and the Attention rule's a*v of Section 1, the
    gated mean z_e*z_w of Section 5.4); all atoms have the output width."""
    y = np.asarray(embs[0])[idx.rows[0][sel]].astype(np.float64)
    for e, r in zip(embs[1:], idx.rows[1:]):
        y = y * np.asarray(e)[r[sel]].astype(np.float64)
    return _act(act_pre, y)


def layer_fwd(idx: Index, embs, W, b, agg="sum", act_pre="none", act_post="none",
              groups=None, tf="linear"):
    """Evaluate the layer for all groups (or the listed group numbers).

    Returns (out, pre, argmax): out = act_post(pre); pre = alpha over the
    group's tuples of act_pre(x W + b) (tf = "product": of the product
    transform, W and b unused); argmax [G', h] is the canonical tuple
    position of the first maximiser (MAX only, else None)."""
    gsel = _groups(idx, groups)
    h = np.asarray(embs[0]).shape[1] if tf == "product" else W.shape[1]
    pre = np.zeros((len(gsel), h), np.float64)
    amax = np.full((len(gsel), h), -1, np.int64) if agg == "max" else None
    for q, g in enumerate(gsel):
        s, e = int(idx.offsets[g]), int(idx.offsets[g + 1])
        if tf == "product":
            y = product(idx, embs, slice(s, e), act_pre)
        else:
            y = transform(gather_concat(idx, embs, slice(s, e)), W, b, act_pre)
        if agg == "sum":
            pre[q] = y.sum(axis=0)
        elif agg == "mean":
            pre[q] = y.sum(axis=0) / (e - s)
        elif agg == "max":
            j = np.argmax(y, axis=0)                 # first maximiser
            pre[q] = y[j, np.arange(h)]
            amax[q] = s + j
        else:
            raise ValueError(agg)
    return _act(act_post, pre), pre, amax


def layer_bwd(idx: Index, embs, W, b, pre, argmax, dout, agg="sum",
              act_pre="none", act_post="none", pre_mask=None):
    """Gradients of sum(out * dout) with respect to every atom's embedding,
    W and b (chain rule through the layer of ``layer_fwd``).

    ``pre_mask`` ([E, h] booleans, optional) gives the per-tuple decisions
    act_pre'(x W + b) > 0 when they were taken in another precision (the
    kernel's); by default they are computed here.  Returns (demb, dW, db);
    demb[j] has the shape of embs[j].  Atoms that share one embedding
    relation (self-joins) get separate entries, which the caller adds."""
    W64 = np.asarray(W, np.float64)
    dA = np.asarray(dout, np.float64) * _act_grad(act_post, np.asarray(pre, np.float64))
    x = gather_concat(idx, embs)
    g = idx.tuple_group
    cnt = np.diff(idx.offsets).astype(np.float64)
    if agg == "sum":
        dY = dA[g]
    elif agg == "mean":
        dY = dA[g] / cnt[g][:, None]
    elif agg == "max":
        pos = np.arange(idx.E)[:, None]
        dY = np.where(np.asarray(argmax)[g] == pos, dA[g], 0.0)
    else:
        raise ValueError(agg)
    if act_pre != "none":
        if pre_mask is not None:
            dY = dY * np.asarray(pre_mask, np.float64)
        else:
            dY = dY * _act_grad(act_pre, x @ W64 + np.asarray(b, np.float64))
    dW = x.T @ dY
    db = dY.sum(axis=0)
    dX = dY @ W64.T
    demb, off = [], 0
    for e, r in zip(embs, idx.rows):
        d = e.shape[1]
        acc = np.zeros(e.shape, np.float64)
        np.add.at(acc, r, dX[:, off:off + d])
        demb.append(acc)
        off += d
    return demb, dW, db


def product_bwd(idx: Index, embs, pre, argmax, dout, agg="sum", act_pre="none", act_post="none",
                pre_mask=None):
    """Gradients of sum(out * dout) through the product transform of
    ``layer_fwd(tf="product")`` with respect to every atom's embedding (the
    transform has no weights).  With y = act_pre(z_1 * ... * z_k) per tuple
    and dY the gradient reaching y (routed as in ``layer_bwd``), the
    gradient of atom j's row is dY * act_pre'(z_1 * ... * z_k) times the
    product of the other atoms' rows, summed over the tuples that join it.
    ``pre_mask`` ([E, h] booleans) gives act_pre' taken in another
    precision.  Returns demb (one entry per atom, shaped as embs[j])."""
    dA = np.asarray(dout, np.float64) * _act_grad(act_post, np.asarray(pre, np.float64))
    g = idx.tuple_group
    cnt = np.diff(idx.offsets).astype(np.float64)
    if agg == "sum":
        dY = dA[g]
    elif agg == "mean":
        dY = dA[g] / cnt[g][:, None]
    elif agg == "max":
        pos = np.arange(idx.E)[:, None]
        dY = np.where(np.asarray(argmax)[g] == pos, dA[g], 0.0)
    else:
        raise ValueError(agg)
    Z = [np.asarray(e, np.float64)[r] for e, r in zip(embs, idx.rows)]
    if act_pre != "none":
        if pre_mask is not None:
            dY = dY * np.asarray(pre_mask, np.float64)
        else:
            full = Z[0].copy()
            for z in Z[1:]:
                full = full * z
            dY = dY * _act_grad(act_pre, full)
    demb = []
    for j, (e, r) in enumerate(zip(embs, idx.rows)):
        others = np.ones_like(dY)
        for i, z in enumerate(Z):
            if i != j:
                others = others * z
        acc = np.zeros(np.asarray(e).shape, np.float64)
        np.add.at(acc, r, dY * others)
        demb.append(acc)
    return demb


# ---------------------------------------------------------------------------
# k-ary projected union (Section 2.2) and union rules (Section 3.1)
# ---------------------------------------------------------------------------
def union_fwd(branches, agg="sum", act_post="none", W_post=None, b_post=None):
    """The projected union over k branches with one aggregate applied once.

    ``branches`` is a list of (idx, embs, W, b, act_pre): the join result of
    one rule (its index) and the transform tau_i of that rule.  The output
    content is the set of head keys that occur in any branch (ascending);
    the multiset B_t of a key t holds every tuple of every branch with that
    key, each with its own branch's transformed embedding tau_i(x); alpha is
    applied once over all of B_t (MEAN = sum over B_t / |B_t|, not a mean of
    the branches' means).  For MAX the maximiser is the first one in the
    order (branch, canonical position in the branch).

    A union rule (Section 3.1) applies its transform after the union:
    ``W_post`` [h, h2] and ``b_post`` give tau(v) = v W_post + b_post on the
    aggregate, then act_post.  Returns (keys, out, pre, arg) with pre the
    aggregate (before tau_post and act_post) and arg [G, h] pairs (branch,
    position) for MAX, else None."""
    keys = sorted(set().union(*[set(int(k) for k in b[0].group_keys) for b in branches]))
    h = np.asarray(branches[0][2]).shape[1]
    pre = np.zeros((len(keys), h))
    arg = np.full((len(keys), h, 2), -1, np.int64) if agg == "max" else None
    for q, key in enumerate(keys):
        ys, origin = [], []
        for bi, (idx, embs, W, b, act_pre) in enumerate(branches):
            g = np.searchsorted(idx.group_keys, key)
            if g < idx.G and idx.group_keys[g] == key:
                s, e = int(idx.offsets[g]), int(idx.offsets[g + 1])
                ys.append(transform(gather_concat(idx, embs, slice(s, e)), W, b, act_pre))
                origin += [(bi, p) for p in range(s, e)]
        y = np.concatenate(ys, axis=0)
        if agg == "sum":
            pre[q] = y.sum(axis=0)
        elif agg == "mean":
            pre[q] = y.sum(axis=0) / y.shape[0]
        elif agg == "max":
            j = np.argmax(y, axis=0)                 # first maximiser in (branch, position) order
            pre[q] = y[j, np.arange(h)]
            arg[q] = np.array([origin[i] for i in j])
        else:
            raise ValueError(agg)
    v = pre if W_post is None else pre @ np.asarray(W_post, np.float64) + (
        0.0 if b_post is None else np.asarray(b_post, np.float64))
    return np.array(keys, np.int64), _act(act_post, v), pre, arg


def union_bwd(branches, pre, arg, dout, agg="sum", act_post="none", W_post=None, b_post=None, pre_masks=None,
              post_mask=None):
    """Gradients of sum(out * dout) through ``union_fwd`` (chain rule, from
    the output back to every branch's weights and embeddings).

    With v = pre the aggregate of key t, u = v W_post + b_post (u = v
    without W_post) and out = act_post(u): dU = dout * act_post'(u),
    dW_post = v^T dU, db_post = sum_t dU[t], dV = dU W_post^T.  A tuple of
    branch i at canonical position p with key t then receives dV[t] (SUM),
    dV[t] / |B_t| (MEAN, |B_t| the members of t over all branches), or, for
    MAX, column c of dV[t] when arg[t, c] == (i, p) and 0 otherwise.  From
    there the gradient runs through branch i's transform as in
    ``layer_bwd``.  ``pre_masks`` (one [E_i, h] boolean array per branch,
    or None) gives act_pre' taken in another precision, ``post_mask``
    ([G, h_out] booleans) act_post'(u) likewise.  Returns (grads,
    dW_post, db_post): grads[i] = (demb_i, dW_i, db_i), demb_i one entry
    per atom (atoms or branches sharing a relation get separate entries,
    which the caller adds); dW_post and db_post are None without W_post."""
    keys = np.array(sorted(set().union(*[set(int(k) for k in b[0].group_keys) for b in branches])), np.int64)
    v = np.asarray(pre, np.float64)
    dout = np.asarray(dout, np.float64)
    if W_post is None:
        dV = dout * _act_grad(act_post, v)
        dW_post = db_post = None
    else:
        Wp = np.asarray(W_post, np.float64)
        u = v @ Wp + (0.0 if b_post is None else np.asarray(b_post, np.float64))
        dU = dout * (_act_grad(act_post, u) if post_mask is None or act_post == "none"
                     else np.asarray(post_mask, np.float64))
        dW_post = v.T @ dU
        db_post = dU.sum(axis=0)
        dV = dU @ Wp.T
    members = np.zeros(len(keys))
    for idx, *_ in branches:
        members[np.searchsorted(keys, idx.group_keys)] += np.diff(idx.offsets)
    grads = []
    for bi, (idx, embs, W, b, act_pre) in enumerate(branches):
        t = np.searchsorted(keys, idx.gkey)              # union row of each tuple
        if agg == "sum":
            dY = dV[t]
        elif agg == "mean":
            dY = dV[t] / members[t][:, None]
        elif agg == "max":
            a = np.asarray(arg)[t]
            mine = (a[..., 0] == bi) & (a[..., 1] == np.arange(idx.E)[:, None])
            dY = np.where(mine, dV[t], 0.0)
        else:
            raise ValueError(agg)
        W64 = np.asarray(W, np.float64)
        x = gather_concat(idx, embs)
        if act_pre != "none":
            if pre_masks is not None and pre_masks[bi] is not None:
                dY = dY * np.asarray(pre_masks[bi], np.float64)
            else:
                dY = dY * _act_grad(act_pre, x @ W64 + (0.0 if b is None else np.asarray(b, np.float64)))
        dX = dY @ W64.T
        demb, off = [], 0
        for e, r in zip(embs, idx.rows):
            d = np.asarray(e).shape[1]
            acc = np.zeros(np.asarray(e).shape, np.float64)
            np.add.at(acc, r, dX[:, off:off + d])
            demb.append(acc)
            off += d
        grads.append((demb, x.T @ dY, dY.sum(axis=0)))
    return grads, dW_post, db_post


# ---------------------------------------------------------------------------
# product transforms and segmented softmax (Section 1's attention example,
# Section 5.2's HGT head)
# ---------------------------------------------------------------------------
def _head_scores(qr, kr, heads, scale):
    """scale * <q_h, k_h> per head: the product transform q*k of the paper's
    Score rule, summed over each head's features.  [n, heads]."""
    n, d = kr.shape
    return scale * (qr * kr).reshape(n, heads, d // heads).sum(axis=2)


def attention_fwd(idx: Index, q, k, v, heads: int, scale: float):
    """Segmented softmax attention over the joined tuples of an index whose
    three body atoms are (Q, K, V): for every group g and head h, the score
    of tuple tau is s = scale <q_h[r_Q(tau)], k_h[r_K(tau)]>, the attention
    weight is the softmax of s over the tuples of g (the maximum subtracted
    before the exponential), and the output is sum_tau a_tau v_h[r_V(tau)]
    (the Attention rule's sum(a*v)).  Returns (out [G, dv], lse [G, heads]),
    lse the log of the sum of exponentials of the group's scores."""
    q, k, v = (np.asarray(a, np.float64) for a in (q, k, v))
    dv = v.shape[1]
    out = np.zeros((idx.G, dv))
    lse = np.zeros((idx.G, heads))
    for g in range(idx.G):
        s0, e0 = int(idx.offsets[g]), int(idx.offsets[g + 1])
        S = _head_scores(q[idx.rows[0][s0:e0]], k[idx.rows[1][s0:e0]], heads, scale)
        m = S.max(axis=0)
        ex = np.exp(S - m)
        l = ex.sum(axis=0)
        a = ex / l
        V = v[idx.rows[2][s0:e0]].reshape(e0 - s0, heads, dv // heads)
        out[g] = (a[:, :, None] * V).sum(axis=0).reshape(dv)
        lse[g] = m + np.log(l)
    return out, lse


def attention_bwd(idx: Index, q, k, v, heads: int, scale: float, dout):
    """Gradients of sum(out * dout) through attention_fwd with respect to the
    Q, K and V relations' embeddings (chain rule through the softmax: ds =
    a (dp - sum_tau a dp), dp = <dout_h, v_h>)."""
    q, k, v, dout = (np.asarray(a, np.float64) for a in (q, k, v, dout))
    d, dv = k.shape[1], v.shape[1]
    dq, dk, dvv = np.zeros_like(q), np.zeros_like(k), np.zeros_like(v)
    for g in range(idx.G):
        s0, e0 = int(idx.offsets[g]), int(idx.offsets[g + 1])
        n = e0 - s0
        rq, rk, rv = idx.rows[0][s0:e0], idx.rows[1][s0:e0], idx.rows[2][s0:e0]
        S = _head_scores(q[rq], k[rk], heads, scale)
        ex = np.exp(S - S.max(axis=0))
        a = ex / ex.sum(axis=0)                                    # [n, heads]
        V = v[rv].reshape(n, heads, dv // heads)
        do = dout[g].reshape(heads, dv // heads)
        dp = (V * do[None]).sum(axis=2)                            # [n, heads]
        ds = a * (dp - (a * dp).sum(axis=0))
        np.add.at(dvv, rv, (a[:, :, None] * do[None]).reshape(n, dv))
        Qh = q[rq].reshape(n, heads, d // heads)
        Kh = k[rk].reshape(n, heads, d // heads)
        np.add.at(dq, rq, (scale * ds[:, :, None] * Kh).reshape(n, d))
        np.add.at(dk, rk, (scale * ds[:, :, None] * Qh).reshape(n, d))
    return dq, dk, dvv
