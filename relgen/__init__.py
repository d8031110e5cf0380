"""Seeded synthetic relations shaped like the relational workloads of the paper.

This module draws random numbers and arranges them into relations; it holds
none of the method's arithmetic (no join, transform or aggregate).  Both the
FP64 oracle and the HIP library consume what it produces, so it is the only
code the two share.

A *rule* follows the join rule of Section 3.1,

    Out(g; alpha(Linear(z_1 (+) ... (+) z_k))) :- Link(...), R_1(c_1; z_1), ..., R_k(c_k; z_k)

where the link relation carries the foreign keys, every body atom R_j is an
embedded relation (Section 2.1: content key plus an embedding row), and the
head key g is one column of the link relation (the projection attribute of
the projected union, Section 2.2).

Every draw uses numpy's ``default_rng`` seeded from ``SeedSequence(seed)``
spawn streams; seed 42 is the first seed of the paper's runs (Section 5.1).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

SEED = 42

AGGS = ("sum", "mean", "max")
ACTS = ("none", "relu")


@dataclass
class Atom:
    """Body atom R_j(key; z_j).  ``keys`` None means dense ids 0..n-1."""
    col: int                       # link (or derived) column holding the FK
    emb: np.ndarray                # [n_rows, d] float32 embedding attribute
    keys: Optional[np.ndarray] = None   # [n_rows] int32 primary key, or None

    @property
    def n_rows(self) -> int:
        return int(self.emb.shape[0])

    @property
    def d(self) -> int:
        return int(self.emb.shape[1])


@dataclass
class Chain:
    """Derived column: value of ``vals`` at the row of a lookup relation whose
    key equals column ``src_col`` (an FK chain such as Buys.item ->
    BelongsTo.cat).  ``keys`` None means the lookup relation is dense."""
    src_col: int
    vals: np.ndarray               # [n_rows] int32
    keys: Optional[np.ndarray] = None

    @property
    def n_rows(self) -> int:
        return int(self.vals.shape[0])


@dataclass
class Step:
    """A further link relation joined into the tuples so far (general and
    cyclic joins): columns ``cols``, matched where column ``on[q]`` of the
    tuples so far equals column ``key[q]`` of this relation, for every q."""
    cols: List[np.ndarray]         # int32 [n_rows] each
    on: List[int]
    key: List[int]

    @property
    def n_rows(self) -> int:
        return int(self.cols[0].shape[0])


# comparison operators of a filter predicate, in the library's numbering
CMP = ("eq", "ne", "lt", "le", "gt", "ge")


@dataclass
class Pred:
    """One atomic predicate of a filter expression: mul_a * col[a] + mul_b *
    col[b] + add  <op>  0 (a or b = -1: the term is absent)."""
    a: int
    op: str
    b: int = -1
    mul_a: int = 1
    mul_b: int = -1
    add: int = 0


@dataclass
class Rule:
    cols: List[np.ndarray]         # link relation columns, int32 [n_link] each
    atoms: List[Atom]
    group_col: int
    W: np.ndarray                  # [K, h] float32, y = x W + b
    b: np.ndarray                  # [h] float32
    agg: str = "sum"
    act_pre: str = "none"
    act_post: str = "none"
    chains: List[Chain] = field(default_factory=list)
    two_hop_mid: int = -1          # column the link relation is self-joined on
    two_hop_cap: int = 0           # paths kept per mid key
    steps: List[Step] = field(default_factory=list)   # further link relations joined in
    preds: List[Pred] = field(default_factory=list)   # filter expression (a conjunction)

    @property
    def K(self) -> int:
        return int(sum(a.d for a in self.atoms))

    @property
    def h(self) -> int:
        return int(self.W.shape[1])

    @property
    def n_link(self) -> int:
        return int(self.cols[0].shape[0])


def rngs(seed: int, n: int) -> List[np.random.Generator]:
    """n independent generators, one per tensor, from one seed."""
    return [np.random.default_rng(s) for s in np.random.SeedSequence(seed).spawn(n)]


def normal(rng, shape, std=1.0) -> np.ndarray:
    x = rng.standard_normal(shape, dtype=np.float32)
    if std != 1.0:
        x *= np.float32(std)
    return x


def zipf_ids(rng, n_draws: int, n_support: int, s: float) -> np.ndarray:
    """Bounded Zipf over ranks 1..N with P(k) proportional to k**-s, drawn by
    inverse CDF; ranks are mapped to ids through a seeded permutation so the
    hot ids are spread over the id space."""
    w = np.arange(1, n_support + 1, dtype=np.float64) ** (-s)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    u = rng.random(n_draws)
    rank = np.searchsorted(cdf, u, side="right")
    rank = np.minimum(rank, n_support - 1)
    perm = rng.permutation(n_support).astype(np.int32)
    return perm[rank]


def uniform_ids(rng, n_draws: int, n_support: int) -> np.ndarray:
    return rng.integers(0, n_support, size=n_draws, dtype=np.int64).astype(np.int32)


# --------------------------------------------------------------------------
# Workload 1: plain single layer.  Node(id, z in R^d) with n_nodes rows,
# z ~ N(0,1); Edge(s,t) with n_edges rows, s and t uniform over the ids;
# z'_t = ReLU(SUM over Edge of Linear(Concat(z_s, z_t))), W ~ N(0, 0.1) (std),
# b = 0.  With d = h = 256 and BF16 it is the precision form.
# --------------------------------------------------------------------------
def node_edge(seed=SEED, n_nodes=1000, n_edges=5000, d=32, h=32, w_std=0.1,
              agg="sum", act_pre="none", act_post="relu", bias_std=0.0,
              src_zipf: Optional[float] = None) -> Rule:
    r = rngs(seed, 6)
    z = normal(r[0], (n_nodes, d))
    if src_zipf is None:
        s = uniform_ids(r[1], n_edges, n_nodes)
    else:
        s = zipf_ids(r[1], n_edges, n_nodes, src_zipf)
    t = uniform_ids(r[2], n_edges, n_nodes)
    W = normal(r[3], (2 * d, h), w_std)
    b = normal(r[4], (h,), bias_std) if bias_std > 0 else np.zeros(h, np.float32)
    return Rule(cols=[s, t], atoms=[Atom(0, z), Atom(1, z)], group_col=1,
                W=W, b=b, agg=agg, act_pre=act_pre, act_post=act_post)


# --------------------------------------------------------------------------
# Workload 2: heterogeneous ER schema.  User(n_user), Item(n_item),
# Category(n_cat); Buys(user, item) with item ~ Zipf(1.1), user uniform;
# BelongsTo(item, cat) one row per item, cat uniform.  Embeddings N(0,1),
# weights N(0, 1/sqrt(fan_in)) (std).  Item rule: SUM of
# Linear(User (+) Item (+) Category) grouped by item; User rule: MEAN of
# Linear(User (+) Item) grouped by user; ReLU after each aggregate.
# --------------------------------------------------------------------------
@dataclass
class ERGraph:
    user: np.ndarray
    item: np.ndarray
    cat: np.ndarray
    buys_u: np.ndarray
    buys_i: np.ndarray
    belongs_cat: np.ndarray        # [n_item] category of each item
    W_item: List[np.ndarray]       # per layer [3d, h]
    W_user: List[np.ndarray]       # per layer [2d, h]
    b_item: List[np.ndarray]
    b_user: List[np.ndarray]


def er_graph(seed=SEED, n_user=1_000_000, n_item=500_000, n_cat=1000,
             n_buys=20_000_000, d=128, h=128, item_zipf=1.1, n_layers=2) -> ERGraph:
    r = rngs(seed, 8 + 4 * n_layers)
    user = normal(r[0], (n_user, d))
    item = normal(r[1], (n_item, d))
    cat = normal(r[2], (n_cat, d))
    bu = uniform_ids(r[3], n_buys, n_user)
    bi = zipf_ids(r[4], n_buys, n_item, item_zipf)
    bc = uniform_ids(r[5], n_item, n_cat)
    Wi, Wu, bi_, bu_ = [], [], [], []
    for L in range(n_layers):
        din = d if L == 0 else h
        Wi.append(normal(r[8 + 4 * L], (3 * din, h), 1.0 / np.sqrt(3 * din)))
        Wu.append(normal(r[9 + 4 * L], (2 * din, h), 1.0 / np.sqrt(2 * din)))
        bi_.append(np.zeros(h, np.float32))
        bu_.append(np.zeros(h, np.float32))
    return ERGraph(user, item, cat, bu, bi, bc, Wi, Wu, bi_, bu_)


def er_item_rule(g: ERGraph, layer=0, user=None, item=None, user_keys=None,
                 item_keys=None) -> Rule:
    """Item'(i; sum(Lin(z_u (+) z_i (+) z_c))) :- Buys(u,i), BelongsTo(i,c),
    User(u; z_u), Item(i; z_i), Category(c; z_c).  Columns: 0 = Buys.user,
    1 = Buys.item, 2 = derived BelongsTo.cat of Buys.item."""
    U = g.user if user is None else user
    I = g.item if item is None else item
    return Rule(cols=[g.buys_u, g.buys_i],
                chains=[Chain(src_col=1, vals=g.belongs_cat)],
                atoms=[Atom(0, U, user_keys), Atom(1, I, item_keys), Atom(2, g.cat)],
                group_col=1, W=g.W_item[layer], b=g.b_item[layer],
                agg="sum", act_post="relu")


def er_user_rule(g: ERGraph, layer=0, user=None, item=None, user_keys=None,
                 item_keys=None) -> Rule:
    """User'(u; mean(Lin(z_u (+) z_i))) :- Buys(u,i), User(u; z_u), Item(i; z_i)."""
    U = g.user if user is None else user
    I = g.item if item is None else item
    return Rule(cols=[g.buys_u, g.buys_i],
                atoms=[Atom(0, U, user_keys), Atom(1, I, item_keys)],
                group_col=0, W=g.W_user[layer], b=g.b_user[layer],
                agg="mean", act_post="relu")


def cobuy_rule(g: ERGraph, seed=SEED, d=256, h=256, cap=50, agg="max") -> Rule:
    """Two-hop precision form: CoBuy(u1; agg(Lin(z_u1 (+) z_u2))) :-
    Buys(u1,i), Buys(u2,i), User(u1), User(u2), at most ``cap`` paths per
    item.  After the self-join on Buys.item the path relation has columns
    0..1 from the first Buys row and 2..3 from the second."""
    r = rngs(seed + 1, 3)
    n_user = g.user.shape[0]
    U = normal(r[0], (n_user, d))
    W = normal(r[1], (2 * d, h), 1.0 / np.sqrt(2 * d))
    return Rule(cols=[g.buys_u, g.buys_i], atoms=[Atom(0, U), Atom(2, U)],
                group_col=0, W=W, b=np.zeros(h, np.float32), agg=agg,
                two_hop_mid=1, two_hop_cap=cap)


# --------------------------------------------------------------------------
# Workload 4: differentiation form.  Node [n, d], Edge with s ~ Zipf(1.2)
# (power-law out-degree) and t uniform; layer 1 SUM + ReLU, layer 2 MAX; MSE
# against N(0,1) targets.
# --------------------------------------------------------------------------
@dataclass
class PowerGraph:
    z: np.ndarray
    s: np.ndarray
    t: np.ndarray
    W: List[np.ndarray]
    b: List[np.ndarray]
    target: np.ndarray


def power_graph(seed=SEED, n_nodes=2_000_000, n_edges=10_000_000, d=128, h=128,
                s_zipf=1.2, bias_std=0.0) -> PowerGraph:
    r = rngs(seed, 8)
    z = normal(r[0], (n_nodes, d))
    s = zipf_ids(r[1], n_edges, n_nodes, s_zipf)
    t = uniform_ids(r[2], n_edges, n_nodes)
    W = [normal(r[3], (2 * d, h), 1.0 / np.sqrt(2 * d)),
         normal(r[4], (2 * h, h), 1.0 / np.sqrt(2 * h))]
    if bias_std > 0:
        b = [normal(r[5], (h,), bias_std), normal(r[6], (h,), bias_std)]
    else:
        b = [np.zeros(h, np.float32), np.zeros(h, np.float32)]
    target = normal(r[7], (n_nodes, h))
    return PowerGraph(z, s, t, W, b, target)


def power_rule(p: PowerGraph, layer: int, z=None, z_keys=None) -> Rule:
    zz = p.z if z is None else z
    agg, post = ("sum", "relu") if layer == 0 else ("max", "none")
    return Rule(cols=[p.s, p.t], atoms=[Atom(0, zz, z_keys), Atom(1, zz, z_keys)],
                group_col=1, W=p.W[layer], b=p.b[layer], agg=agg, act_post=post)


# --------------------------------------------------------------------------
# Cyclic joins: the triangle rule of the paper's DHN encoding (Section 5.2),
# on many small graphs like its graph-classification sets (Section 5.1).
# Each graph has n_nodes nodes with global ids (graph g holds g n .. g n +
# n - 1) and random undirected edges stored in both directions as
# Edge(g, src, dst); H0 gives every node an N(0, 1) embedding.
#
#   C3(n; sum(Lin(h_n (+) h_v (+) h_w))) :- Edge(g,n,v), Edge(g,v,w), Edge(g,w,n),
#                                           H0(n; h_n), H0(v; h_v), H0(w; h_w)
#
# as a link relation Edge (columns 0 g, 1 n, 2 v) with two further Edge
# relations: the first on v = src and g = g (adding columns 3 g, 4 v, 5 w),
# the second on w = src and n = dst (adding 6 g, 7 w, 8 n), which closes the
# cycle.  W ~ N(0, 1/sqrt(3d)).
# --------------------------------------------------------------------------
def triangle_rule(seed=SEED, n_graphs=150, n_nodes=40, avg_degree=6, d=64, h=64, agg="sum",
                  act_post="relu", bias_std=0.0) -> Rule:
    r = rngs(seed + 7, 5)
    n_und = n_graphs * n_nodes * avg_degree // 2
    g = r[0].integers(0, n_graphs, n_und)
    a = r[1].integers(0, n_nodes, n_und)
    b = (a + 1 + r[2].integers(0, n_nodes - 1, n_und)) % n_nodes       # no self-loops
    src = np.concatenate([g * n_nodes + a, g * n_nodes + b]).astype(np.int32)
    dst = np.concatenate([g * n_nodes + b, g * n_nodes + a]).astype(np.int32)
    gg = np.concatenate([g, g]).astype(np.int32)
    edge = [gg, src, dst]
    z = normal(r[3], (n_graphs * n_nodes, d))
    W = normal(r[4], (3 * d, h), 1.0 / np.sqrt(3 * d))
    bb = normal(r[4], (h,), bias_std) if bias_std > 0 else np.zeros(h, np.float32)
    steps = [Step(cols=[c.copy() for c in edge], on=[2, 0], key=[1, 0]),
             Step(cols=[c.copy() for c in edge], on=[5, 1], key=[1, 2])]
    return Rule(cols=edge, atoms=[Atom(1, z), Atom(2, z), Atom(5, z)], group_col=1, W=W, b=bb,
                agg=agg, act_post=act_post, steps=steps)


# --------------------------------------------------------------------------
# Workload 5: serving requests.  Seed-item sets with sizes log-uniform over
# 1..max_seeds, Poisson arrivals at rate ``rate`` per second.
# --------------------------------------------------------------------------
@dataclass
class Request:
    t_arrive: float
    seeds: np.ndarray              # distinct item ids, int32
    req_seed: int


def request_stream(n_items: int, n_req: int, rate: float, seed=SEED,
                   max_seeds=4096) -> List[Request]:
    r = rngs(seed + 5, 3)
    sizes = np.floor(np.exp(r[0].random(n_req) * np.log(max_seeds + 1))).astype(np.int64)
    sizes = np.clip(sizes, 1, max_seeds)
    gaps = r[1].exponential(1.0 / rate, size=n_req)
    t = np.cumsum(gaps) - gaps[0]
    out = []
    for q in range(n_req):
        n = int(min(sizes[q], n_items))
        seeds = r[2].choice(n_items, size=n, replace=False).astype(np.int32)
        out.append(Request(float(t[q]), seeds, int(r[2].integers(0, 2**62))))
    return out
