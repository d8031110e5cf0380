"""FP64 oracle of the serving form.  TEST INFRASTRUCTURE ONLY (see
relnn_oracle's header for who may import it).

The paper evaluates whole graphs and lists sampling and mini-batches as
future work (Section 6), so this part is a reading of ours, stated here and
in the library header: a request is a set of seed items; hop 1 samples up to
fanout1 buyers of each seed, hop 2 up to fanout2 Buys rows of each sampled
buyer; a two-layer network of join rules (Section 3.1) runs on the sampled
rows.  Parity unpinned by the paper (sampling is not in it): the sampler is
pinned by SplitMix64's published test vectors and by properties of Floyd's
algorithm; the network by a hand-worked two-seed request
(tests/golden/serve_two_seeds.json: several buyers per seed, several hop-2
rows per buyer, biases) and by the three join rules of relnn_oracle (pinned
on its own) evaluated on the same sampled link rows.

SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014) and Floyd's sampling algorithm (Bentley and
Floyd, "A sample of brilliance", CACM 1987) are written from their
published definitions; the GPU has its own copy written the same way.
"""
from __future__ import annotations

import numpy as np

M64 = (1 << 64) - 1
GOLDEN = 0x9E3779B97F4A7C15


def mix64(z: int) -> int:
    """SplitMix64 output function."""
    z &= M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return z ^ (z >> 31)


def splitmix64_stream(seed: int, n: int):
    """The first n outputs of SplitMix64 seeded with ``seed``."""
    s, out = seed & M64, []
    for _ in range(n):
        s = (s + GOLDEN) & M64
        out.append(mix64(s))
    return out


def stream_base(req_seed: int, hop: int, node: int) -> int:
    return mix64((req_seed + (2 * node + hop + 1) * GOLDEN) & M64)


def draw(base: int, q: int) -> int:
    """Draw number q of a stream."""
    return mix64((base + (q + 1) * GOLDEN) & M64)


def floyd(base: int, n: int, k: int):
    """k distinct positions of range(n), Floyd's algorithm: for j = n-k ..
    n-1 take t uniform in [0, j]; keep t unless taken, else keep j.  A
    uniform draw in [0, j] from a 64-bit word r is ((r >> 32) * (j + 1)) >> 32.
    Returned sorted."""
    chosen = []
    for q, j in enumerate(range(n - k, n)):
        r = draw(base, q)
        t = ((r >> 32) * (j + 1)) >> 32
        chosen.append(j if t in chosen else t)
    return sorted(chosen)


def adjacency(buys_user: np.ndarray, buys_item: np.ndarray, n_item: int, n_user: int):
    """Buyers of every item ordered by (user, Buys row), and items of every
    user's Buys rows ordered by (item, Buys row)."""
    rows = np.arange(len(buys_user))
    oi = np.lexsort((rows, buys_user, buys_item))
    i_off = np.searchsorted(buys_item[oi], np.arange(n_item + 1), side="left")
    ou = np.lexsort((rows, buys_item, buys_user))
    u_off = np.searchsorted(buys_user[ou], np.arange(n_user + 1), side="left")
    return i_off, buys_user[oi], u_off, buys_item[ou]


def _lin(x, W, b):
    return x @ np.asarray(W, np.float64) + (0.0 if b is None else np.asarray(b, np.float64))


def evaluate(adj, emb, W, b, seeds, req_seed: int, fanout1: int, fanout2: int):
    """One request.  adj = adjacency(...); emb = (user, item, cat, item_cat);
    W = (W_user, W_item1, W_item2), b likewise (None for zero).  Returns
    (out [n, h] FP64, present [n] bool, tuples evaluated)."""
    i_off, i_user, u_off, u_item = adj
    user, item, cat, item_cat = [np.asarray(a) for a in emb]
    user = user.astype(np.float64)
    item = item.astype(np.float64)
    cat = cat.astype(np.float64)
    h = np.asarray(W[0]).shape[1]
    n_item = len(i_off) - 1
    out = np.zeros((len(seeds), h))
    present = np.zeros(len(seeds), bool)
    tuples = 0
    for q, s in enumerate(seeds):
        s = int(s)
        if s < 0 or s >= n_item:
            continue
        deg = int(i_off[s + 1] - i_off[s])
        k1 = min(fanout1, deg)
        if k1 == 0:
            continue
        present[q] = True
        buyers = [int(i_user[i_off[s] + p]) for p in floyd(stream_base(req_seed, 1, s), deg, k1)]
        c = int(item_cat[s])
        # layer 1, User rule: MEAN over the buyer's sampled Buys rows
        u1 = []
        for u in buyers:
            du = int(u_off[u + 1] - u_off[u])
            k2 = min(fanout2, du)
            items = [int(u_item[u_off[u] + p]) for p in floyd(stream_base(req_seed, 2, u), du, k2)]
            x = np.concatenate([np.repeat(user[u][None], k2, 0), item[items]], axis=1)
            u1.append(np.maximum(_lin(x, W[0], b[0]).sum(axis=0) / k2, 0.0))
            tuples += k2
        # layer 1, Item rule: SUM over the seed's sampled Buys rows
        x = np.concatenate([user[buyers], np.repeat(item[s][None], k1, 0), np.repeat(cat[c][None], k1, 0)], axis=1)
        i1 = np.maximum(_lin(x, W[1], b[1]).sum(axis=0), 0.0)
        # layer 2, Item rule on the layer-1 outputs
        x = np.concatenate([np.array(u1), np.repeat(i1[None], k1, 0), np.repeat(cat[c][None], k1, 0)], axis=1)
        out[q] = np.maximum(_lin(x, W[2], b[2]).sum(axis=0), 0.0)
        tuples += 2 * k1
    return out, present, tuples
