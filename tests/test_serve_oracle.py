"""Pins of the serving oracle's sampler (CPU only)."""
import numpy as np
import pytest

from oracle import serve_oracle as so


def test_splitmix64_published_vectors():
    # SplitMix64 reference outputs: seed 1234567, and the first output of seed 0
    assert so.splitmix64_stream(1234567, 5) == [6457827717110365317, 3203168211198807973, 9817491932198370423,
                                                4593380528125082431, 16408922859458223821]
    assert so.splitmix64_stream(0, 1) == [0xE220A8397B1DCDAF]


@pytest.mark.parametrize("n,k", [(1, 1), (5, 5), (20, 15), (1000, 10), (7, 0)])
def test_floyd_distinct_sorted_in_range(n, k):
    for seed in range(50):
        p = so.floyd(so.stream_base(seed, 1, 3), n, k)
        assert len(p) == k and len(set(p)) == k
        assert p == sorted(p) and all(0 <= x < n for x in p)


def test_floyd_takes_everything_when_k_equals_n():
    assert so.floyd(12345, 9, 9) == list(range(9))


def test_floyd_is_uniform():
    n, k, trials = 12, 4, 6000
    counts = np.zeros(n)
    for t in range(trials):
        for x in so.floyd(so.stream_base(t, 2, 7), n, k):
            counts[x] += 1
    expected = trials * k / n
    chi2 = ((counts - expected) ** 2 / expected).sum()
    assert chi2 < 35.0          # 11 degrees of freedom; p < 1e-3 beyond ~31.3


def test_streams_are_keyed_by_request_hop_and_node():
    a = so.stream_base(1, 1, 5)
    assert a != so.stream_base(2, 1, 5) and a != so.stream_base(1, 2, 5) and a != so.stream_base(1, 1, 6)


def test_adjacency_orders():
    u = np.array([3, 1, 2, 1, 0, 3], np.int32)
    i = np.array([0, 0, 1, 0, 1, 1], np.int32)
    i_off, i_user, u_off, u_item = so.adjacency(u, i, 2, 4)
    assert i_off.tolist() == [0, 3, 6]
    assert i_user.tolist() == [1, 1, 3, 0, 2, 3]
    assert u_off.tolist() == [0, 1, 3, 4, 6]
    assert u_item.tolist() == [1, 0, 0, 1, 0, 1]


def test_evaluate_single_buyer_reduces_to_layer_formulas():
    """A seed with one buyer who bought only it: the network is three
    Linear+ReLU maps of the concatenated rows (the aggregates are over one
    tuple)."""
    rng = np.random.default_rng(0)
    d = h = 4
    user = rng.standard_normal((2, d))
    item = rng.standard_normal((1, d))
    cat = rng.standard_normal((1, d))
    W = [rng.standard_normal((2 * d, h)), rng.standard_normal((3 * d, h)), rng.standard_normal((3 * d, h))]
    adj = so.adjacency(np.array([1], np.int32), np.array([0], np.int32), 1, 2)
    out, present, tuples = so.evaluate(adj, (user, item, cat, np.array([0])), W, (None, None, None), [0], 9, 15, 10)
    relu = lambda v: np.maximum(v, 0)
    u1 = relu(np.concatenate([user[1], item[0]]) @ W[0])
    i1 = relu(np.concatenate([user[1], item[0], cat[0]]) @ W[1])
    ref = relu(np.concatenate([u1, i1, cat[0]]) @ W[2])
    np.testing.assert_allclose(out[0], ref, rtol=1e-12, atol=1e-12)
    assert present.tolist() == [True] and tuples == 3


# ------------------------------------------------------------------ network
def _golden():
    import json
    import os
    from fractions import Fraction

    with open(os.path.join(os.path.dirname(__file__), "golden", "serve_two_seeds.json")) as f:
        g = json.load(f)
    a = lambda k: np.array(g[k], np.float64)
    frac = lambda rows: np.array([[float(Fraction(v)) for v in r] for r in rows])
    return g, a, frac


def test_evaluate_golden_two_seeds():
    """Hand-worked two-seed request: two buyers per seed, two or three
    hop-2 rows per buyer, biases in the User rule and in layer 2, a seed
    with no buyer and an id outside the Item relation."""
    g, a, frac = _golden()
    adj = so.adjacency(np.array(g["buys_user"], np.int32), np.array(g["buys_item"], np.int32),
                       len(g["item"]), len(g["user"]))
    out, present, tuples = so.evaluate(
        adj, (a("user"), a("item"), a("cat"), np.array(g["item_cat"])),
        (a("W_user"), a("W_item1"), a("W_item2")), (a("b_user"), a("b_item1"), a("b_item2")),
        g["seeds"], g["req_seed"], g["fanout1"], g["fanout2"])
    np.testing.assert_allclose(out, frac(g["out"]), rtol=1e-14, atol=1e-14)
    assert present.tolist() == g["present"]
    assert tuples == g["tuples"]


def _sampled(adj, seeds, req_seed, f1, f2):
    """The link rows a request samples: (buyer, seed) hop-1 rows and, per
    distinct buyer, its (buyer, item) hop-2 rows."""
    i_off, i_user, u_off, u_item = adj
    hop1, hop2, seen = [], [], set()
    for s in seeds:
        deg = int(i_off[s + 1] - i_off[s])
        for p in so.floyd(so.stream_base(req_seed, 1, s), deg, min(f1, deg)):
            u = int(i_user[i_off[s] + p])
            hop1.append((u, int(s)))
            if u not in seen:
                seen.add(u)
                du = int(u_off[u + 1] - u_off[u])
                for q in so.floyd(so.stream_base(req_seed, 2, u), du, min(f2, du)):
                    hop2.append((u, int(u_item[u_off[u] + q])))
    return hop1, hop2


def test_evaluate_matches_layer_oracle_on_sampled_rows():
    """The serving network equals three join rules of the layer oracle
    (itself pinned by brute force, closed forms and a golden) evaluated on
    the sampled link rows, with fanouts below the degrees so that the
    sampler really chooses."""
    import relgen
    from oracle import relnn_oracle as orc

    rng = np.random.default_rng(11)
    n_user, n_item, n_cat, n_buys, d = 25, 10, 3, 260, 4
    user, item, cat = (rng.standard_normal((n, d)) for n in (n_user, n_item, n_cat))
    item_cat = rng.integers(0, n_cat, n_item).astype(np.int32)
    bu = rng.integers(0, n_user, n_buys).astype(np.int32)
    bi = rng.integers(0, n_item, n_buys).astype(np.int32)
    W = [rng.standard_normal((2 * d, d)), rng.standard_normal((3 * d, d)), rng.standard_normal((3 * d, d))]
    b = [rng.standard_normal(d) for _ in range(3)]
    adj = so.adjacency(bu, bi, n_item, n_user)
    seeds, req_seed, f1, f2 = [7, 2, 5, 0], 12345, 4, 3
    out, present, _ = so.evaluate(adj, (user, item, cat, item_cat), W, b, seeds, req_seed, f1, f2)
    assert present.all()
    hop1, hop2 = _sampled(adj, seeds, req_seed, f1, f2)
    assert all(int(adj[2][u + 1] - adj[2][u]) > f2 for u, _ in hop1[:3])     # the sampler does choose
    col = lambda rows, j: np.array([r[j] for r in rows], np.int32)
    run = lambda rule: orc.layer_fwd(orc.build_index(rule), [x.emb for x in rule.atoms], rule.W, rule.b,
                                     rule.agg, rule.act_pre, rule.act_post)
    ru = relgen.Rule(cols=[col(hop2, 0), col(hop2, 1)], atoms=[relgen.Atom(0, user), relgen.Atom(1, item)],
                     group_col=0, W=W[0], b=b[0], agg="mean", act_post="relu")
    iu = orc.build_index(ru)
    u_out = run(ru)[0]
    chain = [relgen.Chain(src_col=1, vals=item_cat)]
    r1 = relgen.Rule(cols=[col(hop1, 0), col(hop1, 1)], chains=chain,
                     atoms=[relgen.Atom(0, user), relgen.Atom(1, item), relgen.Atom(2, cat)],
                     group_col=1, W=W[1], b=b[1], agg="sum", act_post="relu")
    i1 = orc.build_index(r1)
    i_out = run(r1)[0]
    r2 = relgen.Rule(cols=[col(hop1, 0), col(hop1, 1)], chains=chain,
                     atoms=[relgen.Atom(0, u_out, iu.group_keys.astype(np.int32)),
                            relgen.Atom(1, i_out, i1.group_keys.astype(np.int32)), relgen.Atom(2, cat)],
                     group_col=1, W=W[2], b=b[2], agg="sum", act_post="relu")
    i2 = orc.build_index(r2)
    ref = run(r2)[0]
    for q, s in enumerate(seeds):
        np.testing.assert_allclose(out[q], ref[int(np.nonzero(i2.group_keys == s)[0][0])], rtol=1e-12, atol=1e-12)
