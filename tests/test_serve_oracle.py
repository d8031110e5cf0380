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
