"""Pins of the online-search oracle (CPU only): with a pool larger than the
data and a connected graph the search visits every row, so its answer is the
exact float kNN (checked against the float64 library route of
``oracle.learned.float_knn``); a pool of one is greedy descent, ending at a
row no neighbour of which is closer; the float32 re-rank distance is the
float64 distance up to rounding; the row excluded never appears."""
import numpy as np

import oracle
from oracle import learned
from paper_2102_04656_amd import datagen


def small_world(n, d, bits, K, seed):
    g = np.random.default_rng(seed)
    feats = g.standard_normal((n, d)).astype(np.float32)
    proj = g.standard_normal((d, bits)).astype(np.float32)
    codes = learned.srp_encode(feats, proj)
    gi, _ = oracle.knn_rows(codes, K)
    gi = gi.copy()
    gi[:, K - 1] = (np.arange(n) + 1) % n  # a ring: every row reachable
    return feats, codes, gi


def test_full_pool_gives_exact_float_knn():
    feats, codes, gi = small_world(300, 16, 64, 8, 1)
    entries = np.arange(0, 300, 37)
    want, _ = learned.float_knn(feats[:12], feats, 10, exclude=np.arange(12))
    for q in range(12):
        idx, dist, nvis = oracle.graph_search(codes, gi, feats, codes[q], feats[q], entries,
                                              P=400, N=10, exclude=q)
        assert nvis == 300
        assert list(idx) == list(want[q])


def test_pool_of_one_is_greedy_descent():
    feats, codes, gi = small_world(400, 16, 128, 10, 2)
    u = datagen.unpack_bits(codes).astype(np.int16)
    for q in range(20):
        idx, _, _ = oracle.graph_search(codes, gi, feats, codes[q], feats[q], [5, 100, 250],
                                        P=1, N=1, exclude=q)
        x = int(idx[0])
        hx = int((u[x] != u[q]).sum())
        for v in gi[x]:
            if int(v) != q:
                assert int((u[int(v)] != u[q]).sum()) >= hx


def test_l2_f32_close_to_float64():
    g = np.random.default_rng(3)
    a, b = g.standard_normal(512), g.standard_normal(512)
    exact = float(((a.astype(np.float32).astype(np.float64) - b.astype(np.float32)) ** 2).sum())
    assert abs(float(oracle.l2_f32(a, b)) - exact) <= 1e-5 * exact


def test_planted_missing_exclusion_caught():
    feats, codes, gi = small_world(200, 16, 64, 8, 4)
    q = 7
    idx, _, _ = oracle.graph_search(codes, gi, feats, codes[q], feats[q], [0, 50], P=300, N=5,
                                    exclude=None)
    # without the exclusion the query's own row (distance 0) comes first,
    # which the exact float kNN with the row excluded does not contain
    want, _ = learned.float_knn(feats[q:q + 1], feats, 5, exclude=np.array([q]))
    assert int(idx[0]) == q and list(idx) != list(want[0])
