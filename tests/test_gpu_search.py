"""Online search on the GPU (``bdg_graph_search``) against the CPU oracle:
identical answers (indices and float32 distances, bit for bit) and visited
counts for several pool sizes, queries inside the base (their own row
excluded) and outside it, and graphs with absent entries."""
import numpy as np
import pytest

import oracle
from oracle import learned
from paper_2102_04656_amd import bdg

pytestmark = pytest.mark.gpu

NO_IDX = oracle.NO_IDX


def world(n, d, bits, K, seed, holes=False):
    g = np.random.default_rng(seed)
    centres = g.standard_normal((20, d)) * 2.0
    feats = (centres[g.integers(0, 20, n)] + g.standard_normal((n, d))).astype(np.float32)
    proj = g.standard_normal((d, bits)).astype(np.float32)
    codes = learned.srp_encode(feats, proj)
    gi, _ = oracle.knn_rows(codes, K)
    gi = gi.copy()
    if holes:
        gi[::5, K // 2:] = NO_IDX
        gi[1::7, 0] = n + 5
    return feats, codes, gi, proj, g


def run_gpu(codes, gi, feats, qc, qf, excl, entries, P, N):
    import torch
    t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a).view(dt)).cuda()
    out = bdg.graph_search(t(codes, np.int64), t(gi, np.int32), t(feats, np.float32),
                           t(qc, np.int64), t(qf, np.float32), t(entries, np.int32), P, N,
                           q_exclude=None if excl is None else t(excl, np.int32))
    torch.cuda.synchronize()
    return (out[0].cpu().numpy().view(np.uint32), out[1].cpu().numpy(),
            out[2].cpu().numpy().view(np.uint32))


@pytest.mark.parametrize("n,d,bits,K,P,N,seed,holes", [
    (2000, 32, 128, 16, 16, 10, 51, False),
    (2000, 32, 128, 16, 64, 20, 52, False),
    (1500, 48, 256, 24, 100, 60, 53, True),   # two rows of pool keys, holed graph
    (1200, 16, 64, 12, 256, 60, 54, False),   # four rows of pool keys
    (2500, 24, 128, 16, 512, 60, 56, False),  # eight rows
    (3000, 24, 128, 20, 1000, 100, 57, True), # sixteen rows, ragged
])
def test_search_matches_oracle(n, d, bits, K, P, N, seed, holes):
    print(f"[search] n={n} d={d} bits={bits} K={K} P={P} N={N}", flush=True)
    feats, codes, gi, proj, g = world(n, d, bits, K, seed, holes)
    entries = np.sort(g.choice(n, size=64, replace=False)).astype(np.uint32)
    qrows = np.sort(g.choice(n, size=30, replace=False)).astype(np.uint32)
    gi_i, gi_d, gi_v = run_gpu(codes, gi, feats, codes[qrows], feats[qrows], qrows, entries, P, N)
    for k, q in enumerate(qrows.tolist()):
        oi, od, ov = oracle.graph_search(codes, gi, feats, codes[q], feats[q], entries, P, N,
                                         exclude=q)
        assert np.array_equal(gi_i[k], oi), k
        assert np.array_equal(gi_d[k].view(np.uint32), od.view(np.uint32)), k
        assert int(gi_v[k]) == ov - 1  # the oracle counts the excluded row as visited


def test_search_new_queries():
    n, d, bits, K, P, N = 1500, 24, 128, 16, 48, 12
    feats, codes, gi, proj, g = world(n, d, bits, K, 55)
    qf = (feats[g.choice(n, 20)] + 0.3 * g.standard_normal((20, d))).astype(np.float32)
    qc = learned.srp_encode(qf, proj)
    entries = np.sort(g.choice(n, size=100, replace=False)).astype(np.uint32)
    gi_i, gi_d, gi_v = run_gpu(codes, gi, feats, qc, qf, None, entries, P, N)
    for k in range(20):
        oi, od, ov = oracle.graph_search(codes, gi, feats, qc[k], qf[k], entries, P, N)
        assert np.array_equal(gi_i[k], oi) and np.array_equal(gi_d[k].view(np.uint32), od.view(np.uint32))
        assert int(gi_v[k]) == ov


def test_search_hand_derived_trace():
    """The 9-row fixture of tests/golden/search_small.txt (pool of 3 on a
    graph of 2 neighbours per row): answers, distances and visited counts as
    derived by hand (the GPU count leaves out the excluded row)."""
    from tests import golden_io
    codes, gi, feats, entries, cases = golden_io.search_small()
    qc = np.zeros((1, 1), dtype=np.uint64)
    qf = np.zeros((1, feats.shape[1]), dtype=np.float32)
    for name, c in cases.items():
        excl = None if c["exclude"] is None else np.array([c["exclude"]], dtype=np.uint32)
        print(f"[search] fixture case {name}", flush=True)
        oi, od, ov = run_gpu(codes, gi, feats, qc, qf, excl, np.array(entries, dtype=np.uint32),
                             c["P"], c["N"])
        assert [(int(i), float(d)) for i, d in zip(oi[0], od[0])] == c["answer"], name
        assert int(ov[0]) == c["visited"] - (0 if excl is None else 1), name
