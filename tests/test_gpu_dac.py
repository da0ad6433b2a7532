"""Single-pass divide-and-conquer on the GPU (``bdg_bkmeans``,
``bdg_build_knn_dac``) against the CPU oracle: identical centres after every
number of k-means rounds, bit-exact approximate graphs for several budgets,
code lengths and list classes, the exact graph when every centre is
selected, and the entry points' errors."""
import numpy as np
import pytest

import oracle
from paper_2102_04656_amd import bdg, datagen

pytestmark = pytest.mark.gpu


def dev(codes):
    import torch
    return torch.from_numpy(np.ascontiguousarray(codes).view(np.int64)).cuda()


def seeded_sample(n, ns, m, seed):
    g = np.random.default_rng(seed)
    sample = np.sort(g.choice(n, size=ns, replace=False)).astype(np.uint32)
    init = sample[np.sort(g.choice(ns, size=m, replace=False))]
    return sample, init


@pytest.mark.parametrize("n,bits,centres,m,iters,seed", [
    (2000, 128, 20, 16, 0, 31),
    (2000, 128, 20, 16, 5, 31),
    (1500, 256, 12, 40, 3, 32),
    (1200, 64, 8, 5, 8, 33),
    (900, 512, 6, 70, 2, 34),     # more centres than one 64-lane step
])
def test_bkmeans_matches_oracle(n, bits, centres, m, iters, seed):
    import torch
    print(f"[bkmeans] n={n} bits={bits} m={m} iters={iters}", flush=True)
    codes = datagen.clustered_codes(n, bits, centres, 0.2, seed)
    sample, init = seeded_sample(n, n // 2, m, seed)
    want = oracle.bkmeans(codes, sample, init, iters)
    got = bdg.bkmeans(dev(codes), sample, init, iters)
    torch.cuda.synchronize()
    assert np.array_equal(got.cpu().numpy().view(np.uint64), want)


@pytest.mark.parametrize("n,bits,m,T,coarse,K,seed", [
    (3000, 256, 24, 8, 300, 16, 41),
    (3000, 256, 24, 8, 1000, 64, 41),
    (2500, 128, 40, 16, 600, 100, 42),   # two rows of keys
    (2000, 192, 10, 4, 1, 8, 43),        # budget of one: home clusters only
    (1800, 64, 90, 64, 250, 33, 44),     # T = 64, ragged K
])
def test_dac_graph_matches_oracle(n, bits, m, T, coarse, K, seed):
    import torch
    print(f"[dac] n={n} bits={bits} m={m} T={T} coarse={coarse} K={K}", flush=True)
    codes = datagen.clustered_codes(n, bits, 12, 0.2, seed)
    sample, init = seeded_sample(n, n // 3, m, seed)
    C = oracle.bkmeans(codes, sample, init, 3)
    want = oracle.dac_graph(codes, C, T, coarse, K)
    gi, gd = bdg.build_knn_dac(dev(codes), dev(C), K, T, coarse)
    torch.cuda.synchronize()
    gi, gd = bdg.to_numpy_graph(gi, gd)
    assert np.array_equal(gi, want[0])
    assert np.array_equal(gd, want[1])


def test_dac_every_centre_is_exact():
    import torch
    w = datagen.WORKLOADS["clustered-20k-128b-k32"]
    codes = datagen.clustered_codes(w["n"], w["bits"], w["n_centres"], w["p"], w["seed"])
    sample, init = seeded_sample(w["n"], 4000, 48, 45)
    C = bdg.bkmeans(dev(codes), sample, init, 4)
    gi, gd = bdg.build_knn_dac(dev(codes), C, w["K"], 64, w["n"])
    torch.cuda.synchronize()
    ei, ed = oracle.knn_rows(codes, w["K"])
    gi, gd = bdg.to_numpy_graph(gi, gd)
    assert np.array_equal(gi, ei) and np.array_equal(gd, ed)


def test_dac_errors():
    import torch
    lib = bdg.lib()
    c = torch.zeros((8, 2), dtype=torch.int64, device="cuda")
    C = torch.zeros((2, 2), dtype=torch.int64, device="cuda")
    oi = torch.empty((8, 4), dtype=torch.int32, device="cuda")
    od = torch.empty((8, 4), dtype=torch.int16, device="cuda")
    p = bdg._ptr
    s = bdg._stream(None)
    assert lib.bdg_build_knn_dac(p(c), 8, 100, p(C), 2, 2, 4, 4, p(oi), p(od), s) == bdg.BDG_EINVAL
    assert lib.bdg_build_knn_dac(p(c), 8, 128, p(C), 2, 65, 4, 4, p(oi), p(od), s) == bdg.BDG_EUNSUPPORTED
    assert lib.bdg_build_knn_dac(p(c), 8, 128, p(C), 2, 2, 0, 4, p(oi), p(od), s) == bdg.BDG_EINVAL
    assert lib.bdg_build_knn_dac(p(c), 0, 128, p(C), 2, 2, 4, 4, p(oi), p(od), s) == bdg.BDG_OK
    bad = np.array([0, 9], dtype=np.uint32)  # row 9 of 8
    ok = np.array([0, 1], dtype=np.uint32)
    assert lib.bdg_bkmeans(p(c), 8, 128, ok.ctypes.data, 2, bad.ctypes.data, 2, 1, p(C), s) == bdg.BDG_EINVAL
    assert lib.bdg_bkmeans(p(c), 8, 128, bad.ctypes.data, 2, ok.ctypes.data, 2, 1, p(C), s) == bdg.BDG_EINVAL
