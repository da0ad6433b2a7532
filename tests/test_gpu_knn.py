"""GPU parity: the HIP graph builder (through the C ABI) against the CPU oracle.

Integer work, so the bar is bit-exact equality of indices and distances. The
(distance, index) order makes every row unique, ties included.
"""
import os

import numpy as np
import pytest

import oracle
from paper_2102_04656_amd import bdg, datagen
from tests import golden_io

pytestmark = pytest.mark.gpu

POPC, MFMA = bdg.PATH_POPC, bdg.PATH_MFMA


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    bdg.lib()


def dev(codes):
    import torch
    return torch.from_numpy(np.ascontiguousarray(codes).view(np.int64)).cuda()


def gpu_knn(codes, K, path, **kw):
    import torch
    idx, dist = bdg.build_knn(dev(codes), K, path=path, **kw)
    torch.cuda.synchronize()
    return bdg.to_numpy_graph(idx, dist)


def assert_same(got, want, what=""):
    gi, gd = got
    wi, wd = want
    if not (np.array_equal(gi, wi) and np.array_equal(gd, wd)):
        bad = np.nonzero((gi != wi).any(axis=1) | (gd != wd).any(axis=1))[0]
        r = int(bad[0])
        raise AssertionError(f"{what}: {bad.size} rows differ; first row {r}:\n"
                             f" got  {list(zip(gd[r][:12], gi[r][:12]))}\n"
                             f" want {list(zip(wd[r][:12], wi[r][:12]))}")


# ------------------------------------------------------------ small grid

GRID = [
    # n, bits, K, n_centres, p
    (1, 128, 4, 1, 0.1),
    (2, 64, 1, 1, 0.1),
    (17, 64, 16, 2, 0.1),
    (64, 128, 63, 3, 0.1),
    (65, 192, 64, 3, 0.15),
    (130, 256, 129, 4, 0.2),
    (1000, 64, 32, 20, 0.05),
    (1000, 128, 1, 20, 0.15),
    (1000, 256, 64, 20, 0.2),
    (1000, 320, 65, 20, 0.2),
    (1000, 512, 100, 20, 0.25),
    (1000, 1024, 33, 10, 0.25),
    (777, 448, 128, 7, 0.2),
    (600, 576, 256, 6, 0.2),
    (3001, 256, 7, 40, 0.2),
    # list capacity classes at their bounds (stage rings of 5, 3, 2 and 6 slots)
    (1500, 256, 32, 15, 0.2),
    (900, 512, 112, 9, 0.25),
    (1200, 256, 120, 12, 0.2),
    (1100, 128, 96, 11, 0.15),
]


# matrix-core path under the default schedule (lists in global memory where
# built, else in LDS) and with the lists in LDS everywhere
PATHS = [(POPC, 0), (MFMA, bdg.SCHEDULE_DEFAULT), (MFMA, bdg.SCHEDULE_LDS_LISTS)]
PATH_IDS = ["popc", "mfma", "mfma-lds"]


@pytest.mark.parametrize("path,schedule", PATHS, ids=PATH_IDS)
@pytest.mark.parametrize("n,bits,K,nc,p", GRID)
def test_small_grid(path, schedule, n, bits, K, nc, p):
    codes = datagen.clustered_codes(n, bits, nc, p, seed=n * 7 + bits + K)
    want = oracle.knn_rows(codes, K)
    assert_same(gpu_knn(codes, K, path, schedule=schedule), want, f"n={n} bits={bits} K={K}")


@pytest.mark.parametrize("path,schedule", PATHS, ids=PATH_IDS)
@pytest.mark.parametrize("col_block,row_block", [(37, 0), (100, 333), (999, 64), (1, 2000)])
def test_blocking_does_not_change_the_graph(path, schedule, col_block, row_block):
    codes = datagen.clustered_codes(1500 if col_block > 1 else 200, 256, 15, 0.2, seed=21)
    want = oracle.knn_rows(codes, 24)
    got = gpu_knn(codes, 24, path, col_block=col_block, row_block=row_block, schedule=schedule)
    assert_same(got, want, f"col_block={col_block} row_block={row_block}")


@pytest.mark.parametrize("path", [POPC, MFMA], ids=["popc", "mfma"])
def test_golden_cube3(path):
    layouts, exp_idx, exp_dist = golden_io.cube3()
    for bits, positions, background in layouts:
        codes = golden_io.cube3_codes(bits, positions, background)
        got = gpu_knn(codes, 7, path)
        assert_same(got, (exp_idx, exp_dist), f"cube3 bits={bits}")


@pytest.mark.parametrize("path,schedule", PATHS, ids=PATH_IDS)
def test_tie_heavy_inputs(path, schedule):
    # all codes identical: every distance 0, neighbours are the smallest indices
    codes = np.tile(datagen.uniform_codes(1, 256, seed=5), (300, 1))
    assert_same(gpu_knn(codes, 50, path, schedule=schedule), oracle.knn_rows(codes, 50),
                "identical")
    # 10-cube: 1024 codes, distances 1..10 with binomial multiplicities
    rows = np.array([[(v >> t) & 1 for t in range(10)] + [0] * 118 for v in range(1024)],
                    dtype=np.uint8)
    codes = datagen.pack_bits(rows)
    for K in (10, 256):
        assert_same(gpu_knn(codes, K, path, schedule=schedule), oracle.knn_rows(codes, K),
                    f"cube10 K={K}")


def test_paths_agree_and_are_deterministic():
    codes = datagen.clustered_codes(5000, 256, 50, 0.2, seed=31)
    a = gpu_knn(codes, 64, POPC)
    b = gpu_knn(codes, 64, MFMA)
    assert_same(a, b, "popc vs mfma")
    for sc in (bdg.SCHEDULE_LDS_LISTS, bdg.SCHEDULE_DEEP_RING, bdg.SCHEDULE_GLOBAL_LISTS):
        assert_same(gpu_knn(codes, 64, MFMA, schedule=sc), a, f"mfma schedule {sc}")
    for cb in (5000, 1024, 333):
        assert_same(gpu_knn(codes, 64, MFMA, col_block=cb), a, f"mfma col_block={cb}")
        assert_same(gpu_knn(codes, 64, POPC, col_block=cb), a, f"popc col_block={cb}")


# ---------------------------------------------------- admission bounds

BOUND_CASES = [
    # n, bits, K, n_centres, p
    (3000, 256, 16, 30, 0.2),
    (5000, 512, 100, 25, 0.25),   # lists of 65..128: four waves of 48 rows
    (2000, 128, 200, 20, 0.15),   # lists of 129..256
    (2500, 192, 33, 1000, 0.2),   # clusters smaller than K: many rows without a bound
    (1200, 1024, 64, 12, 0.25),
    (700, 64, 8, 3, 0.3),
]


@pytest.mark.parametrize("n,bits,K,nc,p", BOUND_CASES)
def test_admission_bounds_keep_the_graph(n, bits, K, nc, p):
    codes = datagen.clustered_codes(n, bits, nc, p, seed=n + bits + K)
    want = oracle.knn_rows(codes, K)
    for group in (bdg.BOUND_OFF, 16, 64, bdg.BOUND_GROUP_DEFAULT, 4096, bdg.BOUND_GROUP_MAX):
        print(f"[bounds] n={n} bits={bits} K={K} group={group}", flush=True)
        assert_same(gpu_knn(codes, K, MFMA, bound_group=group), want, f"group={group}")
        if group in (64, bdg.BOUND_GROUP_DEFAULT):
            assert_same(gpu_knn(codes, K, MFMA, bound_group=group,
                                schedule=bdg.SCHEDULE_LDS_LISTS), want, f"group={group} lds")
        if group == 64:
            # several column blocks: the bound also holds for lists carried across them
            assert_same(gpu_knn(codes, K, MFMA, bound_group=group, col_block=n // 3 + 1), want,
                        f"group={group} col_block={n // 3 + 1}")


def test_admission_bounds_on_ties():
    # identical codes: every bound is 0, and the list is the smallest indices
    codes = np.tile(datagen.uniform_codes(1, 256, seed=5), (700, 1))
    for group in (16, bdg.BOUND_GROUP_DEFAULT):
        assert_same(gpu_knn(codes, 50, MFMA, bound_group=group), oracle.knn_rows(codes, 50),
                    f"identical group={group}")
    # 40 distinct codes repeated: ties at the bound decided by index
    g = np.random.default_rng(17)
    base = datagen.clustered_codes(40, 128, 4, 0.2, seed=9)
    codes = base[g.integers(0, 40, 3000)]
    for K in (30, 64, 150):
        assert_same(gpu_knn(codes, K, MFMA, bound_group=32), oracle.knn_rows(codes, K),
                    f"repeated K={K}")


# ------------------------------------- lists in global memory (schedule 2)

@pytest.mark.parametrize("n,bits,K,col_block", [
    (3000, 512, 100, 0), (3000, 512, 100, 700), (2600, 256, 65, 1000), (1100, 512, 128, 300),
    (257, 256, 128, 0),  # K near n: ragged last tile, padded rows
    (129, 512, 127, 50),
    (2000, 256, 64, 500), (1500, 512, 16, 0), (40, 256, 1, 0), (5, 512, 8, 0),
    (2300, 128, 100, 600), (385, 128, 32, 0),  # 128 bits; one row past a 384-row tile
])
def test_global_lists_schedule(n, bits, K, col_block):
    # the running lists stay keys in the output rows between column blocks;
    # the graph is the same as the oracle's, with and without admission bounds
    codes = datagen.clustered_codes(n, bits, max(2, n // 150), 0.2, seed=n + K + bits)
    want = oracle.knn_rows(codes, K)
    for group in (bdg.BOUND_OFF, 64, bdg.BOUND_GROUP_DEFAULT):
        print(f"[global lists] n={n} bits={bits} K={K} col_block={col_block} group={group}",
              flush=True)
        got = gpu_knn(codes, K, MFMA, schedule=bdg.SCHEDULE_GLOBAL_LISTS, col_block=col_block,
                      bound_group=group)
        assert_same(got, want, f"group={group}")


def test_autotune_tries_global_lists():
    # the build autotuner times schedule 2 where it is built; every candidate
    # gives the oracle's graph
    import json
    codes = datagen.clustered_codes(4000, 512, 30, 0.2, seed=41)
    want = oracle.knn_rows(codes, 100)
    d = dev(codes)
    opts, report = bdg.autotune_build(d, 100)
    cands = json.loads(report)["candidates"]
    assert bdg.SCHEDULE_GLOBAL_LISTS in {c["schedule"] for c in cands}
    for c in cands:
        print(f"[autotune] candidate {c}", flush=True)
        got = bdg.to_numpy_graph(*bdg.build_knn(d, 100, path=c["path"], col_block=c["col_block"],
                                                schedule=c["schedule"],
                                                bound_group=c["bound_group"]))
        assert_same(got, want, str(c))


def test_global_lists_schedule_not_everywhere():
    # built for 128, 256 and 512 bits with up to 128 keys
    codes = dev(datagen.uniform_codes(300, 512, seed=3))
    for bits, K in ((512, 129), (192, 100), (384, 60)):
        c = codes if bits == 512 else dev(datagen.uniform_codes(300, bits, seed=3))
        with pytest.raises(RuntimeError, match="schedule"):
            bdg.build_knn(c, K, path=MFMA, schedule=bdg.SCHEDULE_GLOBAL_LISTS)
    with pytest.raises(RuntimeError, match="schedule"):
        bdg.BatchPlan(np.array([0, 300], dtype=np.uint64), 384, 100,
                      schedule=bdg.SCHEDULE_GLOBAL_LISTS)


# ------------------------------------------------- long lists (K > 256)

@pytest.mark.parametrize("n,bits,K,col_block", [
    (1500, 256, 300, 0), (1200, 128, 600, 500), (1100, 64, 1000, 0), (2500, 512, 1024, 1000),
    (700, 192, 1024, 0),  # K > n - 1: padded rows
])
def test_long_lists_on_the_vector_alus(n, bits, K, col_block):
    # K up to 1024 runs on the vector-ALU path (path AUTO picks it beyond the
    # matrix-core tile's 256), with per-column-block lists merged when the
    # columns are split
    codes = datagen.clustered_codes(n, bits, max(2, n // 100), 0.2, seed=n + K)
    want = oracle.knn_rows(codes, K)
    print(f"[long lists] n={n} bits={bits} K={K} col_block={col_block}", flush=True)
    assert_same(gpu_knn(codes, K, POPC, col_block=col_block), want, f"K={K}")
    assert_same(gpu_knn(codes, K, bdg.PATH_AUTO), want, f"K={K} auto")


# ------------------------------------------------------ named workloads

def test_clustered_20k_128b_k32_full():
    """20,000 codes of 128 bits from 100 centres (flip 0.15), K = 32: every row."""
    w = datagen.WORKLOADS["clustered-20k-128b-k32"]
    codes = datagen.clustered_codes(w["n"], w["bits"], w["n_centres"], w["p"], w["seed"])
    want = oracle.knn_rows(codes, w["K"])
    for path in (POPC, MFMA):
        assert_same(gpu_knn(codes, w["K"], path), want, f"path={path}")


def test_clustered_1m_256b_k64_sampled():
    """1,000,000 codes of 256 bits from 1,000 centres (flip 0.2), K = 64, built in
    the benchmark's blocks (131,072 rows x 262,144 columns), merged across
    column blocks. Both paths agree on every row; the oracle checks 4,096
    seeded rows plus the row-tile and block edges and the ends."""
    w = datagen.WORKLOADS["clustered-1m-256b-k64"]
    codes = datagen.clustered_codes(w["n"], w["bits"], w["n_centres"], w["p"], w["seed"])
    K, n = w["K"], w["n"]
    kw = dict(row_block=w["row_block"], col_block=w["col_block"])
    a = gpu_knn(codes, K, MFMA, **kw)
    b = gpu_knn(codes, K, POPC, **kw)
    assert_same(a, b, "mfma vs popc")
    g = np.random.default_rng(99)
    cb = w["col_block"]
    edges = [0, 1, 255, 256, 131071, 131072, 131073, cb - 1, cb, 2 * cb - 1, n - cb, n - 257,
             n - 2, n - 1]
    rows = np.unique(np.concatenate([edges, g.choice(n, 4096, replace=False)])).astype(np.uint32)
    want = oracle.knn_rows(codes, K, rows=rows)
    assert_same((a[0][rows], a[1][rows]), want, "oracle rows")


@pytest.mark.timeout(900)
def test_clustered_1m_256b_k64_every_row():
    """The whole 1,000,000-row graph of the 1M x 256-bit workload (exact
    K = 64, built in the blocks the benchmark uses) equals the C oracle's on
    every row (about 1e12 pairs of oracle work: a few minutes of host CPU)."""
    w = datagen.WORKLOADS["clustered-1m-256b-k64"]
    codes = datagen.clustered_codes(w["n"], w["bits"], w["n_centres"], w["p"], w["seed"])
    got = gpu_knn(codes, w["K"], MFMA, row_block=w["row_block"], col_block=w["col_block"])
    n = w["n"]
    for part, rows in enumerate(np.array_split(np.arange(n, dtype=np.uint32), 8)):
        want = oracle.knn_rows(codes, w["K"], rows=rows)
        assert_same((got[0][rows], got[1][rows]), want, f"1M rows {rows[0]}..{rows[-1]}")
        print(f"[every-row] part {part + 1}/8 identical", flush=True)


def test_clustered_4m_512b_k100_sampled():
    """4,000,000 codes of 512 bits from 20,000 centres (flip 0.25), K = 100
    (the default schedule: lists kept in the output rows, row tiles of 384
    rows), built as the benchmark times it: one persistent launch over column
    blocks of 262,144. The vector-ALU
    path gives the same graph on every row; the oracle checks 4,096 seeded rows
    plus the row-tile and column-block edges and the ends."""
    import torch
    w = datagen.WORKLOADS["clustered-4m-512b-k100"]
    codes = datagen.clustered_codes(w["n"], w["bits"], w["n_centres"], w["p"], w["seed"])
    K, n, cb = w["K"], w["n"], w["col_block"]
    d = dev(codes)
    idx, dist = bdg.build_knn(d, K, path=MFMA, row_block=w["row_block"], col_block=cb)
    pi, pd = bdg.build_knn(d, K, path=POPC, row_block=w["row_block"], col_block=cb)
    torch.cuda.synchronize()
    assert torch.equal(idx, pi) and torch.equal(dist, pd), "matrix-core and vector-ALU graphs differ"
    del pi, pd
    g = np.random.default_rng(100)
    edges = [0, 1, 191, 192, 383, 384, cb - 1, cb, 2 * cb, n - cb, n - 385, n - 384, n - 193,
             n - 192, n - 1]
    rows = np.unique(np.concatenate([edges, g.choice(n, 4096, replace=False)])).astype(np.int64)
    sel = torch.from_numpy(rows).cuda()
    got = bdg.to_numpy_graph(idx[sel], dist[sel])
    want = oracle.knn_rows(codes, K, rows=rows.astype(np.uint32))
    assert_same(got, want, "4M x 512 bits, sampled rows")


# ----------------------------------------------------------------- merge

def test_merge_golden():
    import torch
    K, in_idx, in_dist, out_idx, out_dist = golden_io.merge_small()
    ti = torch.from_numpy(in_idx.view(np.int32)).cuda()
    td = torch.from_numpy(in_dist.view(np.int16)).cuda()
    got = bdg.to_numpy_graph(*bdg.merge_lists(ti, td, K))
    assert_same(got, (out_idx, out_dist), "merge golden")


@pytest.mark.parametrize("K_in,K", [(16, 16), (64, 32), (100, 100), (40, 128), (256, 256),
                                    (300, 500), (700, 1024)])
def test_merge_api_with_duplicates(K_in, K):
    import torch
    codes = datagen.clustered_codes(2000, 128, 25, 0.15, seed=K_in + K)
    bi, bd = oracle.knn_blocks(codes, K_in, col_block=450)
    # add repeated lists (a copy and a shifted copy of the same blocks)
    bi = np.concatenate([bi, bi[:2], bi[1:3]])
    bd = np.concatenate([bd, bd[:2], bd[1:3]])
    rows = np.arange(0, 2000, 13)
    want = oracle.merge_lists(bi[:, rows], bd[:, rows], K)
    ti = torch.from_numpy(np.ascontiguousarray(bi).view(np.int32)).cuda()
    td = torch.from_numpy(np.ascontiguousarray(bd).view(np.int16)).cuda()
    gi, gd = bdg.to_numpy_graph(*bdg.merge_lists(ti, td, K))
    assert_same((gi[rows], gd[rows]), want, "merge")


# ------------------------------------------------- driver: resume, workspace

def test_resume_by_row_blocks():
    import torch
    codes = datagen.clustered_codes(3000, 256, 30, 0.2, seed=41)
    K = 16
    want = gpu_knn(codes, K, MFMA, row_block=700, col_block=1000)
    d = dev(codes)
    idx = torch.full((3000, K), -7, dtype=torch.int32, device="cuda")
    dist = torch.full((3000, K), -7, dtype=torch.int16, device="cuda")
    for first, stop in ((0, 2), (2, 3), (3, 0)):
        o = bdg.make_opts(path=MFMA, row_block=700, col_block=1000, first_rowblock=first,
                          stop_rowblock=stop)
        assert bdg.bdg_build_knn_ex(d, 3000, 256, K, idx, dist, o, None) == 0
        if first == 0:
            torch.cuda.synchronize()
            part = bdg.to_numpy_graph(idx, dist)
            assert (part[0][1400:] == np.uint32(0xFFFFFFF9)).all()  # untouched beyond block 2
    torch.cuda.synchronize()
    assert_same(bdg.to_numpy_graph(idx, dist), want, "resumed")


def test_caller_workspace_and_alloc_failure():
    import torch
    codes = datagen.clustered_codes(2500, 128, 25, 0.15, seed=43)
    K = 20
    want = oracle.knn_rows(codes, K)
    d = dev(codes)
    o = bdg.make_opts(col_block=600)
    need = bdg.bdg_build_knn_workspace_size(2500, 128, K, o)
    assert need > 0
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    o.workspace, o.workspace_bytes = ws.data_ptr(), need
    idx = torch.empty((2500, K), dtype=torch.int32, device="cuda")
    dist = torch.empty((2500, K), dtype=torch.int16, device="cuda")
    assert bdg.bdg_build_knn_ex(d, 2500, 128, K, idx, dist, o, None) == 0
    torch.cuda.synchronize()
    assert_same(bdg.to_numpy_graph(idx, dist), want, "caller workspace")
    # too small a workspace -> ENOMEM, outputs untouched
    o.workspace_bytes = need - 1
    idx.fill_(5)
    assert bdg.bdg_build_knn_ex(d, 2500, 128, K, idx, dist, o, None) == bdg.BDG_ENOMEM
    # forced allocation failure -> ENOMEM, outputs untouched
    os.environ["BDG_TEST_FAIL_ALLOC"] = "1"
    try:
        o2 = bdg.make_opts(col_block=600)
        assert bdg.bdg_build_knn_ex(d, 2500, 128, K, idx, dist, o2, None) == bdg.BDG_ENOMEM
        assert bdg.bdg_build_knn(d, 2500, 128, K, idx, dist) == bdg.BDG_ENOMEM
    finally:
        del os.environ["BDG_TEST_FAIL_ALLOC"]
    torch.cuda.synchronize()
    assert (idx.cpu().numpy() == 5).all()


@pytest.mark.parametrize("schedule", [bdg.SCHEDULE_DEFAULT, bdg.SCHEDULE_LDS_LISTS],
                         ids=["default", "lds"])
@pytest.mark.parametrize("n,bits,K,col_block", [
    (1500, 256, 24, 37),    # 6 tiles (4 of 384 rows) x 41 column blocks: chains of 41 items
    (2000, 512, 100, 300),  # tiles of 192 (384) rows, lists of 128 keys
    (700, 64, 8, 5000),     # one column block: no item waits
])
def test_sweep_control_words(n, bits, K, col_block, schedule):
    # The matrix-core build is one persistent launch over (row tile, column
    # block) items. Besides the graph, its control words at the end of the
    # workspace show that every item ran once and no dependency wait ran out:
    # claim counter = items + work-groups (each work-group's last claim finds
    # the list empty), stall flag 0, every tile's progress = column blocks.
    import torch
    codes = datagen.clustered_codes(n, bits, 12, 0.2, seed=n + bits + K)
    want = oracle.knn_rows(codes, K)
    o = bdg.make_opts(path=MFMA, col_block=col_block, tile_schedule=schedule)
    need = bdg.bdg_build_knn_workspace_size(n, bits, K, o)
    ws = torch.zeros(need, dtype=torch.uint8, device="cuda")
    o.workspace, o.workspace_bytes = ws.data_ptr(), need
    idx = torch.empty((n, K), dtype=torch.int32, device="cuda")
    dist = torch.empty((n, K), dtype=torch.int16, device="cuda")
    assert bdg.bdg_build_knn_ex(dev(codes), n, bits, K, idx, dist, o, None) == 0
    torch.cuda.synchronize()
    assert_same(bdg.to_numpy_graph(idx, dist), want, f"sweep n={n} col_block={col_block}")
    # tiles of 384 rows where the default resolves to the global-lists schedule
    gl = schedule == bdg.SCHEDULE_DEFAULT and bits in (128, 256, 512) and K <= 128
    rt = 384 if gl else (256 if K <= 64 else 192)
    ntiles = -(-n // rt)
    ncb = -(-n // col_block)
    off = ((((n + 15) // 16 * 16 + 256) * bits) + 255) // 256 * 256
    ctl = ws[off:off + 4 * (ntiles + 2)].cpu().numpy().view(np.uint32)
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    assert ctl[0] == ntiles * ncb + min(cus, ntiles * ncb)
    assert ctl[1] == 0
    assert (ctl[2:] == ncb).all()


def test_sync_entry_point():
    import torch
    codes = datagen.clustered_codes(900, 192, 9, 0.2, seed=47)
    d = dev(codes)
    idx = torch.empty((900, 12), dtype=torch.int32, device="cuda")
    dist = torch.empty((900, 12), dtype=torch.int16, device="cuda")
    assert bdg.bdg_build_knn(d, 900, 192, 12, idx, dist) == 0
    assert_same(bdg.to_numpy_graph(idx, dist), oracle.knn_rows(codes, 12), "sync")


def test_check_reports_a_wait_that_gave_up():
    # The persistent build's dependency waits are bounded. Forced from the host
    # to give up after one poll on a build with many dependent items, some
    # wait gives up: every kernel still exits, and the async build's outcome
    # query reports BDG_EDEVICE. The default bound is never reached, and a
    # build with one column block has no waits at all.
    import torch
    n, bits, K = 3000, 256, 16
    codes = datagen.clustered_codes(n, bits, 12, 0.2, seed=61)
    d = dev(codes)
    idx = torch.empty((n, K), dtype=torch.int32, device="cuda")
    dist = torch.empty((n, K), dtype=torch.int16, device="cuda")
    for col_block, limit, want in ((40, 1, bdg.BDG_EDEVICE), (40, 0, bdg.BDG_OK),
                                   (5000, 1, bdg.BDG_OK)):
        o = bdg.make_opts(path=MFMA, col_block=col_block, wait_limit=limit)
        need = bdg.bdg_build_knn_workspace_size(n, bits, K, o)
        ws = torch.empty(need, dtype=torch.uint8, device="cuda")
        o.workspace, o.workspace_bytes = ws.data_ptr(), need
        print(f"[check] col_block={col_block} wait_limit={limit}", flush=True)
        assert bdg.bdg_build_knn_ex(d, n, bits, K, idx, dist, o, None) == 0
        assert bdg.bdg_build_knn_check(n, bits, K, o, None) == want, bdg.last_error()
        if want == bdg.BDG_OK:
            assert_same(bdg.to_numpy_graph(idx, dist), oracle.knn_rows(codes, K),
                        f"col_block={col_block}")


# ------------------------------------------- queries against a base set

@pytest.mark.parametrize("nq,nb,bits,K", [
    (1000, 3000, 256, 32), (777, 5001, 512, 64), (300, 40, 128, 50),  # nb < K: padding
    (129, 1, 64, 8), (2048, 20000, 1024, 16), (65, 700, 192, 1),
])
def test_hamming_knn_against_a_base(nq, nb, bits, K):
    g = np.random.default_rng(nq + nb)
    base = datagen.clustered_codes(nb, bits, max(1, nb // 100), 0.2, seed=nq + bits)
    # queries: fresh codes of the same clusters, and some rows of the base itself
    queries = datagen.clustered_codes(nq, bits, max(1, nb // 100), 0.2, seed=nq + bits)
    queries[::7] = base[g.integers(0, nb, queries[::7].shape[0])]
    want = oracle.knn_rect(queries, base, K)
    print(f"[hamming knn] nq={nq} nb={nb} bits={bits} K={K}", flush=True)
    got = bdg.hamming_knn(dev(queries), dev(base), K)
    import torch
    torch.cuda.synchronize()
    assert_same(bdg.to_numpy_graph(*got), want, f"nq={nq} nb={nb}")


def test_hamming_knn_empty_base_and_ties():
    import torch
    queries = datagen.uniform_codes(70, 256, seed=3)
    base = np.zeros((0, 4), dtype=np.uint64)
    gi, gd = bdg.to_numpy_graph(*bdg.hamming_knn(dev(queries), dev(base), 5, bits=256))
    assert (gi == 0xFFFFFFFF).all() and (gd == 0xFFFF).all()
    # identical base codes: every distance equal, neighbours are the smallest indices
    base = np.tile(datagen.uniform_codes(1, 256, seed=4), (500, 1))
    got = bdg.hamming_knn(dev(queries), dev(base), 40)
    torch.cuda.synchronize()
    assert_same(bdg.to_numpy_graph(*got), oracle.knn_rect(queries, base, 40), "ties")
