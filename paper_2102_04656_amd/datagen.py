"""Seeded synthetic inputs for the Hamming kNN-graph builder and for its checks.

This module holds none of the method's arithmetic. It only draws random numbers
and lays them out in the library's input layout, so that the GPU path and the
CPU oracle can consume the very same host arrays.

Code layout (the packed code matrix): a code of ``bits`` bits is stored as
``bits // 64`` little-endian ``uint64`` words; bit ``j`` of the code is bit
``j % 64`` of word ``j // 64``. Rows are codes, row-major, ``[n][bits // 64]``.

Every generator uses ``numpy.random.Generator(PCG64(seed))`` and consumes the
stream in a fixed order (documented per function), so the arrays are a pure
function of the arguments.

The paper measures on proprietary image collections encoded to 512-bit codes
(Sec. 4.1, Table 1). Those are not available; the clustered generators below
stand in for them with the paper's code lengths and with the cluster structure
that the divide-and-conquer step (Sec. 3.2) is built around.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "make_rng",
    "pack_bits",
    "unpack_bits",
    "clustered_codes",
    "uniform_codes",
    "sharded_codes",
    "gmm_features",
    "gaussian_projection",
    "WORKLOADS",
]

# Rows generated per chunk. Part of the recipe: the flip draws are consumed
# chunk by chunk in row order.
_CHUNK = 65536


def make_rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def pack_bits(bits01: np.ndarray) -> np.ndarray:
    """``[n][b]`` array of 0/1 (any integer dtype) -> ``[n][b // 64]`` uint64."""
    bits01 = np.ascontiguousarray(bits01, dtype=np.uint8)
    n, b = bits01.shape
    if b % 64:
        raise ValueError("bit count must be a multiple of 64")
    packed = np.packbits(bits01, axis=1, bitorder="little")
    return np.ascontiguousarray(packed).view("<u8").reshape(n, b // 64)


def unpack_bits(codes: np.ndarray) -> np.ndarray:
    """``[n][W]`` uint64 -> ``[n][64 W]`` uint8 of 0/1 (inverse of pack_bits)."""
    codes = np.ascontiguousarray(codes, dtype="<u8")
    n, w = codes.shape
    return np.unpackbits(codes.view(np.uint8).reshape(n, 8 * w), axis=1,
                         bitorder="little")


def clustered_codes(n: int, bits: int, n_centres: int, p: float, seed: int) -> np.ndarray:
    """Codes drawn around random binary centres.

    Stream order: centres ``[n_centres][bits]`` as integers in {0, 1}; then one
    centre index per point, uniform; then, chunk by chunk in row order, a
    ``float32`` uniform per (point, bit); a bit of the centre is flipped when
    its uniform is below ``p``.
    """
    g = make_rng(seed)
    centres = pack_bits(g.integers(0, 2, size=(n_centres, bits), dtype=np.uint8))
    assign = g.integers(0, n_centres, size=n)
    out = np.empty((n, bits // 64), dtype=np.uint64)
    for r0 in range(0, n, _CHUNK):
        r1 = min(n, r0 + _CHUNK)
        flips = g.random((r1 - r0, bits), dtype=np.float32) < np.float32(p)
        out[r0:r1] = centres[assign[r0:r1]] ^ pack_bits(flips)
    return out


def uniform_codes(n: int, bits: int, seed: int) -> np.ndarray:
    """Independent uniform codes (every bit a fair coin)."""
    g = make_rng(seed)
    return g.integers(0, np.iinfo(np.uint64).max, size=(n, bits // 64),
                      dtype=np.uint64, endpoint=True)


def shard_sizes(n_shards: int, lo: int, hi: int, seed: int):
    """Shard sizes log-uniform in [lo, hi] and centres per shard (first draws
    of the sharded workload's stream)."""
    g = make_rng(seed)
    sizes = np.rint(np.exp(g.uniform(np.log(lo), np.log(hi), size=n_shards))).astype(np.int64)
    return g, sizes


def sharded_codes(n_shards: int = 512, lo: int = 2000, hi: int = 200_000,
                  c_lo: int = 10, c_hi: int = 500, bits: int = 256, p: float = 0.2,
                  seed: int = 3):
    """Many independent partitions of uneven size, each with its own centres.

    Stream order: ``n_shards`` log-uniform sizes, ``n_shards`` centre counts
    uniform in ``[c_lo, c_hi]``; then per shard in order: its centres, its
    assignment, its flips (as in ``clustered_codes``, chunked per shard).

    Returns ``(codes [sum n_s][bits/64] uint64, offsets [n_shards + 1] uint64)``.
    """
    g, sizes = shard_sizes(n_shards, lo, hi, seed)
    ncent = g.integers(c_lo, c_hi + 1, size=n_shards)
    offsets = np.zeros(n_shards + 1, dtype=np.uint64)
    offsets[1:] = np.cumsum(sizes)
    total = int(offsets[-1])
    out = np.empty((total, bits // 64), dtype=np.uint64)
    for s in range(n_shards):
        ns, base = int(sizes[s]), int(offsets[s])
        centres = pack_bits(g.integers(0, 2, size=(int(ncent[s]), bits), dtype=np.uint8))
        assign = g.integers(0, int(ncent[s]), size=ns)
        for r0 in range(0, ns, _CHUNK):
            r1 = min(ns, r0 + _CHUNK)
            flips = g.random((r1 - r0, bits), dtype=np.float32) < np.float32(p)
            out[base + r0: base + r1] = centres[assign[r0:r1]] ^ pack_bits(flips)
    return out, offsets


def gmm_features(n: int = 1_000_000, d: int = 512, n_comp: int = 1000,
                 centre_std: float = 2.0, seed: int = 5) -> np.ndarray:
    """Isotropic Gaussian mixture: x = mu_z + N(0, I), mu_k ~ N(0, centre_std^2 I),
    z uniform over components. float32 ``[n][d]``.

    Stream order: centres, component per point, then the unit noise in row
    chunks.
    """
    g = make_rng(seed)
    mu = g.standard_normal((n_comp, d), dtype=np.float32) * np.float32(centre_std)
    z = g.integers(0, n_comp, size=n)
    x = np.empty((n, d), dtype=np.float32)
    for r0 in range(0, n, _CHUNK):
        r1 = min(n, r0 + _CHUNK)
        x[r0:r1] = mu[z[r0:r1]] + g.standard_normal((r1 - r0, d), dtype=np.float32)
    return x


def gaussian_projection(d: int = 512, bits: int = 256, seed: int = 6) -> np.ndarray:
    """Random projection matrix ``[d][bits]`` float32 with N(0, 1) entries."""
    g = make_rng(seed)
    return g.standard_normal((d, bits), dtype=np.float32)


# The named workloads (sizes, seeds, parameters). ``scale`` in the test suite
# shrinks n while keeping the structure.
WORKLOADS = {
    "clustered-20k-128b-k32": dict(n=20_000, bits=128, n_centres=100, p=0.15, seed=1, K=32),
    "clustered-1m-256b-k64": dict(n=1_000_000, bits=256, n_centres=1000, p=0.2, seed=2, K=64,
                                  row_block=131072, col_block=262144),
    "sharded-512x-256b-k32": dict(n_shards=512, lo=2000, hi=200_000, c_lo=10, c_hi=500,
                                  bits=256, p=0.2, seed=3, K=32),
    "clustered-4m-512b-k100": dict(n=4_000_000, bits=512, n_centres=20_000, p=0.25, seed=4,
                                   K=100, row_block=250_000, col_block=262144),
    "gmm-1m-512d": dict(n=1_000_000, d=512, n_comp=1000, centre_std=2.0, seed=5,
                        proj_seed=6, code_bits=256, K_train=32, K_eval=64,
                        train_rows=100_000, eval_queries=10_000),
}
