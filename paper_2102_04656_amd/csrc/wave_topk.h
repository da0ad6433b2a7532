// Wave-level exact top-K selection for the Hamming kNN tiles (gfx950).
//
// A wave owns Q queries (rows). For each query it keeps, in LDS,
//   list[q][0..K)  the K smallest keys seen so far, ascending;
//   buf[q][0..B)   keys that beat the query's threshold but are not merged yet;
//   cnt[q]         how many keys buf[q] holds.
// A key packs (distance, column) as  dist << IDX_BITS | (column - block start),
// so unsigned key order is the (distance, index) order of the graph rows.
//
// Columns are scanned in increasing index order, so a new candidate can only
// displace the current K-th key if its distance is strictly smaller: the
// threshold test is `dist < thr`, thr = distance of list[q][K-1] (or "none"
// while the list is not full). Passing candidates are appended to buf; when a
// buffer may overflow, the whole wave merges it into the list: a bitonic sort
// of the buffer across the 64 lanes, then the bitonic merge of the sorted
// buffer with the list. Flushes are rare once the threshold is tight.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bdg {

constexpr int kWave = 64;
constexpr uint32_t kKeyNone = 0xFFFFFFFFu;
constexpr int kIdxBits = 21;  // column-block index field: blocks of <= 2^21 columns
constexpr uint32_t kIdxMask = (1u << kIdxBits) - 1u;
constexpr uint32_t kDistNone = 0x7FFFu;  // threshold while a list is not full

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

__device__ __forceinline__ uint32_t shfl_xor_u32(uint32_t x, int m) {
  return (uint32_t)__shfl_xor((int)x, m, kWave);
}

__device__ __forceinline__ uint32_t shfl_u32(uint32_t x, int src) {
  return (uint32_t)__shfl((int)x, src, kWave);
}

__device__ __forceinline__ uint32_t umin32(uint32_t a, uint32_t b) { return a < b ? a : b; }
__device__ __forceinline__ uint32_t umax32(uint32_t a, uint32_t b) { return a < b ? b : a; }

// Ascending bitonic sort of one key per lane across the wave.
__device__ __forceinline__ uint32_t wave_sort64(uint32_t x, uint32_t lane) {
#pragma unroll
  for (int k = 2; k <= kWave; k <<= 1) {
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1) {
      uint32_t y = shfl_xor_u32(x, j);
      bool up = (lane & k) == 0;
      bool lower = (lane & j) == 0;
      x = (lower == up) ? umin32(x, y) : umax32(x, y);
    }
  }
  return x;
}

// Ascending bitonic merge of a bitonic sequence of 64*NR keys held as
// seq[64 r + lane] = R[r].
template <int NR>
__device__ __forceinline__ void wave_bitonic_merge(uint32_t (&R)[NR], uint32_t lane) {
#pragma unroll
  for (int j = NR / 2; j >= 1; j >>= 1) {
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      if ((r & j) == 0) {
        uint32_t a = R[r], b = R[r + j];
        R[r] = umin32(a, b);
        R[r + j] = umax32(a, b);
      }
    }
  }
#pragma unroll
  for (int j = kWave / 2; j >= 1; j >>= 1) {
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      uint32_t y = shfl_xor_u32(R[r], j);
      R[r] = (lane & j) ? umax32(R[r], y) : umin32(R[r], y);
    }
  }
}

// Merge the c pending keys of one query into its sorted list (wave-wide; every
// lane must call it with the same arguments). Returns the new K-th key.
template <int NR, int B>
__device__ __forceinline__ uint32_t flush_query(uint32_t* list_q, const uint32_t* buf_q,
                                                uint32_t c, uint32_t K, uint32_t lane) {
  static_assert(B <= kWave, "buffer holds at most one key per lane");
  uint32_t x = (lane < c) ? buf_q[lane] : kKeyNone;
  x = wave_sort64(x, lane);
  uint32_t xr = shfl_u32(x, kWave - 1 - lane);  // buffer descending
  uint32_t R[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    uint32_t p = r * kWave + lane;
    R[r] = (p < K) ? list_q[p] : kKeyNone;
  }
  // min(list[i], buf_padded[N-1-i]) keeps the N smallest of the union as a
  // bitonic sequence; only the last 64 positions meet real buffer keys.
  R[NR - 1] = umin32(R[NR - 1], xr);
  wave_bitonic_merge<NR>(R, lane);
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    uint32_t p = r * kWave + lane;
    if (p < K) list_q[p] = R[r];
  }
  const uint32_t last = K - 1;
  uint32_t kth = kKeyNone;
#pragma unroll
  for (int r = 0; r < NR; ++r)
    if ((last >> 6) == (uint32_t)r) kth = __builtin_amdgcn_readlane(R[r], last & 63);
  return kth;
}

__device__ __forceinline__ uint32_t key_dist(uint32_t key) {
  return key == kKeyNone ? kDistNone : (key >> kIdxBits);
}

// Write the lists of the wave's queries as (global index, distance) rows.
//   nq      queries owned by the wave; query q is output row (row_out0 + q)
//   nvalid  queries that exist (q < nvalid)
__device__ __forceinline__ void write_lists(const uint32_t* list, uint32_t nq, uint32_t nvalid,
                                            uint32_t K, uint32_t col_base, uint32_t* out_idx,
                                            uint16_t* out_dist, size_t row_out0, uint32_t lane) {
  for (uint32_t q = 0; q < nq && q < nvalid; ++q) {
    const uint32_t* lq = list + (size_t)q * K;
    size_t o = (row_out0 + q) * (size_t)K;
    for (uint32_t p = lane; p < K; p += kWave) {
      uint32_t key = lq[p];
      bool none = key == kKeyNone;
      out_idx[o + p] = none ? 0xFFFFFFFFu : col_base + (key & kIdxMask);
      out_dist[o + p] = none ? (uint16_t)0xFFFFu : (uint16_t)(key >> kIdxBits);
    }
  }
}

}  // namespace bdg
