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

__device__ __forceinline__ uint32_t umin32(uint32_t a, uint32_t b) { return a < b ? a : b; }
__device__ __forceinline__ uint32_t umax32(uint32_t a, uint32_t b) { return a < b ? b : a; }

// x of lane (lane ^ M), M a power of two below 64. Masks inside a row of 16
// lanes use DPP moves (quad permutes for 1 and 2; a row shift each way and a
// select for 4 and 8); 16 and 32 use the row and half-wave swaps of gfx950
// (v_permlane16_swap / v_permlane32_swap: the exchange stays in the vector
// ALU, with no LDS round trip) and a select.
template <int M>
__device__ __forceinline__ uint32_t xshfl(uint32_t x, uint32_t lane) {
  if constexpr (M == 1) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0xB1, 0xF, 0xF, false);
  } else if constexpr (M == 2) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x4E, 0xF, 0xF, false);
  } else if constexpr (M == 4 || M == 8) {
    const uint32_t up = (uint32_t)__builtin_amdgcn_update_dpp((int)x, (int)x, 0x100 + M, 0xF, 0xF,
                                                              false);  // lane i <- i + M
    const uint32_t dn = (uint32_t)__builtin_amdgcn_update_dpp((int)x, (int)x, 0x110 + M, 0xF, 0xF,
                                                              false);  // lane i <- i - M
    return (lane & M) ? dn : up;
  } else if constexpr (M == 16) {
    // [0] = odd rows replaced by the even rows, [1] = even rows by the odd
    const auto s = __builtin_amdgcn_permlane16_swap(x, x, false, false);
    return (lane & 16) ? (uint32_t)s[0] : (uint32_t)s[1];
  } else {
    static_assert(M == 32, "xor mask");
    // [0] = upper half replaced by the lower, [1] = lower half by the upper
    const auto r = __builtin_amdgcn_permlane32_swap(x, x, false, false);
    return (lane & 32) ? (uint32_t)r[0] : (uint32_t)r[1];
  }
}

__device__ __forceinline__ uint32_t shfl_xor_u32(uint32_t x, int m) {
  return (uint32_t)__shfl_xor((int)x, m, kWave);
}

// One compare-exchange stage of a bitonic network over one key per lane:
// keep the min if `take_min`, else the max, of x and the key of lane ^ J.
template <int J>
__device__ __forceinline__ uint32_t cx_stage(uint32_t x, uint32_t lane, bool take_min) {
  const uint32_t y = xshfl<J>(x, lane);
  return take_min ? umin32(x, y) : umax32(x, y);
}

__device__ __forceinline__ uint32_t shfl_u32(uint32_t x, int src) {
  return (uint32_t)__shfl((int)x, src, kWave);
}


// Bitonic sort of one key per lane across the wave (ascending, or descending
// with DESC: every comparison direction flipped).
template <int K2, int J, bool DESC>
__device__ __forceinline__ uint32_t sort_steps(uint32_t x, uint32_t lane) {
  const bool up = ((lane & K2) == 0) != DESC;
  const bool lower = (lane & J) == 0;
  x = cx_stage<J>(x, lane, lower == up);
  if constexpr (J > 1) return sort_steps<K2, J / 2, DESC>(x, lane);
  return x;
}

template <bool DESC = false>
__device__ __forceinline__ uint32_t wave_sort64(uint32_t x, uint32_t lane) {
  x = sort_steps<2, 1, DESC>(x, lane);
  x = sort_steps<4, 2, DESC>(x, lane);
  x = sort_steps<8, 4, DESC>(x, lane);
  x = sort_steps<16, 8, DESC>(x, lane);
  x = sort_steps<32, 16, DESC>(x, lane);
  x = sort_steps<64, 32, DESC>(x, lane);
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
  for (int r = 0; r < NR; ++r) {
    R[r] = cx_stage<32>(R[r], lane, (lane & 32) == 0);
    R[r] = cx_stage<16>(R[r], lane, (lane & 16) == 0);
    R[r] = cx_stage<8>(R[r], lane, (lane & 8) == 0);
    R[r] = cx_stage<4>(R[r], lane, (lane & 4) == 0);
    R[r] = cx_stage<2>(R[r], lane, (lane & 2) == 0);
    R[r] = cx_stage<1>(R[r], lane, (lane & 1) == 0);
  }
}

// Up to 32 keys held by lanes 32..63 (lanes 0..31 hold kKeyNone) sorted into
// a descending sequence over the whole wave: the bitonic network of 32-lane
// blocks only, whose last stage runs the upper block downwards.
__device__ __forceinline__ uint32_t wave_sort_upper32_desc(uint32_t x, uint32_t lane) {
  x = sort_steps<2, 1, false>(x, lane);
  x = sort_steps<4, 2, false>(x, lane);
  x = sort_steps<8, 4, false>(x, lane);
  x = sort_steps<16, 8, false>(x, lane);
  x = sort_steps<32, 16, false>(x, lane);
  return x;
}

// The sorted list of one query as NR rows of 64 keys (kKeyNone past K).
template <int NR>
__device__ __forceinline__ void load_list(const uint32_t* list_q, uint32_t (&R)[NR], uint32_t K,
                                          uint32_t lane) {
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    uint32_t p = r * kWave + lane;
    R[r] = (p < K) ? list_q[p] : kKeyNone;
  }
}

// Merge 64 new keys given as a descending sequence over the lanes (kKeyNone
// for none) into the sorted list of one query, already loaded as R
// (wave-wide; every lane must call it with the same list). Returns the new
// K-th key (kKeyNone while the list is not full).
template <int NR>
__device__ __forceinline__ uint32_t merge_desc_with(uint32_t* list_q, uint32_t (&R)[NR], uint32_t xr,
                                                    uint32_t K, uint32_t lane) {
  // min(list[i], new_padded[N-1-i]) keeps the N smallest of the union as a
  // bitonic sequence; only the last 64 positions meet real new keys.
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

// Merge up to 64 new keys (one per lane, any order, kKeyNone for none) into
// the sorted list of one query.
template <int NR>
__device__ __forceinline__ uint32_t merge_into_list(uint32_t* list_q, uint32_t x, uint32_t K,
                                                    uint32_t lane) {
  uint32_t R[NR];
  load_list<NR>(list_q, R, K, lane);
  return merge_desc_with<NR>(list_q, R, wave_sort64<true>(x, lane), K, lane);
}

// Merge the c pending keys buf_q[0..c) of one query into its list.
template <int NR, int B>
__device__ __forceinline__ uint32_t flush_query(uint32_t* list_q, const uint32_t* buf_q,
                                                uint32_t c, uint32_t K, uint32_t lane) {
  static_assert(B <= kWave, "buffer holds at most one key per lane");
  const uint32_t x = (lane < c) ? buf_q[lane] : kKeyNone;
  return merge_into_list<NR>(list_q, x, K, lane);
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
