// Wave-level bitonic sort and merge of 64-bit keys (one key per lane), for
// lists whose keys do not fit 32 bits: (distance << 32 | index) of the list
// merge, and (float distance bits << 32 | index) of the real-valued kNN.
// Unsigned key order is the (distance, index) order; ~0 is "no entry".
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "wave_topk.h"

namespace bdg {

constexpr uint64_t kNone64 = ~0ull;

template <int M>
__device__ __forceinline__ uint64_t xshfl64(uint64_t x, uint32_t lane) {
  const uint32_t lo = xshfl<M>((uint32_t)x, lane);
  const uint32_t hi = xshfl<M>((uint32_t)(x >> 32), lane);
  return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint64_t umin64(uint64_t a, uint64_t b) { return a < b ? a : b; }
__device__ __forceinline__ uint64_t umax64(uint64_t a, uint64_t b) { return a < b ? b : a; }

template <int J>
__device__ __forceinline__ uint64_t cx64(uint64_t x, uint32_t lane, bool take_min) {
  const uint64_t y = xshfl64<J>(x, lane);
  return take_min ? umin64(x, y) : umax64(x, y);
}

template <int K2, int J, bool DESC>
__device__ __forceinline__ uint64_t sort64_steps(uint64_t x, uint32_t lane) {
  const bool up = ((lane & K2) == 0) != DESC;
  x = cx64<J>(x, lane, ((lane & J) == 0) == up);
  if constexpr (J > 1) return sort64_steps<K2, J / 2, DESC>(x, lane);
  return x;
}

// Bitonic sort of one 64-bit key per lane (ascending, or descending).
template <bool DESC = false>
__device__ __forceinline__ uint64_t wave_sort64_u64(uint64_t x, uint32_t lane) {
  x = sort64_steps<2, 1, DESC>(x, lane);
  x = sort64_steps<4, 2, DESC>(x, lane);
  x = sort64_steps<8, 4, DESC>(x, lane);
  x = sort64_steps<16, 8, DESC>(x, lane);
  x = sort64_steps<32, 16, DESC>(x, lane);
  x = sort64_steps<64, 32, DESC>(x, lane);
  return x;
}

// R (64 NR keys, ascending, seq[64 r + lane] = R[r]) <- the 64 NR smallest of
// R and up to 64 new keys x (one per lane, any order).
template <int NR>
__device__ __forceinline__ void merge64_into(uint64_t (&R)[NR], uint64_t x, uint32_t lane) {
  const uint64_t xr = wave_sort64_u64<true>(x, lane);  // descending
  R[NR - 1] = umin64(R[NR - 1], xr);  // the union's smallest, as a bitonic sequence
#pragma unroll
  for (int j = NR / 2; j >= 1; j >>= 1) {
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      if ((r & j) == 0) {
        const uint64_t a = R[r], b = R[r + j];
        R[r] = umin64(a, b);
        R[r + j] = umax64(a, b);
      }
    }
  }
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    R[r] = cx64<32>(R[r], lane, (lane & 32) == 0);
    R[r] = cx64<16>(R[r], lane, (lane & 16) == 0);
    R[r] = cx64<8>(R[r], lane, (lane & 8) == 0);
    R[r] = cx64<4>(R[r], lane, (lane & 4) == 0);
    R[r] = cx64<2>(R[r], lane, (lane & 2) == 0);
    R[r] = cx64<1>(R[r], lane, (lane & 1) == 0);
  }
}

}  // namespace bdg
