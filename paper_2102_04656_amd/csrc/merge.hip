// Merge of per-row neighbour lists: the second reduce of the single-pass
// divide-and-conquer gathers all partial kNN lists of one label and sorts out
// the final kNN (Sec. 3.2); propagation merge-sorts its candidates the same
// way (Sec. 3.3).
//
// One wave per row. The running result R (64*NR keys, ascending) starts
// empty; every sorted input chunk of 64 entries x is merged in with
//   R[i] = min(R[i], x_padded[N-1-i]),  then a bitonic merge of R,
// which keeps the N smallest of R and x. Keys are dist << 32 | idx, so the
// sentinel entry (0xFFFF, 0xFFFFFFFF) is the largest key.
// With dedup, entries of x already in R (binary search of R in LDS) and
// repeats inside x are dropped before the merge.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.h"
#include "wave_topk64.h"

namespace bdg {

namespace {

constexpr int kW = 64;

template <int NR>
__global__ __launch_bounds__(256) void merge_lists_kernel(const uint32_t* __restrict__ in_idx,
                                                          const uint16_t* __restrict__ in_dist,
                                                          uint32_t n, uint32_t L, uint32_t K_in,
                                                          uint32_t K, uint32_t* __restrict__ out_idx,
                                                          uint16_t* __restrict__ out_dist,
                                                          int dedup) {
  __shared__ uint64_t lds[4][kW * NR];
  const uint32_t wave = threadIdx.x >> 6;
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t row = blockIdx.x * 4 + wave;
  if (row >= n) return;  // wave-uniform
  uint64_t* Rl = lds[wave];
  constexpr uint32_t N = kW * NR;

  uint64_t R[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) R[r] = kNone64;

  for (uint32_t l = 0; l < L; ++l) {
    const size_t base = ((size_t)l * n + row) * K_in;
    for (uint32_t c0 = 0; c0 < K_in; c0 += kW) {
      const uint32_t p = c0 + lane;
      uint64_t x = kNone64;
      if (p < K_in) {
        const uint32_t idx = in_idx[base + p];
        const uint16_t d = in_dist[base + p];
        x = (idx == 0xFFFFFFFFu) ? kNone64 : (((uint64_t)d << 32) | idx);
      }
      if (dedup) {
#pragma unroll
        for (int r = 0; r < NR; ++r) Rl[r * kW + lane] = R[r];
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        bool drop = false;
        if (x != kNone64) {
          // lower bound of x in R (ascending, N entries)
          uint32_t lo = 0, hi = N;
          while (lo < hi) {
            uint32_t mid = (lo + hi) >> 1;
            if (Rl[mid] < x) lo = mid + 1; else hi = mid;
          }
          drop = lo < N && Rl[lo] == x;
        }
        const uint64_t prev =
            ((uint64_t)(uint32_t)__shfl((int)(uint32_t)(x >> 32), lane == 0 ? 0 : (int)lane - 1,
                                        kW) << 32) |
            (uint32_t)__shfl((int)(uint32_t)x, lane == 0 ? 0 : (int)lane - 1, kW);
        if (lane > 0 && prev == x) drop = true;
        if (__any(drop)) {
          if (drop) x = kNone64;
          x = wave_sort64_u64(x, lane);
        }
        __builtin_amdgcn_wave_barrier();
      }
      merge64_into<NR>(R, x, lane);
    }
  }
  const size_t o = (size_t)row * K;
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const uint32_t p = r * kW + lane;
    if (p < K) {
      const uint64_t key = R[r];
      out_idx[o + p] = key == kNone64 ? 0xFFFFFFFFu : (uint32_t)key;
      out_dist[o + p] = key == kNone64 ? (uint16_t)0xFFFFu : (uint16_t)(key >> 32);
    }
  }
}

}  // namespace

hipError_t launch_merge(const uint32_t* in_idx, const uint16_t* in_dist, uint32_t n, uint32_t L,
                        uint32_t K_in, uint32_t K, uint32_t* out_idx, uint16_t* out_dist,
                        int dedup, hipStream_t stream) {
  if (n == 0) return hipSuccess;
  dim3 grid((n + 3) / 4);
  if (K <= 64)
    hipLaunchKernelGGL(merge_lists_kernel<1>, grid, dim3(256), 0, stream, in_idx, in_dist, n, L,
                       K_in, K, out_idx, out_dist, dedup);
  else if (K <= 128)
    hipLaunchKernelGGL(merge_lists_kernel<2>, grid, dim3(256), 0, stream, in_idx, in_dist, n, L,
                       K_in, K, out_idx, out_dist, dedup);
  else if (K <= 256)
    hipLaunchKernelGGL(merge_lists_kernel<4>, grid, dim3(256), 0, stream, in_idx, in_dist, n, L,
                       K_in, K, out_idx, out_dist, dedup);
  else if (K <= 512)
    hipLaunchKernelGGL(merge_lists_kernel<8>, grid, dim3(256), 0, stream, in_idx, in_dist, n, L,
                       K_in, K, out_idx, out_dist, dedup);
  else
    hipLaunchKernelGGL(merge_lists_kernel<16>, grid, dim3(256), 0, stream, in_idx, in_dist, n, L,
                       K_in, K, out_idx, out_dist, dedup);
  return hipGetLastError();
}

}  // namespace bdg
