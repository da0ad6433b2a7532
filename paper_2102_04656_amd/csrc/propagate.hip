// Neighbourhood propagation on the graph: one more floor of neighbours
// (Sec. 3.3). The flat, depth-one breadth-first step compares every row x
// with all neighbours of its first-floor neighbours and keeps the K nearest
// of its own list and that second floor. The paper moves (reverse neighbour,
// base neighbour) pairs through two shuffles; on one GPU the row gathers its
// second floor directly: the neighbours y of x are the rows whose lists hold
// x's second floor, so row x reads the lists of its K neighbours and the
// codes of their entries.
//
// One wave per row; the row's code stays in registers. Every distance is
// recomputed from the codes (the input lists are read for their indices
// only). The running result R (64 NR keys dist << 32 | idx, ascending, as in
// the list merge) starts with the row's own list; each 64-entry chunk of a
// neighbour's list becomes 64 candidates, and only a chunk in which some
// candidate passes the filter is merged in: drop entries already in R
// (binary search of R in LDS) and repeats inside the chunk, then the bitonic
// merge. The filter is the propagation filter of Sec. 3.6 (3) applied
// continuously: a candidate farther than the current K-th distance of R
// cannot enter (ties are kept, since a smaller index may still displace the
// K-th key), and R's K-th distance only decreases, so the result is the
// exact top-K of the union of both floors.
//
// Bound: random gathers of codes (8 bytes per word per candidate, K^2
// candidates per row) and of list rows; memory latency is hidden by many
// resident waves (few registers, 512 NR bytes of LDS per wave).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.h"
#include "wave_topk64.h"

namespace bdg {

namespace {

constexpr int kPW = 64;
constexpr uint32_t kMaxWords = 16;
constexpr uint32_t kAbsent = 0xFFFFFFFFu;

template <int NR>
__global__ __launch_bounds__(256) void propagate_kernel(const uint64_t* __restrict__ codes,
                                                        uint32_t n, uint32_t words, uint32_t K,
                                                        const uint32_t* __restrict__ in_idx,
                                                        uint32_t* __restrict__ out_idx,
                                                        uint16_t* __restrict__ out_dist) {
  __shared__ uint64_t lds[4][kPW * NR];
  const uint32_t wave = threadIdx.x >> 6;
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t row = blockIdx.x * 4 + wave;
  if (row >= n) return;  // wave-uniform
  uint64_t* Rl = lds[wave];
  constexpr uint32_t N = kPW * NR;

  uint64_t xw[kMaxWords];
#pragma unroll
  for (uint32_t w = 0; w < kMaxWords; ++w) xw[w] = w < words ? codes[(size_t)row * words + w] : 0;
  auto ham_to = [&](uint32_t z) {
    uint32_t h = 0;
#pragma unroll
    for (uint32_t w = 0; w < kMaxWords; ++w)
      if (w < words) h += __popcll(xw[w] ^ codes[(size_t)z * words + w]);
    return h;
  };

  uint64_t R[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) R[r] = kNone64;
  // Merge up to 64 candidate keys (one per lane, kNone64 for none) into R.
  auto absorb = [&](uint64_t x) {
    x = wave_sort64_u64(x, lane);
#pragma unroll
    for (int r = 0; r < NR; ++r) Rl[r * kPW + lane] = R[r];
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    bool drop = false;
    if (x != kNone64) {
      uint32_t lo = 0, hi = N;  // lower bound of x in R
      while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (Rl[mid] < x) lo = mid + 1; else hi = mid;
      }
      drop = lo < N && Rl[lo] == x;
    }
    const int src = lane == 0 ? 0 : (int)lane - 1;
    const uint64_t prev = ((uint64_t)(uint32_t)__shfl((int)(uint32_t)(x >> 32), src, kPW) << 32) |
                          (uint32_t)__shfl((int)(uint32_t)x, src, kPW);
    if (lane > 0 && prev == x) drop = true;
    if (drop) x = kNone64;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    merge64_into<NR>(R, x, lane);
  };
  // distance of R's K-th key; 0xFFFF (every candidate passes) while R has
  // fewer than K keys
  auto kth_dist = [&]() {
    const uint32_t last = K - 1;
    uint64_t kth = kNone64;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      if ((last >> 6) == (uint32_t)r) {
        const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)R[r], last & 63);
        const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(R[r] >> 32), last & 63);
        kth = ((uint64_t)hi << 32) | lo;
      }
    }
    return kth == kNone64 ? 0xFFFFu : (uint32_t)(kth >> 32);
  };

  // First floor: the row's own list.
  const size_t base = (size_t)row * K;
  uint32_t yv[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const uint32_t p = r * kPW + lane;
    const uint32_t y = p < K ? in_idx[base + p] : kAbsent;
    const bool ok = y != kAbsent && y < n && y != row;
    yv[r] = ok ? y : kAbsent;
    const uint64_t key = ok ? (((uint64_t)ham_to(y) << 32) | y) : kNone64;
    if (__any(ok)) absorb(key);
  }
  uint32_t maxd = kth_dist();

  // Second floor: the lists of the first-floor neighbours.
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    for (uint32_t tt = 0; tt < (uint32_t)kPW; ++tt) {
      const uint32_t t = r * kPW + tt;
      if (t >= K) break;
      const uint32_t y = __builtin_amdgcn_readlane(yv[r], tt);
      if (y == kAbsent) continue;  // wave-uniform
      const size_t ybase = (size_t)y * K;
      for (uint32_t c0 = 0; c0 < K; c0 += kPW) {
        const uint32_t p = c0 + lane;
        const uint32_t z = p < K ? in_idx[ybase + p] : kAbsent;
        const bool ok = z != kAbsent && z < n && z != row;
        const uint32_t h = ok ? ham_to(z) : 0xFFFFFFFFu;
        const bool pass = ok && h <= maxd;
        if (!__any(pass)) continue;
        absorb(pass ? (((uint64_t)h << 32) | z) : kNone64);
        maxd = kth_dist();
      }
    }
  }

#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const uint32_t p = r * kPW + lane;
    if (p < K) {
      const uint64_t key = R[r];
      out_idx[base + p] = key == kNone64 ? kAbsent : (uint32_t)key;
      out_dist[base + p] = key == kNone64 ? (uint16_t)0xFFFFu : (uint16_t)(key >> 32);
    }
  }
}

}  // namespace

hipError_t launch_propagate(const uint64_t* codes, uint32_t n, uint32_t words, uint32_t K,
                            const uint32_t* in_idx, uint32_t* out_idx, uint16_t* out_dist,
                            hipStream_t stream) {
  if (n == 0) return hipSuccess;
  if (words == 0 || words > kMaxWords || K == 0 || K > 4 * kPW) return hipErrorInvalidValue;
  const dim3 grid((n + 3) / 4);
  if (K <= 64)
    hipLaunchKernelGGL(propagate_kernel<1>, grid, dim3(256), 0, stream, codes, n, words, K, in_idx,
                       out_idx, out_dist);
  else if (K <= 128)
    hipLaunchKernelGGL(propagate_kernel<2>, grid, dim3(256), 0, stream, codes, n, words, K, in_idx,
                       out_idx, out_dist);
  else
    hipLaunchKernelGGL(propagate_kernel<4>, grid, dim3(256), 0, stream, codes, n, words, K, in_idx,
                       out_idx, out_dist);
  return hipGetLastError();
}

}  // namespace bdg
