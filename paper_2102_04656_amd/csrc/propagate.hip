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
// only). Neighbours of neighbours repeat a lot (points of one cluster sit in
// each other's lists), so before a candidate's code is gathered its index is
// entered in a per-wave hash set in LDS (linear probing, compare-and-swap):
// only the first occurrence of an index is measured. The running result R
// (64 NR keys dist << 32 | idx, ascending, as in the list merge) starts with
// the row's own list; each 64-entry chunk of a neighbour's list becomes up
// to 64 new candidates, and only a chunk in which some candidate passes the
// filter is merged in. While every index of the row has been recorded in the
// set, new candidates are distinct from each other and from R; once an
// insertion gives up (the probe limit), the row falls back to dropping
// entries already in R (binary search of R in LDS) and repeats inside a
// chunk before the bitonic merge. The filter is the propagation filter of Sec. 3.6 (3) applied
// continuously: a candidate farther than the current K-th distance of R
// cannot enter (ties are kept, since a smaller index may still displace the
// K-th key), and R's K-th distance only decreases, so the result is the
// exact top-K of the union of both floors.
//
// Bound: random gathers of list rows and of the codes of distinct
// candidates (8 bytes per word, a cache line per code); memory latency is
// hidden by many resident waves (few registers, 8 KB + 512 NR bytes of LDS
// per wave).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.h"
#include "wave_topk64.h"

namespace bdg {

namespace {

constexpr int kPW = 64;
constexpr uint32_t kMaxWords = 16;
constexpr uint32_t kAbsent = 0xFFFFFFFFu;
constexpr uint32_t kSetBits = 11;  // hash set of 2048 indices per wave
constexpr uint32_t kSetSize = 1u << kSetBits;
constexpr int kProbes = 8;

// Insert z into the set: 1 = new, 0 = already there, 2 = not recorded (every
// probed slot held another index).
__device__ __forceinline__ uint32_t set_insert(uint32_t* set, uint32_t z) {
  uint32_t slot = (z * 0x9E3779B1u) >> (32 - kSetBits);
  for (int i = 0; i < kProbes; ++i) {
    uint32_t expect = kAbsent;
    if (__hip_atomic_compare_exchange_strong(&set[slot], &expect, z, __ATOMIC_RELAXED,
                                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP))
      return 1u;
    if (expect == z) return 0u;
    slot = (slot + 1) & (kSetSize - 1);
  }
  return 2u;
}

template <int NR>
__global__ __launch_bounds__(256) void propagate_kernel(const uint64_t* __restrict__ codes,
                                                        uint32_t n, uint32_t words, uint32_t K,
                                                        const uint32_t* __restrict__ in_idx,
                                                        uint32_t* __restrict__ out_idx,
                                                        uint16_t* __restrict__ out_dist) {
  __shared__ uint64_t lds[4][kPW * NR];
  __shared__ uint32_t sets[4][kSetSize];
  const uint32_t wave = threadIdx.x >> 6;
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t row = blockIdx.x * 4 + wave;
  if (row >= n) return;  // wave-uniform
  uint64_t* Rl = lds[wave];
  uint32_t* set = sets[wave];
  constexpr uint32_t N = kPW * NR;
#pragma unroll
  for (uint32_t i = 0; i < kSetSize / kPW; ++i) set[i * kPW + lane] = kAbsent;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  bool exact_set = true;  // wave-uniform: every index so far is in the set

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
  // Merge up to 64 candidate keys (one per lane, kNone64 for none) into R;
  // with dedup, keys already in R and repeats among them are dropped first.
  auto absorb = [&](uint64_t x, bool dedup) {
    if (!dedup) {
      merge64_into<NR>(R, x, lane);
      return;
    }
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
    const bool valid = y != kAbsent && y < n && y != row;
    const uint32_t ins = valid ? set_insert(set, y) : 0u;
    if (__any(ins == 2u)) exact_set = false;
    const bool ok = ins != 0u;  // first occurrence (or not recorded)
    yv[r] = ok ? y : kAbsent;
    const uint64_t key = ok ? (((uint64_t)ham_to(y) << 32) | y) : kNone64;
    if (__any(ok)) absorb(key, !exact_set);
  }
  uint32_t maxd = kth_dist();

  // Second floor: the lists of the first-floor neighbours, kNb neighbours at
  // a time (all their list chunks, then all the chunks' codes, are gathered
  // before any is filtered, so each group costs one round of dependent
  // loads). A later chunk is filtered again after the earlier ones' merges; a
  // filter with an older, larger K-th distance only admits more, so it stays
  // exact.
  constexpr int kNb = 4;
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    for (uint32_t tt = 0; tt < (uint32_t)kPW; tt += kNb) {
      const uint32_t t = r * kPW + tt;
      if (t >= K) break;
      uint32_t yn[kNb];
      bool some = false;
#pragma unroll
      for (int i = 0; i < kNb; ++i) {
        yn[i] = t + i < K ? __builtin_amdgcn_readlane(yv[r], tt + i) : kAbsent;
        some |= yn[i] != kAbsent;
      }
      if (!some) continue;  // wave-uniform
      for (uint32_t c0 = 0; c0 < K; c0 += kPW) {
        const uint32_t p = c0 + lane;
        uint32_t z[kNb], ins[kNb], h[kNb];
#pragma unroll
        for (int i = 0; i < kNb; ++i)
          z[i] = (yn[i] != kAbsent && p < K) ? in_idx[(size_t)yn[i] * K + p] : kAbsent;
        bool lost = false;
#pragma unroll
        for (int i = 0; i < kNb; ++i) {
          const bool v = z[i] != kAbsent && z[i] < n && z[i] != row;
          ins[i] = v ? set_insert(set, z[i]) : 0u;
          lost |= ins[i] == 2u;
        }
        if (__any(lost)) exact_set = false;
#pragma unroll
        for (int i = 0; i < kNb; ++i) h[i] = ins[i] != 0u ? ham_to(z[i]) : 0xFFFFFFFFu;
#pragma unroll
        for (int i = 0; i < kNb; ++i) {
          const bool pass = ins[i] != 0u && h[i] <= maxd;
          if (__any(pass)) {
            absorb(pass ? (((uint64_t)h[i] << 32) | z[i]) : kNone64, !exact_set);
            maxd = kth_dist();
          }
        }
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
