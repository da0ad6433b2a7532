// Online search on the graph (Sec. 3.5): sampled "long-link" entry points,
// hill-climbing on the kNN graph ("short-link") with a candidate pool, and a
// re-rank of the whole pool by the real-valued features.
//
// One wave per query. Entry: the nearest of the S sampled rows (Hamming;
// ties to the smaller index). The pool holds the P smallest (distance,
// index) seen, as sorted 64-bit keys dist << 33 | idx << 1 | expanded: the
// expanded flag sits below the index, so it never changes the order, and an
// empty slot (all ones) reads as expanded. Each step expands the smallest
// pool member not yet expanded: every neighbour in its graph row that has
// not been visited is marked visited (a per-query bitmap over all rows,
// set with atomic OR: exactly one lane wins a row listed twice), measured,
// and offered to the pool (a chunk is merged only if some key beats the
// P-th). The search stops when every pool member is expanded. Re-rank:
// squared L2 in float32 with each operation rounded (no fused
// multiply-add), accumulated over the dimensions in order, ties to the
// smaller index; the N best are the answer.
//
// Bound: latency of dependent gathers (graph rows, codes, bitmap words) per
// expansion; many resident waves (queries) hide it.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "kernels.h"
#include "wave_topk64.h"

namespace bdg {

namespace {

constexpr int kSW = 64;
constexpr uint32_t kSMaxWords = 16;
constexpr uint32_t kNoRow = 0xFFFFFFFFu;
constexpr uint32_t kMaxExpand = 1u << 20;

// Wait until every vector-memory operation of the wave has completed (gfx9
// encoding: vmcnt 0, lgkmcnt and expcnt left alone): the single-lane visits
// below return nothing the wave waits on, and later atomics on the same
// bitmap words must see them.
__device__ __forceinline__ void wait_vm() {
  __builtin_amdgcn_s_waitcnt((7 << 4) | (15 << 8));
}

__device__ __forceinline__ uint64_t wave_min64(uint64_t x, uint32_t lane) {
  x = umin64(x, xshfl64<32>(x, lane));
  x = umin64(x, xshfl64<16>(x, lane));
  x = umin64(x, xshfl64<8>(x, lane));
  x = umin64(x, xshfl64<4>(x, lane));
  x = umin64(x, xshfl64<2>(x, lane));
  x = umin64(x, xshfl64<1>(x, lane));
  return x;
}

template <int NR>
__global__ __launch_bounds__(256) void search_kernel(
    const uint64_t* __restrict__ codes, uint32_t n, uint32_t words,
    const uint32_t* __restrict__ graph, uint32_t K, const float* __restrict__ feats, uint32_t d,
    const uint64_t* __restrict__ qcodes, const float* __restrict__ qfeats,
    const uint32_t* __restrict__ qexcl, uint32_t q0, uint32_t nq,
    const uint32_t* __restrict__ entries, uint32_t S, uint32_t P, uint32_t N,
    uint32_t* __restrict__ maps, uint32_t mapw, uint32_t* __restrict__ out_idx,
    float* __restrict__ out_dist, uint32_t* __restrict__ out_vis) {
  const uint32_t wave = threadIdx.x >> 6, lane = threadIdx.x & 63u;
  const uint32_t qb = blockIdx.x * 4 + wave;  // query within the batch
  if (qb >= nq) return;                       // wave-uniform
  const uint32_t q = q0 + qb;
  uint32_t* vis = maps + (size_t)qb * mapw;
  uint64_t x[kSMaxWords];
#pragma unroll
  for (uint32_t w = 0; w < kSMaxWords; ++w) x[w] = w < words ? qcodes[(size_t)q * words + w] : 0;
  auto ham_to = [&](uint32_t v) {
    uint32_t h = 0;
#pragma unroll
    for (uint32_t w = 0; w < kSMaxWords; ++w)
      if (w < words) h += __popcll(x[w] ^ codes[(size_t)v * words + w]);
    return h;
  };
  // true iff this call marked row v visited first
  auto visit = [&](uint32_t v) {
    const uint32_t bit = 1u << (v & 31u);
    return (atomicOr(&vis[v >> 5], bit) & bit) == 0u;
  };
  const uint32_t excl = qexcl ? qexcl[q] : kNoRow;
  if (lane == 0 && excl < n) visit(excl);
  wait_vm();
  uint32_t nvis = 0;

  // Entry point.
  uint64_t best = kNone64;
  for (uint32_t e0 = 0; e0 < S; e0 += kSW) {
    const uint32_t e = e0 + lane < S ? entries[e0 + lane] : kNoRow;
    const bool ok = e < n && e != excl;
    best = umin64(best, ok ? (((uint64_t)ham_to(e) << 32) | e) : kNone64);
  }
  best = wave_min64(best, lane);

  uint64_t R[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) R[r] = kNone64;
  if (best != kNone64) {
    const uint32_t e = (uint32_t)best;
    if (lane == 0) visit(e);
    wait_vm();
    nvis = 1;
    if (lane == 0) R[0] = ((best >> 32) << 33) | ((uint64_t)e << 1);
  }
  auto pth_key = [&]() {
    const uint32_t last = P - 1;
    uint64_t k = kNone64;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      if ((last >> 6) == (uint32_t)r) {
        const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)R[r], last & 63);
        const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(R[r] >> 32), last & 63);
        k = ((uint64_t)hi << 32) | lo;
      }
    }
    return k;
  };

  for (uint32_t step = 0; step < kMaxExpand; ++step) {
    // the smallest pool member not yet expanded
    uint32_t u = kNoRow;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      if (u != kNoRow) continue;
      const uint64_t m = __ballot(R[r] != kNone64 && (R[r] & 1ull) == 0);
      if (m) {
        const uint32_t sel = (uint32_t)__builtin_ctzll(m);
        const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)R[r], sel);
        const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(R[r] >> 32), sel);
        u = (uint32_t)((((uint64_t)hi << 32) | lo) >> 1);
        if (lane == sel) R[r] |= 1ull;
      }
    }
    if (u == kNoRow) break;
    const size_t ub = (size_t)u * K;
    for (uint32_t c0 = 0; c0 < K; c0 += kSW) {
      const uint32_t p = c0 + lane;
      const uint32_t v = p < K ? graph[ub + p] : kNoRow;
      const bool fresh = v < n && visit(v);
      nvis += (uint32_t)__builtin_popcountll(__ballot(fresh));
      const uint64_t key = fresh ? (((uint64_t)ham_to(v) << 33) | ((uint64_t)v << 1)) : kNone64;
      const uint64_t pth = pth_key();
      const bool pass = fresh && key < pth;
      if (!__any(pass)) continue;
      merge64_into<NR>(R, pass ? key : kNone64, lane);
#pragma unroll
      for (int r = 0; r < NR; ++r)
        if (r * kSW + lane >= P) R[r] = kNone64;
    }
  }

  // Re-rank the pool by float32 squared L2.
  uint64_t F[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) F[r] = kNone64;
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const uint32_t v = R[r] == kNone64 ? kNoRow : (uint32_t)(R[r] >> 1);
    uint64_t key = kNone64;
    if (v != kNoRow) {
      const float* a = feats + (size_t)v * d;
      const float* b = qfeats + (size_t)q * d;
      float acc = 0.0f;
      for (uint32_t i = 0; i < d; ++i) {
#pragma clang fp contract(off)
        const float t = a[i] - b[i];
        const float t2 = t * t;
        acc = acc + t2;
      }
      key = ((uint64_t)__float_as_uint(acc) << 32) | v;
    }
    if (__any(key != kNone64)) merge64_into<NR>(F, key, lane);
  }
  const size_t o = (size_t)q * N;
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const uint32_t p = r * kSW + lane;
    if (p < N) {
      out_idx[o + p] = F[r] == kNone64 ? kNoRow : (uint32_t)F[r];
      out_dist[o + p] = F[r] == kNone64 ? INFINITY : __uint_as_float((uint32_t)(F[r] >> 32));
    }
  }
  if (out_vis && lane == 0) out_vis[q] = nvis;
}

}  // namespace

size_t search_map_words(uint32_t n) { return ((size_t)n + 31) / 32; }

hipError_t launch_search(const uint64_t* codes, uint32_t n, uint32_t words, const uint32_t* graph,
                         uint32_t K, const float* feats, uint32_t d, const uint64_t* qcodes,
                         const float* qfeats, const uint32_t* qexcl, uint32_t q0, uint32_t nq,
                         const uint32_t* entries, uint32_t S, uint32_t P, uint32_t N,
                         uint32_t* maps, uint32_t* out_idx, float* out_dist, uint32_t* out_vis,
                         hipStream_t stream) {
  if (nq == 0) return hipSuccess;
  if (words == 0 || words > kSMaxWords || P == 0 || P > 1024 || N == 0 || N > P || K == 0)
    return hipErrorInvalidValue;
  const uint32_t mapw = (uint32_t)search_map_words(n);
  hipError_t e = hipMemsetAsync(maps, 0, (size_t)nq * mapw * sizeof(uint32_t), stream);
  if (e != hipSuccess) return e;
  const dim3 grid((nq + 3) / 4);
  if (P <= 64)
    hipLaunchKernelGGL(search_kernel<1>, grid, dim3(256), 0, stream, codes, n, words, graph, K, feats,
                       d, qcodes, qfeats, qexcl, q0, nq, entries, S, P, N, maps, mapw, out_idx,
                       out_dist, out_vis);
  else if (P <= 128)
    hipLaunchKernelGGL(search_kernel<2>, grid, dim3(256), 0, stream, codes, n, words, graph, K, feats,
                       d, qcodes, qfeats, qexcl, q0, nq, entries, S, P, N, maps, mapw, out_idx,
                       out_dist, out_vis);
  else if (P <= 256)
    hipLaunchKernelGGL(search_kernel<4>, grid, dim3(256), 0, stream, codes, n, words, graph, K, feats,
                       d, qcodes, qfeats, qexcl, q0, nq, entries, S, P, N, maps, mapw, out_idx,
                       out_dist, out_vis);
  else if (P <= 512)
    hipLaunchKernelGGL(search_kernel<8>, grid, dim3(256), 0, stream, codes, n, words, graph, K, feats,
                       d, qcodes, qfeats, qexcl, q0, nq, entries, S, P, N, maps, mapw, out_idx,
                       out_dist, out_vis);
  else
    hipLaunchKernelGGL(search_kernel<16>, grid, dim3(256), 0, stream, codes, n, words, graph, K,
                       feats, d, qcodes, qfeats, qexcl, q0, nq, entries, S, P, N, maps, mapw,
                       out_idx, out_dist, out_vis);
  return hipGetLastError();
}

}  // namespace bdg
