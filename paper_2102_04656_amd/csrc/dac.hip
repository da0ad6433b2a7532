// Single-pass divide-and-conquer (Sec. 3.2) on one GPU.
//
// Binary k-means on a sample (Eq. 1-2): each sample point joins its nearest
// centre (ties to the smaller centre), then every centre bit becomes the
// majority bit of its points (a tie gives 0; a centre without points keeps
// its bits). Then every point finds its T nearest centres; its home is the
// nearest, D_j = the points whose home is j (disjoint). Point q selects its
// nearest centres in order until the summed |D_j| reaches coarse_num (the
// crossing centre included, at most T), and its row is the K nearest of the
// home members of the selected centres, q excluded. The paper moves records
// by centre through a shuffle and searches each partition on its own
// (Reduce1), then merges a point's lists (Reduce2); on one GPU the members
// are laid out by home centre once (counting sort, codes gathered into that
// order) and each point streams the contiguous members of its selected
// centres, so the partitions' lists never need a merge: the sets are
// disjoint and one running top-K per point receives them all.
//
// Kernels: sample assignment on the matrix cores (rectangular tile, K = 1),
// or with the centres staged in LDS (one thread per point); bit counts with atomics and the majority update; the T nearest
// centres per point on the matrix cores (the running-list tile of
// tile_mfma.hip in its rectangular mode: rows = the codes, columns = the
// centres), or one wave per point on the vector ALUs where the tile does not
// take the shape; sizes, offsets and the scatter into home order; the search
// (one wave per point, coalesced member codes, a filter against the running
// K-th distance before each merge).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.h"
#include "wave_topk64.h"

namespace bdg {

namespace {

constexpr int kDW = 64;
constexpr uint32_t kDMaxWords = 16;
constexpr uint32_t kStageU64 = 4096;  // centre words staged in LDS per pass (32 KB)

// home[i] = nearest centre of code rows[i] (ties to the smaller index).
__global__ __launch_bounds__(256) void bk_assign_kernel(const uint64_t* __restrict__ codes,
                                                        uint32_t words,
                                                        const uint32_t* __restrict__ rows,
                                                        uint32_t nrows,
                                                        const uint64_t* __restrict__ centres,
                                                        uint32_t m, uint32_t* __restrict__ home) {
  __shared__ uint64_t cs[kStageU64];
  const uint32_t i = blockIdx.x * 256 + threadIdx.x;
  uint64_t x[kDMaxWords];
  const uint32_t r = i < nrows ? rows[i] : 0u;
#pragma unroll
  for (uint32_t w = 0; w < kDMaxWords; ++w) x[w] = (i < nrows && w < words) ? codes[(size_t)r * words + w] : 0;
  uint32_t best = 0, bd = 0xFFFFFFFFu;
  const uint32_t per = kStageU64 / words;  // centres per pass
  for (uint32_t j0 = 0; j0 < m; j0 += per) {
    const uint32_t cnt = (m - j0) < per ? (m - j0) : per;
    __syncthreads();
    for (uint32_t t = threadIdx.x; t < cnt * words; t += 256) cs[t] = centres[(size_t)j0 * words + t];
    __syncthreads();
    for (uint32_t j = 0; j < cnt; ++j) {
      uint32_t d = 0;
#pragma unroll
      for (uint32_t w = 0; w < kDMaxWords; ++w)
        if (w < words) d += __popcll(x[w] ^ cs[j * words + w]);
      if (d < bd) {
        bd = d;
        best = j0 + j;
      }
    }
  }
  if (i < nrows) home[i] = best;
}

// cnt[j][bit] += bits of the sample rows in centre j; size[j] += 1.
__global__ __launch_bounds__(256) void bk_count_kernel(const uint64_t* __restrict__ codes,
                                                       uint32_t words,
                                                       const uint32_t* __restrict__ rows,
                                                       uint32_t nrows,
                                                       const uint32_t* __restrict__ home,
                                                       uint32_t* __restrict__ cnt,
                                                       uint32_t* __restrict__ size) {
  const uint32_t t = blockIdx.x * 256 + threadIdx.x;
  const uint32_t i = t / words, w = t - i * words;
  if (i >= nrows) return;
  const uint32_t j = home[i];
  uint64_t v = codes[(size_t)rows[i] * words + w];
  uint32_t* c = cnt + ((size_t)j * words + w) * 64;
  while (v) {
    const uint32_t b = (uint32_t)__builtin_ctzll(v);
    v &= v - 1;
    atomicAdd(&c[b], 1u);
  }
  if (w == 0) atomicAdd(&size[j], 1u);
}

// Centre word (j, w) from the counts: bit b = 1 iff 2 cnt > size.
__global__ __launch_bounds__(256) void bk_update_kernel(uint32_t m, uint32_t words,
                                                        const uint32_t* __restrict__ cnt,
                                                        const uint32_t* __restrict__ size,
                                                        uint64_t* __restrict__ centres) {
  const uint32_t t = blockIdx.x * 256 + threadIdx.x;
  if (t >= m * words) return;
  const uint32_t j = t / words;
  const uint32_t s = size[j];
  if (s == 0) return;
  const uint32_t* c = cnt + (size_t)t * 64;
  uint64_t v = 0;
  for (uint32_t b = 0; b < 64; ++b)
    if (2u * c[b] > s) v |= 1ull << b;
  centres[t] = v;
}

__global__ void bk_init_kernel(const uint64_t* __restrict__ codes, uint32_t words,
                               const uint32_t* __restrict__ init, uint32_t m,
                               uint64_t* __restrict__ centres) {
  const uint32_t t = blockIdx.x * 256 + threadIdx.x;
  if (t >= m * words) return;
  const uint32_t j = t / words, w = t - j * words;
  centres[t] = codes[(size_t)init[j] * words + w];
}

// top[i][0..T) = the T nearest centres of point i, ascending (distance,
// centre); one wave per point.
__global__ __launch_bounds__(256) void top_centres_kernel(const uint64_t* __restrict__ codes,
                                                          uint32_t n, uint32_t words,
                                                          const uint64_t* __restrict__ centres,
                                                          uint32_t m, uint32_t T,
                                                          uint32_t* __restrict__ top) {
  const uint32_t wave = threadIdx.x >> 6, lane = threadIdx.x & 63u;
  const uint32_t i = blockIdx.x * 4 + wave;
  if (i >= n) return;  // wave-uniform
  uint64_t x[kDMaxWords];
#pragma unroll
  for (uint32_t w = 0; w < kDMaxWords; ++w) x[w] = w < words ? codes[(size_t)i * words + w] : 0;
  uint64_t R[1] = {kNone64};
  uint64_t kth = kNone64;
  for (uint32_t j0 = 0; j0 < m; j0 += kDW) {
    const uint32_t j = j0 + lane;
    uint64_t key = kNone64;
    if (j < m) {
      uint32_t d = 0;
#pragma unroll
      for (uint32_t w = 0; w < kDMaxWords; ++w)
        if (w < words) d += __popcll(x[w] ^ centres[(size_t)j * words + w]);
      key = ((uint64_t)d << 32) | j;
    }
    if (!__any(key < kth)) continue;
    merge64_into<1>(R, key, lane);
    const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)R[0], T - 1);
    const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(R[0] >> 32), T - 1);
    kth = ((uint64_t)hi << 32) | lo;
  }
  if (lane < T) top[(size_t)i * T + lane] = R[0] == kNone64 ? 0xFFFFFFFFu : (uint32_t)R[0];
}

__global__ __launch_bounds__(256) void home_size_kernel(const uint32_t* __restrict__ top,
                                                        uint32_t n, uint32_t T,
                                                        uint32_t* __restrict__ size) {
  const uint32_t i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) atomicAdd(&size[top[(size_t)i * T]], 1u);
}

// off[j] = sum of size[0..j), off[m] = n; cursor[j] = 0 (one thread: m is small).
__global__ void offsets_kernel(const uint32_t* __restrict__ size, uint32_t m,
                               uint32_t* __restrict__ off, uint32_t* __restrict__ cursor) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  uint32_t acc = 0;
  for (uint32_t j = 0; j < m; ++j) {
    off[j] = acc;
    cursor[j] = 0;
    acc += size[j];
  }
  off[m] = acc;
}

// Members in home order: member[p] = point index, hcodes[p] = its code.
__global__ __launch_bounds__(256) void scatter_home_kernel(const uint64_t* __restrict__ codes,
                                                           uint32_t n, uint32_t words,
                                                           const uint32_t* __restrict__ top,
                                                           uint32_t T,
                                                           const uint32_t* __restrict__ off,
                                                           uint32_t* __restrict__ cursor,
                                                           uint32_t* __restrict__ member,
                                                           uint64_t* __restrict__ hcodes) {
  const uint32_t i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const uint32_t j = top[(size_t)i * T];
  const uint32_t p = off[j] + atomicAdd(&cursor[j], 1u);
  member[p] = i;
  for (uint32_t w = 0; w < words; ++w) hcodes[(size_t)p * words + w] = codes[(size_t)i * words + w];
}

// Row q = the K nearest home members of q's selected centres (q excluded).
template <int NR>
__global__ __launch_bounds__(256) void dac_search_kernel(
    const uint64_t* __restrict__ codes, uint32_t n, uint32_t words, const uint32_t* __restrict__ top,
    uint32_t T, const uint32_t* __restrict__ size, const uint32_t* __restrict__ off,
    const uint32_t* __restrict__ member, const uint64_t* __restrict__ hcodes, uint32_t coarse_num,
    uint32_t K, uint32_t* __restrict__ out_idx, uint16_t* __restrict__ out_dist) {
  const uint32_t wave = threadIdx.x >> 6, lane = threadIdx.x & 63u;
  const uint32_t q = blockIdx.x * 4 + wave;
  if (q >= n) return;  // wave-uniform
  uint64_t x[kDMaxWords];
#pragma unroll
  for (uint32_t w = 0; w < kDMaxWords; ++w) x[w] = w < words ? codes[(size_t)q * words + w] : 0;
  uint64_t R[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) R[r] = kNone64;
  uint32_t maxd = 0xFFFFu;  // running K-th distance (none while R holds fewer than K)
  const uint32_t tl = lane < T ? top[(size_t)q * T + lane] : 0xFFFFFFFFu;
  uint32_t total = 0;
  for (uint32_t t = 0; t < T; ++t) {
    const uint32_t j = __builtin_amdgcn_readlane(tl, t);
    if (j == 0xFFFFFFFFu) break;
    const uint32_t b0 = off[j], b1 = off[j + 1];
    for (uint32_t p0 = b0; p0 < b1; p0 += kDW) {
      const uint32_t p = p0 + lane;
      uint64_t key = kNone64;
      bool pass = false;
      if (p < b1) {
        const uint32_t b = member[p];
        uint32_t d = 0;
#pragma unroll
        for (uint32_t w = 0; w < kDMaxWords; ++w)
          if (w < words) d += __popcll(x[w] ^ hcodes[(size_t)p * words + w]);
        pass = b != q && d <= maxd;
        key = ((uint64_t)d << 32) | b;
      }
      if (!__any(pass)) continue;
      merge64_into<NR>(R, pass ? key : kNone64, lane);
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
      maxd = kth == kNone64 ? 0xFFFFu : (uint32_t)(kth >> 32);
    }
    total += size[j];
    if (total >= coarse_num) break;
  }
  const size_t o = (size_t)q * K;
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const uint32_t p = r * kDW + lane;
    if (p < K) {
      out_idx[o + p] = R[r] == kNone64 ? 0xFFFFFFFFu : (uint32_t)R[r];
      out_dist[o + p] = R[r] == kNone64 ? (uint16_t)0xFFFFu : (uint16_t)(R[r] >> 32);
    }
  }
}

inline dim3 grid_of(size_t threads) { return dim3((unsigned)((threads + 255) / 256)); }

}  // namespace

size_t bkmeans_tile_scratch_bytes(uint32_t ns, uint32_t m, uint32_t words) {
  if (ns == 0 || !run_supported(m, words, 1)) return 0;
  return (((size_t)ns * words * 8 + 255) & ~size_t(255)) +
         ((prep_bytes(m, words) + 255) & ~size_t(255)) + (size_t)ns * sizeof(uint16_t);
}

hipError_t launch_bkmeans(const uint64_t* codes, uint32_t words, const uint32_t* sample,
                          uint32_t ns, const uint32_t* init, uint32_t m, uint32_t iters,
                          uint64_t* centres, uint32_t* home, uint32_t* cnt, uint32_t* size,
                          void* tile_scratch, hipStream_t stream) {
  if (words == 0 || words > kDMaxWords || m == 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(bk_init_kernel, grid_of((size_t)m * words), dim3(256), 0, stream, codes,
                     words, init, m, centres);
  // With scratch, the assignment runs on the matrix cores: the sample's codes
  // are gathered once into rows, and each round the centres become the
  // columns of a rectangular tile with K = 1 ((distance, centre) order: ties
  // to the smaller centre).
  const bool tile = tile_scratch != nullptr && ns > 0 && run_supported(m, words, 1);
  uint64_t* scode = static_cast<uint64_t*>(tile_scratch);
  char* frags = tile ? static_cast<char*>(tile_scratch) + (((size_t)ns * words * 8 + 255) & ~size_t(255))
                     : nullptr;
  uint16_t* tdist = tile ? reinterpret_cast<uint16_t*>(frags + ((prep_bytes(m, words) + 255) & ~size_t(255)))
                         : nullptr;
  if (tile)
    hipLaunchKernelGGL(bk_init_kernel, grid_of((size_t)ns * words), dim3(256), 0, stream, codes,
                       words, sample, ns, scode);
  for (uint32_t it = 0; it < iters && ns > 0; ++it) {
    if (tile) {
      hipError_t e = launch_prep(centres, m, words, frags, stream);
      if (e != hipSuccess) return e;
      RunArgs a;
      a.codes = scode;
      a.frags = frags;
      a.words = words;
      a.bits = words * 64;
      a.K = 1;
      a.idx_bits = run_idx_bits(words * 64);
      a.row0 = 0;
      a.nrows = ns;
      a.cb = 0;
      a.ce = m;
      a.fresh = 1;
      a.out_idx = home;
      a.out_dist = tdist;
      a.rect = 1;
      e = launch_mfma_run(a, stream);
      if (e != hipSuccess) return e;
    } else {
      hipLaunchKernelGGL(bk_assign_kernel, grid_of(ns), dim3(256), 0, stream, codes, words, sample,
                         ns, centres, m, home);
    }
    hipError_t e = hipMemsetAsync(cnt, 0, (size_t)m * words * 64 * sizeof(uint32_t), stream);
    if (e != hipSuccess) return e;
    e = hipMemsetAsync(size, 0, (size_t)m * sizeof(uint32_t), stream);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(bk_count_kernel, grid_of((size_t)ns * words), dim3(256), 0, stream, codes,
                       words, sample, ns, home, cnt, size);
    hipLaunchKernelGGL(bk_update_kernel, grid_of((size_t)m * words), dim3(256), 0, stream, m,
                       words, cnt, size, centres);
  }
  return hipGetLastError();
}

size_t dac_top_scratch_bytes(uint32_t n, uint32_t m, uint32_t words, uint32_t T) {
  if (!run_supported(m, words, T)) return 0;
  return ((prep_bytes(m, words) + 255) & ~size_t(255)) + (size_t)n * T * sizeof(uint16_t);
}

hipError_t launch_dac(const uint64_t* codes, uint32_t n, uint32_t words, const uint64_t* centres,
                      uint32_t m, uint32_t T, uint32_t coarse_num, uint32_t K, uint32_t* top,
                      uint32_t* size, uint32_t* off, uint32_t* cursor, uint32_t* member,
                      uint64_t* hcodes, uint32_t* out_idx, uint16_t* out_dist, void* top_scratch,
                      hipStream_t stream) {
  if (words == 0 || words > kDMaxWords || m == 0 || T == 0 || T > 64 || K == 0 || K > 256)
    return hipErrorInvalidValue;
  hipError_t e = hipSuccess;
  if (top_scratch != nullptr && run_supported(m, words, T)) {
    // The exhaustive comparison of every row with the centres is a rectangular
    // tile on the matrix cores: rows = the codes, columns = the centres, K = T,
    // (distance, centre) order, no own-row exclusion.
    char* frags = static_cast<char*>(top_scratch);
    uint16_t* tdist =
        reinterpret_cast<uint16_t*>(frags + ((prep_bytes(m, words) + 255) & ~size_t(255)));
    e = launch_prep(centres, m, words, frags, stream);
    if (e != hipSuccess) return e;
    RunArgs a;
    a.codes = codes;
    a.frags = frags;
    a.words = words;
    a.bits = words * 64;
    a.K = T;
    a.idx_bits = run_idx_bits(words * 64);
    a.row0 = 0;
    a.nrows = n;
    a.cb = 0;
    a.ce = m;
    a.fresh = 1;
    a.out_idx = top;
    a.out_dist = tdist;
    a.rect = 1;
    e = launch_mfma_run(a, stream);
  } else {
    hipLaunchKernelGGL(top_centres_kernel, dim3((n + 3) / 4), dim3(256), 0, stream, codes, n,
                       words, centres, m, T, top);
  }
  if (e != hipSuccess) return e;
  e = hipMemsetAsync(size, 0, (size_t)m * sizeof(uint32_t), stream);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(home_size_kernel, grid_of(n), dim3(256), 0, stream, top, n, T, size);
  hipLaunchKernelGGL(offsets_kernel, dim3(1), dim3(1), 0, stream, size, m, off, cursor);
  hipLaunchKernelGGL(scatter_home_kernel, grid_of(n), dim3(256), 0, stream, codes, n, words, top,
                     T, off, cursor, member, hcodes);
  const dim3 g((n + 3) / 4);
  if (K <= 64)
    hipLaunchKernelGGL(dac_search_kernel<1>, g, dim3(256), 0, stream, codes, n, words, top, T, size,
                       off, member, hcodes, coarse_num, K, out_idx, out_dist);
  else if (K <= 128)
    hipLaunchKernelGGL(dac_search_kernel<2>, g, dim3(256), 0, stream, codes, n, words, top, T, size,
                       off, member, hcodes, coarse_num, K, out_idx, out_dist);
  else
    hipLaunchKernelGGL(dac_search_kernel<4>, g, dim3(256), 0, stream, codes, n, words, top, T, size,
                       off, member, hcodes, coarse_num, K, out_idx, out_dist);
  return hipGetLastError();
}

}  // namespace bdg
