// Admission bounds for the matrix-core tile: an upper bound on the K-th
// neighbour distance of every row, computed before the exhaustive search.
//
// The first reduce searches every record of a partition against all its
// records (Sec. 3.2). Most of the tile's vector work is spent on admissions:
// with a running threshold, a row whose candidates arrive in input order
// admits about K (1 + ln(N / K)) of N candidates, most of them from other
// clusters before its own cluster's members have been seen. The distances to
// any K other rows of the partition bound the final K-th distance from above,
// and a bound close to it removes those early admissions.
//
// Here the K other rows are a row's neighbours in a cheap grouping: pivots
// every `group` rows of the partition (input order, so a strided sample), each
// row joining the group of its nearest pivot (ties to the lower pivot), and
// the bound is the K-th smallest distance to up to `cap` other members of its
// group (the binary k-means of Sec. 3.2 groups similar codes the same way;
// here the grouping only bounds an exact search). Where a group has fewer than
// K other members the row gets no bound (0xFFFF).
//
// Exactness: every candidate of the row's true top K lies at a distance of at
// most the true K-th distance, hence at most the bound, so a tile that admits
// only candidates at most the bound while a list is not full still admits all
// of them; at least K candidates pass that test (the group members that gave
// the bound), so every list fills, after which the usual running threshold
// applies.
//
// Steps (one segment per partition): nearest pivot of every row (one thread
// per row, pivot codes read wave-uniformly when the wave's rows share a
// segment), group sizes by atomics, one work-group's scan to group offsets,
// a scatter of rows and codes into group order, and one wave per row (in
// group order, so the group's codes stay in cache) measuring the group's
// members into a histogram over distances 0..bits in LDS, whose prefix sums
// give the K-th smallest.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.h"

namespace bdg {
namespace {

constexpr uint32_t kNoBound = 0xFFFFu;
constexpr int kBoundWaves = 4;  // rows per work-group of the bound kernel

struct BK {
  const uint64_t* codes;
  uint32_t K, bits, group, cap, nseg, base, total, npiv;
  const uint32_t* seg;   // nullptr: one segment [base, base + total)
  const uint32_t* pseg;  // nullptr: its pivots [0, npiv)
  uint32_t* nearest;  // [total] group of row base + i
  uint32_t* offs;     // [npiv + 1] group sizes, then offsets
  uint32_t* cursor;   // [npiv]
  uint32_t* members;  // [total] rows (relative) in group order
  uint64_t* gcodes;   // [total][W] their codes
  uint16_t* bound;    // [total]
};

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

__device__ __forceinline__ void wave_fence_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The last segment s with seg[s] <= r (seg ascending, seg[0] <= r < seg[nseg]),
// so empty segments are skipped.
__device__ __forceinline__ uint32_t segment_of(const uint32_t* __restrict__ seg, uint32_t nseg,
                                               uint32_t r) {
  uint32_t lo = 0, hi = nseg;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (seg[mid] <= r) lo = mid;
    else hi = mid;
  }
  return lo;
}

__global__ __launch_bounds__(256) void clear_words_kernel(uint32_t* p, uint32_t count) {
  const uint32_t i = blockIdx.x * 256 + threadIdx.x;
  if (i < count) p[i] = 0;
}

template <int W>
__device__ __forceinline__ uint32_t ham_to(const uint64_t (&q)[W], const uint64_t* __restrict__ c) {
  uint32_t d = 0;
#pragma unroll
  for (int w = 0; w < W; ++w) d += (uint32_t)__popcll(q[w] ^ c[w]);
  return d;
}

template <int W>
__global__ __launch_bounds__(256) void nearest_pivot_kernel(BK a) {
  const uint32_t i = blockIdx.x * 256 + threadIdx.x;
  const bool live = i < a.total;
  const uint32_t r = a.base + (live ? i : a.total - 1);
  const uint32_t s = a.seg ? segment_of(a.seg, a.nseg, r) : 0u;
  uint64_t q[W];
#pragma unroll
  for (int w = 0; w < W; ++w) q[w] = a.codes[(size_t)r * W + w];
  uint32_t best = 0xFFFFFFFFu, bj = 0, p0;
  const uint32_t s0 = __builtin_amdgcn_readfirstlane(s);
  if (__ballot(s != s0) == 0) {
    // every lane in one segment: the pivot codes are wave-uniform loads
    const uint32_t lo = __builtin_amdgcn_readfirstlane(a.seg ? a.seg[s0] : a.base);
    p0 = __builtin_amdgcn_readfirstlane(a.pseg ? a.pseg[s0] : 0u);
    const uint32_t np = __builtin_amdgcn_readfirstlane(a.pseg ? a.pseg[s0 + 1] : a.npiv) - p0;
    for (uint32_t j = 0; j < np; ++j) {
      const uint32_t d = ham_to<W>(q, a.codes + (size_t)(lo + j * a.group) * W);
      if (d < best) {
        best = d;
        bj = j;
      }
    }
  } else {
    const uint32_t lo = a.seg ? a.seg[s] : a.base;
    p0 = a.pseg ? a.pseg[s] : 0u;
    const uint32_t np = (a.pseg ? a.pseg[s + 1] : a.npiv) - p0;
    for (uint32_t j = 0; j < np; ++j) {
      const uint32_t d = ham_to<W>(q, a.codes + (size_t)(lo + j * a.group) * W);
      if (d < best) {
        best = d;
        bj = j;
      }
    }
  }
  if (live) {
    const uint32_t g = p0 + bj;
    a.nearest[i] = g;
    atomicAdd(&a.offs[g + 1], 1u);
  }
}

// offs[1..npiv] (group sizes) -> inclusive prefix sums in place (offs[0] = 0),
// so group g is [offs[g], offs[g + 1]); cursor[g] = offs[g]. One work-group.
__global__ __launch_bounds__(1024) void group_scan_kernel(uint32_t* offs, uint32_t* cursor,
                                                          uint32_t npiv) {
  __shared__ uint32_t part[1024];
  const uint32_t t = threadIdx.x;
  const uint32_t per = (npiv + 1023) / 1024;
  const uint64_t b64 = 1 + (uint64_t)t * per;
  const uint32_t b = b64 > npiv + 1 ? npiv + 1 : (uint32_t)b64;
  const uint32_t e = b + per > npiv + 1 ? npiv + 1 : b + per;
  uint32_t sum = 0;
  for (uint32_t x = b; x < e; ++x) sum += offs[x];
  part[t] = sum;
  __syncthreads();
  for (uint32_t off = 1; off < 1024; off <<= 1) {
    const uint32_t v = t >= off ? part[t - off] : 0u;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  uint32_t run = t ? part[t - 1] : 0u;
  for (uint32_t x = b; x < e; ++x) {
    run += offs[x];
    offs[x] = run;
  }
  __syncthreads();
  for (uint32_t g = t; g < npiv; g += 1024) cursor[g] = offs[g];
}

template <int W>
__global__ __launch_bounds__(256) void scatter_group_kernel(BK a) {
  const uint32_t i = blockIdx.x * 256 + threadIdx.x;
  if (i >= a.total) return;
  const uint32_t pos = atomicAdd(&a.cursor[a.nearest[i]], 1u);
  a.members[pos] = i;
#pragma unroll
  for (int w = 0; w < W; ++w) a.gcodes[(size_t)pos * W + w] = a.codes[(size_t)(a.base + i) * W + w];
}

// One wave per position of the group order: the row at that position against
// up to cap + 1 members of its group (itself skipped), distances counted in a
// histogram in LDS; the bound is the smallest distance with at least K members
// at or below it.
template <int W>
__global__ __launch_bounds__(64 * kBoundWaves) void group_bound_kernel(BK a) {
  extern __shared__ uint32_t hist_all[];
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t wave = threadIdx.x >> 6;
  const uint32_t pos = blockIdx.x * kBoundWaves + wave;
  if (pos >= a.total) return;  // whole wave
  const uint32_t nb = a.bits + 1;
  uint32_t* hist = hist_all + wave * nb;
  for (uint32_t x = lane; x < nb; x += 64) hist[x] = 0;
  const uint32_t i = a.members[pos];
  const uint32_t g = a.nearest[i];
  const uint32_t gb = a.offs[g], ge = a.offs[g + 1];
  const uint32_t m = (ge - gb) < a.cap + 1 ? (ge - gb) : a.cap + 1;
  uint64_t q[W];
#pragma unroll
  for (int w = 0; w < W; ++w) q[w] = a.gcodes[(size_t)pos * W + w];
  wave_fence_sync();  // the cleared histogram before any count
  for (uint32_t t = lane; t < m; t += 64) {
    const uint32_t p = gb + t;
    if (p != pos) atomicAdd(&hist[ham_to<W>(q, a.gcodes + (size_t)p * W)], 1u);
  }
  wave_fence_sync();
  const uint32_t others = m - ((pos - gb) < m ? 1u : 0u);
  uint32_t bnd = kNoBound;
  if (others >= a.K) {
    const uint32_t per = (nb + 63) / 64;
    const uint32_t x0 = lane * per;
    uint32_t sum = 0;
    for (uint32_t k = 0; k < per; ++k)
      if (x0 + k < nb) sum += hist[x0 + k];
    uint32_t inc = sum;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const uint32_t v = __shfl_up(inc, off);
      if (lane >= (uint32_t)off) inc += v;
    }
    const uint64_t hit = __ballot(inc >= a.K);  // nonzero: the last lane holds all `others`
    const uint32_t L = (uint32_t)__builtin_ctzll(hit);
    if (lane == L) {
      uint32_t run = inc - sum;
      for (uint32_t k = 0; k < per && x0 + k < nb; ++k) {
        run += hist[x0 + k];
        if (run >= a.K) {
          bnd = x0 + k;
          break;
        }
      }
    }
    bnd = __shfl(bnd, (int)L);
  }
  if (lane == 0) a.bound[i] = (uint16_t)bnd;
}

template <int W>
hipError_t launch_words(const BK& k, hipStream_t stream) {
  const dim3 rows((k.total + 255) / 256);
  hipLaunchKernelGGL(nearest_pivot_kernel<W>, rows, dim3(256), 0, stream, k);
  hipLaunchKernelGGL(group_scan_kernel, dim3(1), dim3(1024), 0, stream, k.offs, k.cursor, k.npiv);
  hipLaunchKernelGGL(scatter_group_kernel<W>, rows, dim3(256), 0, stream, k);
  const size_t lds = (size_t)kBoundWaves * (k.bits + 1) * 4;
  hipLaunchKernelGGL(group_bound_kernel<W>, dim3((k.total + kBoundWaves - 1) / kBoundWaves),
                     dim3(64 * kBoundWaves), lds, stream, k);
  return hipGetLastError();
}

}  // namespace

uint32_t bound_pivots(uint32_t rows, uint32_t group) {
  return (uint32_t)(((uint64_t)rows + group - 1) / group);
}

size_t bound_scratch_bytes(uint32_t total, uint32_t words, uint32_t npiv) {
  return align256((size_t)total * 4) * 2 + align256(((size_t)npiv + 1) * 4) +
         align256((size_t)npiv * 4) + align256((size_t)total * words * 8);
}

hipError_t launch_bounds_pass(const BoundArgs& a, hipStream_t stream) {
  if (a.total == 0) return hipSuccess;
  if (a.words < 1 || a.words > 16 || a.group == 0 || a.npiv == 0 || a.K == 0)
    return hipErrorInvalidValue;
  char* p = static_cast<char*>(a.scratch);
  BK k;
  k.codes = a.codes;
  k.K = a.K;
  k.bits = a.bits;
  k.group = a.group;
  k.cap = a.cap;
  k.nseg = a.nseg;
  k.base = a.base;
  k.total = a.total;
  k.npiv = a.npiv;
  k.seg = a.seg;
  k.pseg = a.pseg;
  k.nearest = reinterpret_cast<uint32_t*>(p);
  p += align256((size_t)a.total * 4);
  k.members = reinterpret_cast<uint32_t*>(p);
  p += align256((size_t)a.total * 4);
  k.offs = reinterpret_cast<uint32_t*>(p);
  p += align256(((size_t)a.npiv + 1) * 4);
  k.cursor = reinterpret_cast<uint32_t*>(p);
  p += align256((size_t)a.npiv * 4);
  k.gcodes = reinterpret_cast<uint64_t*>(p);
  k.bound = a.bound;
  hipLaunchKernelGGL(clear_words_kernel, dim3((a.npiv + 1 + 255) / 256), dim3(256), 0, stream,
                     k.offs, a.npiv + 1);
  switch (a.words) {
    case 1: return launch_words<1>(k, stream);
    case 2: return launch_words<2>(k, stream);
    case 3: return launch_words<3>(k, stream);
    case 4: return launch_words<4>(k, stream);
    case 5: return launch_words<5>(k, stream);
    case 6: return launch_words<6>(k, stream);
    case 7: return launch_words<7>(k, stream);
    case 8: return launch_words<8>(k, stream);
    case 9: return launch_words<9>(k, stream);
    case 10: return launch_words<10>(k, stream);
    case 11: return launch_words<11>(k, stream);
    case 12: return launch_words<12>(k, stream);
    case 13: return launch_words<13>(k, stream);
    case 14: return launch_words<14>(k, stream);
    case 15: return launch_words<15>(k, stream);
    case 16: return launch_words<16>(k, stream);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace bdg
