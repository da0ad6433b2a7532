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
// own group and up to `cap` members of each of the groups of its second- and
// third-nearest pivots (a cluster larger than the group size holds several
// pivots, and three groups cover more of it; the binary k-means of Sec. 3.2
// groups similar codes the same way and also lets a record join more than one
// partition; here the grouping only bounds an exact search). Where the three
// groups have fewer than K other members the row gets no bound (0xFFFF).
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
// a scatter of rows and codes into group order, and 16 lanes per row (in
// group order, so the group's codes stay in cache) measuring the group's
// members into a histogram over distances 0..bits in LDS, whose prefix sums
// give the K-th smallest.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.h"

namespace bdg {
namespace {

constexpr uint32_t kNoBound = 0xFFFFu;
constexpr uint32_t kKeyShift = 21;  // pivot field of a (distance, pivot) key
constexpr uint32_t kKeyPivots = 1u << kKeyShift;
constexpr int kBoundWaves = 4;  // waves per work-group of the bound kernel
constexpr int kBoundSlots = 4;  // rows per wave of the bound kernel

struct BK {
  const uint64_t* codes;
  uint32_t K, bits, group, cap, nseg, base, total, npiv;
  const uint32_t* seg;   // nullptr: one segment [base, base + total)
  const uint32_t* pseg;  // nullptr: its pivots [0, npiv)
  uint32_t* nearest;  // [total] group of row base + i
  uint32_t* second;   // [total] group of its second-nearest pivot (= nearest if none)
  uint32_t* third;    // [total] group of its third-nearest pivot (= nearest if none)
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
  // the three nearest pivots (b1, j1) <= (b2, j2) <= (b3, j3), ties to the
  // lower pivot
  uint32_t b1 = 0xFFFFFFFFu, j1 = 0, b2 = 0xFFFFFFFFu, j2 = 0xFFFFFFFFu, p0;
  uint32_t b3 = 0xFFFFFFFFu, j3 = 0xFFFFFFFFu;
#define BDG_OFFER(dv, jv)                                          \
  do {                                                             \
    const uint32_t d_ = (dv), jj_ = (jv);                          \
    const bool lt1_ = d_ < b1, lt2_ = d_ < b2, lt3_ = d_ < b3;     \
    b3 = lt2_ ? b2 : (lt3_ ? d_ : b3);                             \
    j3 = lt2_ ? j2 : (lt3_ ? jj_ : j3);                            \
    b2 = lt1_ ? b1 : (lt2_ ? d_ : b2);                             \
    j2 = lt1_ ? j1 : (lt2_ ? jj_ : j2);                            \
    b1 = lt1_ ? d_ : b1;                                           \
    j1 = lt1_ ? jj_ : j1;                                          \
  } while (0)
  const uint32_t s0 = __builtin_amdgcn_readfirstlane(s);
  if (__ballot(s != s0) == 0) {
    // every lane in one segment: the pivot codes are wave-uniform loads
    const uint32_t lo = __builtin_amdgcn_readfirstlane(a.seg ? a.seg[s0] : a.base);
    p0 = __builtin_amdgcn_readfirstlane(a.pseg ? a.pseg[s0] : 0u);
    const uint32_t np = __builtin_amdgcn_readfirstlane(a.pseg ? a.pseg[s0 + 1] : a.npiv) - p0;
    const uint64_t* pc = a.codes + (size_t)lo * W;
    const size_t stride = (size_t)a.group * W;
    uint32_t j = 0;
    if (np <= kKeyPivots) {
      // (distance, pivot) as one key, distance << 21 | pivot (distances are at
      // most 1024): the three smallest keys by min / max; four pivots per
      // step, their loads issued together
      uint32_t k1 = 0xFFFFFFFFu, k2 = 0xFFFFFFFFu, k3 = 0xFFFFFFFFu;
#define BDG_PUT(dv, jv)                                   \
  do {                                                    \
    const uint32_t k_ = ((dv) << kKeyShift) | (jv);       \
    const uint32_t t1_ = max(k1, k_);                     \
    k1 = min(k1, k_);                                     \
    const uint32_t t2_ = max(k2, t1_);                    \
    k2 = min(k2, t1_);                                    \
    k3 = min(k3, t2_);                                    \
  } while (0)
      for (; j + 4 <= np; j += 4) {
        const uint64_t* c = pc + (size_t)j * stride;
        const uint32_t d0 = ham_to<W>(q, c), d1 = ham_to<W>(q, c + stride);
        const uint32_t d2 = ham_to<W>(q, c + 2 * stride), d3 = ham_to<W>(q, c + 3 * stride);
        BDG_PUT(d0, j);
        BDG_PUT(d1, j + 1);
        BDG_PUT(d2, j + 2);
        BDG_PUT(d3, j + 3);
      }
      for (; j < np; ++j) BDG_PUT(ham_to<W>(q, pc + (size_t)j * stride), j);
#undef BDG_PUT
      j1 = k1 & (kKeyPivots - 1);
      j2 = k2 == 0xFFFFFFFFu ? 0xFFFFFFFFu : (k2 & (kKeyPivots - 1));
      j3 = k3 == 0xFFFFFFFFu ? 0xFFFFFFFFu : (k3 & (kKeyPivots - 1));
    } else {
      for (; j < np; ++j) BDG_OFFER(ham_to<W>(q, pc + (size_t)j * stride), j);
    }
  } else {
    const uint32_t lo = a.seg ? a.seg[s] : a.base;
    p0 = a.pseg ? a.pseg[s] : 0u;
    const uint32_t np = (a.pseg ? a.pseg[s + 1] : a.npiv) - p0;
    for (uint32_t j = 0; j < np; ++j) BDG_OFFER(ham_to<W>(q, a.codes + (size_t)(lo + j * a.group) * W), j);
  }
#undef BDG_OFFER
  if (live) {
    const uint32_t g = p0 + j1;
    a.nearest[i] = g;
    a.second[i] = j2 == 0xFFFFFFFFu ? g : p0 + j2;
    a.third[i] = j3 == 0xFFFFFFFFu ? g : p0 + j3;
    atomicAdd(&a.offs[g + 1], 1u);
  }
}

// Codes of the pivots of one segment, contiguous (for the matrix-core tile).
__global__ __launch_bounds__(256) void gather_pivots_kernel(const uint64_t* __restrict__ codes,
                                                            uint32_t base, uint32_t group,
                                                            uint32_t npiv, uint32_t words,
                                                            uint64_t* __restrict__ out) {
  const size_t t = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= (size_t)npiv * words) return;
  const size_t j = t / words, w = t - j * words;
  out[t] = codes[((size_t)base + j * group) * words + w];
}

// The three nearest pivots from the tile's three-element lists ((distance,
// pivot) order; missing entries when there are fewer pivots). Every entry
// becomes an index below, so anything outside [0, npiv) is taken as missing
// (a first entry as pivot 0): a bound from any group of other rows is still an
// upper bound on the K-th distance, only a looser one.
__global__ __launch_bounds__(256) void top3_kernel(BK a, const uint32_t* __restrict__ top) {
  const uint32_t i = blockIdx.x * 256 + threadIdx.x;
  if (i >= a.total) return;
  uint32_t g = top[3 * (size_t)i];
  const uint32_t g2 = top[3 * (size_t)i + 1], g3 = top[3 * (size_t)i + 2];
  if (g >= a.npiv) g = 0;
  a.nearest[i] = g;
  a.second[i] = g2 >= a.npiv ? g : g2;
  a.third[i] = g3 >= a.npiv ? g : g3;
  atomicAdd(&a.offs[g + 1], 1u);
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

// Four rows per wave (16 lanes each, kBoundSlots slots), at consecutive
// positions of the group order: the row against up to cap + 1 members of its
// group (itself skipped) and up to cap members of each of its second and third
// groups (each group once), distances
// counted in the slot's histogram in LDS; the bound is the smallest distance
// with at least K members at or below it. Several rows per wave keep several
// chains of dependent loads (position -> row -> groups -> members) in flight.
template <int W>
__global__ __launch_bounds__(64 * kBoundWaves) void group_bound_kernel(BK a) {
  extern __shared__ uint32_t smem[];
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t wave = threadIdx.x >> 6;
  const uint32_t slot = lane >> 4, sub = lane & 15u;
  const uint32_t nb = a.bits + 1;
  uint32_t* hist = smem + (wave * kBoundSlots + slot) * nb;
  const uint32_t pos = (blockIdx.x * kBoundWaves + wave) * kBoundSlots + slot;
  const bool live = pos < a.total;
  for (uint32_t x = sub; x < nb; x += 16) hist[x] = 0;
  uint32_t i = 0, m = 0, m2 = 0, m3 = 0, gb = 0, gb2 = 0, gb3 = 0;
  if (live) {
    i = a.members[pos];
    const uint32_t g = a.nearest[i], g2 = a.second[i], g3 = a.third[i];
    gb = a.offs[g];
    const uint32_t s1 = a.offs[g + 1] - gb;
    m = s1 < a.cap + 1 ? s1 : a.cap + 1;
    if (g2 != g) {
      gb2 = a.offs[g2];
      const uint32_t s2 = a.offs[g2 + 1] - gb2;
      m2 = s2 < a.cap ? s2 : a.cap;
    }
    if (g3 != g && g3 != g2) {
      gb3 = a.offs[g3];
      const uint32_t s3 = a.offs[g3 + 1] - gb3;
      m3 = s3 < a.cap ? s3 : a.cap;
    }
  }
  uint64_t q[W];
#pragma unroll
  for (int w = 0; w < W; ++w) q[w] = live ? a.gcodes[(size_t)pos * W + w] : 0ull;
  wave_fence_sync();  // the cleared histograms before any count
  const uint32_t self = pos - gb;  // the row's place in its group (it is a member)
  for (uint32_t t = sub; t < m + m2 + m3; t += 16) {
    const uint32_t p = t < m ? gb + t : (t < m + m2 ? gb2 + (t - m) : gb3 + (t - m - m2));
    if (t != self) atomicAdd(&hist[ham_to<W>(q, a.gcodes + (size_t)p * W)], 1u);
  }
  wave_fence_sync();
  // the row is a member of its own group only
  const uint32_t others = m + m2 + m3 - (self < m ? 1u : 0u);
  const bool want = live && others >= a.K;
  // prefix sums over the slot's 16 lanes of their bins' counts
  const uint32_t per = (nb + 15) / 16;
  const uint32_t x0 = sub * per;
  uint32_t sum = 0;
  for (uint32_t k = 0; k < per; ++k)
    if (x0 + k < nb) sum += hist[x0 + k];
  uint32_t inc = sum;
#pragma unroll
  for (int off = 1; off < 16; off <<= 1) {
    const uint32_t v = __shfl_up(inc, off, 16);
    if (sub >= (uint32_t)off) inc += v;
  }
  // the slot's first lane whose prefix reaches K (the last lane holds all `others`)
  const uint64_t hit = __ballot(want && inc >= a.K);
  const uint32_t mine = (uint32_t)(hit >> (16 * slot)) & 0xFFFFu;
  if (want && mine && sub == (uint32_t)__builtin_ctz(mine)) {
    uint32_t run = inc - sum, bnd = kNoBound;
    for (uint32_t k = 0; k < per && x0 + k < nb; ++k) {
      run += hist[x0 + k];
      if (run >= a.K) {
        bnd = x0 + k;
        break;
      }
    }
    a.bound[i] = (uint16_t)bnd;
  } else if (live && !want && sub == 0) {
    a.bound[i] = (uint16_t)kNoBound;
  }
}

template <int W>
hipError_t launch_words(const BK& k, const BoundArgs& a, hipStream_t stream) {
  const dim3 rows((k.total + 255) / 256);
  if (a.rect_scratch && !a.seg) {
    // every row against every pivot on the matrix cores: a rectangular tile
    // with three-element lists (rows = the codes, columns = the pivots)
    char* p = static_cast<char*>(a.rect_scratch);
    uint64_t* pcodes = reinterpret_cast<uint64_t*>(p);
    p += align256((size_t)k.npiv * W * 8);
    void* pfrags = p;
    p += align256(prep_bytes(k.npiv, W));
    uint32_t* top = reinterpret_cast<uint32_t*>(p);
    p += align256((size_t)k.total * 12);
    uint16_t* tdist = reinterpret_cast<uint16_t*>(p);
    hipLaunchKernelGGL(gather_pivots_kernel, dim3((unsigned)(((size_t)k.npiv * W + 255) / 256)),
                       dim3(256), 0, stream, k.codes, k.base, k.group, k.npiv, (uint32_t)W, pcodes);
    hipError_t e = launch_prep(pcodes, k.npiv, W, pfrags, stream);
    if (e != hipSuccess) return e;
    RunArgs r;
    r.codes = k.codes;
    r.frags = pfrags;
    r.words = W;
    r.bits = k.bits;
    r.K = 3;
    r.idx_bits = run_idx_bits(k.bits);
    r.row0 = k.base;
    r.nrows = k.total;
    r.cb = 0;
    r.ce = k.npiv;
    r.fresh = 1;
    r.out_idx = top;
    r.out_dist = tdist;
    r.rect = 1;
    e = launch_mfma_run(r, stream);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(top3_kernel, rows, dim3(256), 0, stream, k, top);
  } else {
    hipLaunchKernelGGL(nearest_pivot_kernel<W>, rows, dim3(256), 0, stream, k);
  }
  hipLaunchKernelGGL(group_scan_kernel, dim3(1), dim3(1024), 0, stream, k.offs, k.cursor, k.npiv);
  hipLaunchKernelGGL(scatter_group_kernel<W>, rows, dim3(256), 0, stream, k);
  const size_t lds = (size_t)kBoundWaves * kBoundSlots * (k.bits + 1) * 4;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(group_bound_kernel<W>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  const uint32_t per_wg = kBoundWaves * kBoundSlots;
  hipLaunchKernelGGL(group_bound_kernel<W>, dim3((k.total + per_wg - 1) / per_wg),
                     dim3(64 * kBoundWaves), lds, stream, k);
  return hipGetLastError();
}

}  // namespace

size_t bound_rect_bytes(uint32_t total, uint32_t words, uint32_t npiv) {
  if (!run_supported(npiv, words, 3)) return 0;
  return align256((size_t)npiv * words * 8) + align256(prep_bytes(npiv, words)) +
         align256((size_t)total * 12) + align256((size_t)total * 6);
}

uint32_t bound_pivots(uint32_t rows, uint32_t group) {
  return (uint32_t)(((uint64_t)rows + group - 1) / group);
}

size_t bound_scratch_bytes(uint32_t total, uint32_t words, uint32_t npiv) {
  return align256((size_t)total * 4) * 4 + align256(((size_t)npiv + 1) * 4) +
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
  k.second = reinterpret_cast<uint32_t*>(p);
  p += align256((size_t)a.total * 4);
  k.third = reinterpret_cast<uint32_t*>(p);
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
    case 1: return launch_words<1>(k, a, stream);
    case 2: return launch_words<2>(k, a, stream);
    case 3: return launch_words<3>(k, a, stream);
    case 4: return launch_words<4>(k, a, stream);
    case 5: return launch_words<5>(k, a, stream);
    case 6: return launch_words<6>(k, a, stream);
    case 7: return launch_words<7>(k, a, stream);
    case 8: return launch_words<8>(k, a, stream);
    case 9: return launch_words<9>(k, a, stream);
    case 10: return launch_words<10>(k, a, stream);
    case 11: return launch_words<11>(k, a, stream);
    case 12: return launch_words<12>(k, a, stream);
    case 13: return launch_words<13>(k, a, stream);
    case 14: return launch_words<14>(k, a, stream);
    case 15: return launch_words<15>(k, a, stream);
    case 16: return launch_words<16>(k, a, stream);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace bdg
