// Hamming distance tiles with fused exact top-K (gfx950 / CDNA4).
//
// The first reduce of the single-pass divide-and-conquer (Sec. 3.2) searches
// every record of a partition against the partition exhaustively; the paper
// moved this "large numbers of distance calculations" loop to native code
// (Sec. 3.6 (2)). Here one wave owns a group of query rows and streams a
// column block past them, keeping the per-row top-K in LDS (wave_topk.h).
// Distances never reach HBM: only the K-lists of each (row, column block) do.
//
// Two ways to compute the distances, giving identical graphs:
//   * popc: lane = column; a few queries per wave are wave-uniform (scalar
//           registers); distance = sum over 32-bit words of popcount(q ^ c).
//   * mfma: 16 candidates x 16*QG queries per step on the int8 matrix cores.
//           Candidate bits are expanded to 0/1 bytes, query bits to +-1 bytes;
//           dot = <a, 2q - 1> = 2 popc(a & q) - popc(a), hence
//           ham(a, q) = popc(q) - dot, exact in int32.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.h"
#include "wave_topk.h"

namespace bdg {

typedef int v4i __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------------ popc --

// Queries per wave of the popcount tile: their words are wave-uniform and live
// in scalar registers (about 64 of them), so QS * W is held near 32 words.
template <int W>
constexpr int popc_queries() {
  return (32 / W) > 16 ? 16 : ((32 / W) < 1 ? 1 : 32 / W);
}

// Lane = column: every step the wave takes 64 consecutive columns (one per
// lane, coalesced loads, a D-deep prefetch ring) and scores them against its
// QS queries. A passing lane appends its key at cnt + (passing lanes below
// it); a buffer that would overflow is merged into the list first and the
// step's candidates are re-tested against the new threshold.
template <int W, int NR, int QS, int D>
__global__ __launch_bounds__(64) void knn_popc_kernel(const uint64_t* __restrict__ codes,
                                                      uint32_t K, uint32_t row0, uint32_t nrows,
                                                      uint32_t col0, uint32_t col1,
                                                      uint32_t col_block,
                                                      uint32_t* __restrict__ out_idx,
                                                      uint16_t* __restrict__ out_dist) {
  constexpr int B = kWave;
  extern __shared__ uint32_t smem[];
  uint32_t* list = smem;         // [QS][K]
  uint32_t* buf = list + QS * K; // [QS][B]
  const uint32_t lane = threadIdx.x;
  const uint32_t tile0 = blockIdx.x * QS;
  const uint32_t cb = col0 + blockIdx.y * col_block;
  const uint32_t ce = min(cb + col_block, col1);

  for (uint32_t p = lane; p < QS * K; p += kWave) list[p] = kKeyNone;

  uint64_t q[QS][W];
  uint32_t thr[QS], cnt[QS], qrow[QS];
#pragma unroll
  for (int s = 0; s < QS; ++s) {
    const uint32_t ql = tile0 + s;
    const bool valid = ql < nrows;
    const uint64_t* qp = codes + (size_t)(row0 + (valid ? ql : 0u)) * W;
#pragma unroll
    for (int w = 0; w < W; ++w) q[s][w] = qp[w];
    thr[s] = valid ? kDistNone : 0u;  // an absent query never passes
    cnt[s] = 0;
    qrow[s] = row0 + ql;
  }
  __syncthreads();

  const uint32_t ngroups = (ce - cb + kWave - 1) / kWave;
  uint64_t colw[D][W];
#pragma unroll
  for (int d = 0; d < D; ++d) {
    const uint64_t* cp = codes + (size_t)min(cb + kWave * d + lane, ce - 1) * W;
#pragma unroll
    for (int w = 0; w < W; ++w) colw[d][w] = cp[w];
  }

  for (uint32_t t0 = 0; t0 < ngroups; t0 += D) {
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const uint32_t t = t0 + d;
      if (t >= ngroups) break;
      uint32_t dd[QS];
      bool pass = false;
#pragma unroll
      for (int s = 0; s < QS; ++s) {
        uint32_t acc = 0;
#pragma unroll
        for (int w = 0; w < W; ++w) acc += (uint32_t)__popcll(q[s][w] ^ colw[d][w]);
        dd[s] = acc;
        pass |= acc < thr[s];
      }
      {
        const uint64_t* cp = codes + (size_t)min(cb + kWave * (t + D) + lane, ce - 1) * W;
#pragma unroll
        for (int w = 0; w < W; ++w) colw[d][w] = cp[w];
      }
      if (__any(pass)) {
        const uint32_t col = cb + kWave * t + lane;
#pragma unroll
        for (int s = 0; s < QS; ++s) {
          bool p = dd[s] < thr[s] && col < ce && col != qrow[s];
          uint64_t m = __ballot(p);
          if (m) {
            uint32_t c = (uint32_t)__popcll(m);
            if (cnt[s] + c > (uint32_t)B) {
              __syncthreads();
              const uint32_t kth = flush_query<NR, B>(list + s * K, buf + s * B, cnt[s], K, lane);
              cnt[s] = 0;
              thr[s] = key_dist(kth);
              __syncthreads();
              p = dd[s] < thr[s] && col < ce && col != qrow[s];
              m = __ballot(p);
              c = (uint32_t)__popcll(m);
            }
            if (p) {
              const uint32_t below = __builtin_amdgcn_mbcnt_hi(
                  (uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
              buf[s * B + cnt[s] + below] = (dd[s] << kIdxBits) | (col - cb);
            }
            cnt[s] += c;
          }
        }
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int s = 0; s < QS; ++s) {
    if (cnt[s]) {
      flush_query<NR, B>(list + s * K, buf + s * B, cnt[s], K, lane);
      __syncthreads();
    }
  }
  if (tile0 < nrows)
    write_lists(list, QS, nrows - tile0, K, cb, out_idx, out_dist,
                (size_t)blockIdx.y * nrows + tile0, lane);
}

// ------------------------------------------------------------------ mfma --

// 4 bits -> 4 bytes in {0, 1}: byte t = bit t. The multiplier places copies
// of the nibble at bit offsets 0, 7, 14, 21 (no two terms overlap), so bit t
// of the nibble lands at bit 8t.
__device__ __forceinline__ int spread_nibble(uint32_t nib) {
  return (int)((nib * 0x00204081u) & 0x01010101u);
}

// 16 code bits -> the 16 int8 operand values of one lane, 0/1.
__device__ __forceinline__ v4i expand01(uint32_t h) {
  v4i r;
  r[0] = spread_nibble(h & 15u);
  r[1] = spread_nibble((h >> 4) & 15u);
  r[2] = spread_nibble((h >> 8) & 15u);
  r[3] = spread_nibble((h >> 12) & 15u);
  return r;
}

// 16 code bits -> +-1 bytes (0x01 for a set bit, 0xFF for a clear one).
__device__ __forceinline__ v4i expand_pm1(uint32_t h) {
  v4i r = expand01(h);
#pragma unroll
  for (int t = 0; t < 4; ++t) r[t] = (int)(((uint32_t)r[t] * 0xFEu) ^ 0xFFFFFFFFu);
  return r;
}

// Raw words one lane loads per code: quarter g of the code, 2W bytes at byte
// offset 2W g, as W/2 dwords (W even) or W 16-bit halves (W odd).
template <int W>
constexpr int raw_words() {
  return (W % 2 == 0) ? W / 2 : W;
}

template <int W>
__device__ __forceinline__ void load_raw(const uint64_t* code, uint32_t g,
                                         uint32_t (&r)[raw_words<W>()]) {
  if constexpr (W % 4 == 0) {
    const uint64_t* p = code + g * (W / 4);
#pragma unroll
    for (int t = 0; t < W / 4; ++t) {
      const uint64_t v = p[t];
      r[2 * t] = (uint32_t)v;
      r[2 * t + 1] = (uint32_t)(v >> 32);
    }
  } else if constexpr (W % 2 == 0) {
    const uint32_t* p = reinterpret_cast<const uint32_t*>(code) + g * (W / 2);
#pragma unroll
    for (int t = 0; t < W / 2; ++t) r[t] = p[t];
  } else {
    const uint16_t* p = reinterpret_cast<const uint16_t*>(code) + g * W;
#pragma unroll
    for (int t = 0; t < W; ++t) r[t] = p[t];
  }
}

// Chunk s (16 bits) of the lane's quarter: code bits [16 (W g + s), +16).
// Candidates and queries use the same mapping, so every int8 product pairs
// the same code bit of both operands.
template <int W>
__device__ __forceinline__ uint32_t raw_chunk(const uint32_t (&r)[raw_words<W>()], int s) {
  if constexpr (W % 2 == 0)
    return (r[s >> 1] >> ((s & 1) * 16)) & 0xFFFFu;
  else
    return r[s];
}

// Output layout of v_mfma_i32_16x16x64_i8 with A = 16 candidates (rows) and
// B = 16 queries (columns): lane l holds D[4 (l / 16) + r][l % 16] in
// element r, so a lane sees one query (l % 16) and four candidates.
//
// The accumulator input of the first k-step is -thr_dot (per query), so the
// result is dot - thr_dot and a candidate passes iff it is > 0; the test of
// a whole step is one max-reduction and one compare.
template <int W, int NR, int QG, int D>
__global__ __launch_bounds__(64) void knn_mfma_kernel(const uint64_t* __restrict__ codes,
                                                      uint32_t K, uint32_t row0, uint32_t nrows,
                                                      uint32_t col0, uint32_t col1,
                                                      uint32_t col_block,
                                                      uint32_t* __restrict__ out_idx,
                                                      uint16_t* __restrict__ out_dist) {
  constexpr int B = kWave;
  constexpr int Q = 16 * QG;
  constexpr int RW = raw_words<W>();
  constexpr int kStepKeys = 16;      // keys one query can gain per 16-candidate step
  constexpr int kNoQuery = 1 << 20;  // thr_dot of an absent query: never passes
  extern __shared__ uint32_t smem[];
  uint32_t* list = smem;         // [Q][K]
  uint32_t* buf = list + Q * K;  // [Q][B]
  uint32_t* cnt = buf + Q * B;   // [Q]
  const uint32_t lane = threadIdx.x;
  const uint32_t g = lane >> 4;
  const uint32_t i16 = lane & 15u;
  const uint32_t tile0 = blockIdx.x * Q;
  const uint32_t cb = col0 + blockIdx.y * col_block;
  const uint32_t ce = min(cb + col_block, col1);

  for (uint32_t p = lane; p < Q * K; p += kWave) list[p] = kKeyNone;
  if (lane < Q) cnt[lane] = 0;

  v4i bq[QG][W];
  v4i thrC[QG];
  int pq[QG], thr_dot[QG];
  uint32_t qrow[QG];
#pragma unroll
  for (int gq = 0; gq < QG; ++gq) {
    const uint32_t ql = tile0 + 16 * gq + i16;
    const bool valid = ql < nrows;
    uint32_t r[RW];
    load_raw<W>(codes + (size_t)(row0 + (valid ? ql : 0u)) * W, g, r);
    int pc = 0;
#pragma unroll
    for (int s = 0; s < W; ++s) {
      const uint32_t h = raw_chunk<W>(r, s);
      pc += __popc(h);
      bq[gq][s] = expand_pm1(h);
    }
    pc += __shfl_xor(pc, 16, kWave);
    pc += __shfl_xor(pc, 32, kWave);
    pq[gq] = pc;
    thr_dot[gq] = valid ? pc - (int)kDistNone : kNoQuery;
    thrC[gq] = v4i{-thr_dot[gq], -thr_dot[gq], -thr_dot[gq], -thr_dot[gq]};
    qrow[gq] = row0 + ql;
  }
  __syncthreads();

  const uint32_t ngroups = (ce - cb + 15) / 16;
  uint32_t raw[D][RW];
#pragma unroll
  for (int d = 0; d < D; ++d)
    load_raw<W>(codes + (size_t)min(cb + 16 * d + i16, ce - 1) * W, g, raw[d]);

  for (uint32_t t0 = 0; t0 < ngroups; t0 += D) {
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const uint32_t t = t0 + d;
      if (t >= ngroups) break;
      v4i a[W];
#pragma unroll
      for (int s = 0; s < W; ++s) a[s] = expand01(raw_chunk<W>(raw[d], s));
      load_raw<W>(codes + (size_t)min(cb + 16 * (t + D) + i16, ce - 1) * W, g, raw[d]);
      v4i acc[QG];
#pragma unroll
      for (int gq = 0; gq < QG; ++gq)
        acc[gq] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[0], bq[gq][0], thrC[gq], 0, 0, 0);
#pragma unroll
      for (int s = 1; s < W; ++s)
#pragma unroll
        for (int gq = 0; gq < QG; ++gq)
          acc[gq] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[s], bq[gq][s], acc[gq], 0, 0, 0);
      int mx = acc[0][0];
#pragma unroll
      for (int gq = 0; gq < QG; ++gq)
#pragma unroll
        for (int r = 0; r < 4; ++r) mx = max(mx, acc[gq][r]);
      if (__any(mx > 0)) {
        const uint32_t c0 = cb + 16 * t;
#pragma unroll
        for (int gq = 0; gq < QG; ++gq) {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const uint32_t col = c0 + 4 * g + r;
            if (acc[gq][r] > 0 && col < ce && col != qrow[gq]) {
              const uint32_t dist = (uint32_t)(pq[gq] - (acc[gq][r] + thr_dot[gq]));
              const uint32_t qi = 16 * gq + i16;
              const uint32_t slot = atomicAdd(&cnt[qi], 1u);
              buf[qi * B + slot] = (dist << kIdxBits) | (col - cb);
            }
          }
        }
        __syncthreads();
        const uint32_t myc = lane < (uint32_t)Q ? cnt[lane] : 0u;
        uint64_t m = __ballot(myc > (uint32_t)(B - kStepKeys));
        while (m) {
          const uint32_t qi = __builtin_ctzll(m);
          m &= m - 1;
          const uint32_t cq = __builtin_amdgcn_readlane(myc, qi);
          const uint32_t kth = flush_query<NR, B>(list + qi * K, buf + qi * B, cq, K, lane);
          const int kd = (int)key_dist(kth);
#pragma unroll
          for (int gq = 0; gq < QG; ++gq) {
            if ((qi >> 4) == (uint32_t)gq && (qi & 15u) == i16) {
              thr_dot[gq] = pq[gq] - kd;
              thrC[gq] = v4i{-thr_dot[gq], -thr_dot[gq], -thr_dot[gq], -thr_dot[gq]};
            }
          }
          if (lane == qi) cnt[qi] = 0;
          __syncthreads();
        }
      }
    }
  }
  __syncthreads();
  {
    const uint32_t myc = lane < (uint32_t)Q ? cnt[lane] : 0u;
    uint64_t m = __ballot(myc > 0);
    while (m) {
      const uint32_t qi = __builtin_ctzll(m);
      m &= m - 1;
      const uint32_t cq = __builtin_amdgcn_readlane(myc, qi);
      flush_query<NR, B>(list + qi * K, buf + qi * B, cq, K, lane);
      __syncthreads();
    }
  }
  if (tile0 < nrows)
    write_lists(list, Q, nrows - tile0, K, cb, out_idx, out_dist,
                (size_t)blockIdx.y * nrows + tile0, lane);
}

// ---------------------------------------------------------------- launch --

template <int W>
constexpr int mfma_qgroups() {
  return W <= 8 ? 4 : 2;
}

constexpr int kPrefetchPopc = 4;
constexpr int kPrefetchMfma = 8;

static uint32_t popc_queries_rt(uint32_t words) {
  uint32_t q = 32 / words;
  return q > 16 ? 16 : (q < 1 ? 1 : q);
}

static size_t lds_bytes(int path, uint32_t words, uint32_t K) {
  if (path == kPathPopc) return (size_t)popc_queries_rt(words) * (K + kWave) * 4;
  const uint32_t Q = 16u * (words <= 8 ? 4u : 2u);
  return (size_t)Q * (K + kWave + 1) * 4;
}

static constexpr size_t kLdsMax = 160 * 1024;

bool tile_supported(int path, uint32_t words, uint32_t K) {
  if (words < 1 || words > 16 || K < 1 || K > 256) return false;
  if (path != kPathPopc && path != kPathMfma) return false;
  return lds_bytes(path, words, K) <= kLdsMax;
}

uint32_t tile_rows(int path, uint32_t words) {
  return path == kPathPopc ? popc_queries_rt(words) : 16u * (words <= 8 ? 4u : 2u);
}

template <int W, int NR>
static hipError_t launch_w(int path, const TileArgs& a, hipStream_t stream) {
  const size_t lds = lds_bytes(path, W, a.K);
  const uint32_t rows = tile_rows(path, W);
  const uint32_t nblk = (a.col1 - a.col0 + a.col_block - 1) / a.col_block;
  dim3 grid((a.nrows + rows - 1) / rows, nblk);
  if (path == kPathPopc) {
    auto kern = knn_popc_kernel<W, NR, popc_queries<W>(), kPrefetchPopc>;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, grid, dim3(kWave), lds, stream, a.codes, a.K, a.row0, a.nrows,
                       a.col0, a.col1, a.col_block, a.out_idx, a.out_dist);
  } else {
    auto kern = knn_mfma_kernel<W, NR, mfma_qgroups<W>(), kPrefetchMfma>;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, grid, dim3(kWave), lds, stream, a.codes, a.K, a.row0, a.nrows,
                       a.col0, a.col1, a.col_block, a.out_idx, a.out_dist);
  }
  return hipGetLastError();
}

template <int W>
static hipError_t launch_nr(int path, const TileArgs& a, hipStream_t stream) {
  if (a.K <= 64) return launch_w<W, 1>(path, a, stream);
  if (a.K <= 128) return launch_w<W, 2>(path, a, stream);
  return launch_w<W, 4>(path, a, stream);
}

hipError_t launch_tile(int path, const TileArgs& a, hipStream_t stream) {
  switch (a.words) {
    case 1: return launch_nr<1>(path, a, stream);
    case 2: return launch_nr<2>(path, a, stream);
    case 3: return launch_nr<3>(path, a, stream);
    case 4: return launch_nr<4>(path, a, stream);
    case 5: return launch_nr<5>(path, a, stream);
    case 6: return launch_nr<6>(path, a, stream);
    case 7: return launch_nr<7>(path, a, stream);
    case 8: return launch_nr<8>(path, a, stream);
    case 9: return launch_nr<9>(path, a, stream);
    case 10: return launch_nr<10>(path, a, stream);
    case 11: return launch_nr<11>(path, a, stream);
    case 12: return launch_nr<12>(path, a, stream);
    case 13: return launch_nr<13>(path, a, stream);
    case 14: return launch_nr<14>(path, a, stream);
    case 15: return launch_nr<15>(path, a, stream);
    case 16: return launch_nr<16>(path, a, stream);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace bdg
