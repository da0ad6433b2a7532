// Hamming distance tiles with fused exact top-K (gfx950 / CDNA4).
//
// The first reduce of the single-pass divide-and-conquer (Sec. 3.2) searches
// every record of a partition against the partition exhaustively; the paper
// moved this "large numbers of distance calculations" loop to native code
// (Sec. 3.6 (2)). Here one wave owns a group of query rows and streams a
// column block past them, keeping the per-row top-K in LDS (wave_topk.h).
// Distances never reach HBM: only the K-lists of each (row, column block) do.
//
// This file holds the vector-ALU path: lane = column; a few queries per wave
// are wave-uniform (scalar registers); distance = sum over 32-bit words of
// popcount(q ^ c). The matrix-core path is in tile_mfma.hip; both give
// identical graphs.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.h"
#include "wave_topk.h"

namespace bdg {

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

// ---------------------------------------------------------------- launch --

constexpr int kPrefetchPopc = 4;

static uint32_t popc_queries_rt(uint32_t words) {
  uint32_t q = 32 / words;
  return q > 16 ? 16 : (q < 1 ? 1 : q);
}

static size_t lds_bytes(uint32_t words, uint32_t K) {
  return (size_t)popc_queries_rt(words) * (K + kWave) * 4;
}

static constexpr size_t kLdsMax = 160 * 1024;

bool tile_supported(int path, uint32_t words, uint32_t K) {
  if (words < 1 || words > 16 || K < 1 || K > 1024) return false;
  if (path != kPathPopc) return false;
  return lds_bytes(words, K) <= kLdsMax;
}

uint32_t tile_rows(int path, uint32_t words) {
  (void)path;
  return popc_queries_rt(words);
}

template <int W, int NR>
static hipError_t launch_w(int path, const TileArgs& a, hipStream_t stream) {
  if (path != kPathPopc) return hipErrorInvalidValue;
  const size_t lds = lds_bytes(W, a.K);
  const uint32_t rows = tile_rows(path, W);
  const uint32_t nblk = (a.col1 - a.col0 + a.col_block - 1) / a.col_block;
  dim3 grid((a.nrows + rows - 1) / rows, nblk);
  auto kern = knn_popc_kernel<W, NR, popc_queries<W>(), kPrefetchPopc>;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, grid, dim3(kWave), lds, stream, a.codes, a.K, a.row0, a.nrows, a.col0,
                     a.col1, a.col_block, a.out_idx, a.out_dist);
  return hipGetLastError();
}

template <int W>
static hipError_t launch_nr(int path, const TileArgs& a, hipStream_t stream) {
  if (a.K <= 64) return launch_w<W, 1>(path, a, stream);
  if (a.K <= 128) return launch_w<W, 2>(path, a, stream);
  if (a.K <= 256) return launch_w<W, 4>(path, a, stream);
  if (a.K <= 512) return launch_w<W, 8>(path, a, stream);
  return launch_w<W, 16>(path, a, stream);
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
