// Exact squared-L2 kNN in FP32 with the top-K fused (gfx950): the
// real-valued ground truth of recall (Sec. 4.2, Eq. 3) and the source of the
// learned binariser's training pairs.
//
// Distances are assembled as |q|^2 + |y|^2 - 2 <q, y>, the inner products on
// the FP32 matrix cores (v_mfma_f32_16x16x4_f32) and never written to HBM:
// each wave holds 16 queries as B operands in registers for the whole launch,
// the work-group's 4 waves share a stream of 16-row base groups staged in LDS
// (double-buffered, one barrier per group), and every 16 x 16 tile of
// distances goes straight to the per-query top-K.
//
// k order. In k-step (t, s) of a group, lane l (row l % 16, quarter q = l / 16)
// feeds dimension 16 t + 4 q + s, for both operands; over s = 0..3 and the four
// quarters every dimension of the 16-wide chunk t is covered once. A lane's four
// values of chunk t are then one contiguous 16-byte load, for the query (held
// in registers) and the base row (staged in LDS).
//
// Top-K. Keys are (float bits of the distance) << 32 | base index: distances
// are >= 0, so unsigned key order is the (distance, index) order. Each query
// keeps its K smallest keys sorted in LDS and a threshold (the K-th distance)
// in a register; base rows arrive in increasing index, so a candidate enters
// only at a distance strictly below the threshold. Passing candidates go to a
// pending buffer owned by the lane that computed them (4 sub-buffers of 8 per
// query); a buffer that would overflow is merged into the list by the whole
// wave (64-bit bitonic sort and merge). Queries with their own row in the base
// leave it out through `exclude`.
//
// Wide bases are split over work-groups (so a few thousand queries still fill
// the chip); each split writes its exact top-K of its rows, and a merge kernel
// takes the top-K of the union (the splits are disjoint). d must be a multiple
// of 4 and at most 512 for the matrix-core kernel; other shapes take a plain
// vector-ALU kernel (one wave per query, direct sums).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "bdg.h"
#include "kernels.h"
#include "wave_topk64.h"

namespace bdg {
int api_error(int status, const char* fmt, ...);
int api_device_error(hipError_t e, const char* what);
void api_clear_error();

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int kQW = 16;             // queries per wave
constexpr int kWaves = 4;           // waves per work-group
constexpr int kQB = kQW * kWaves;   // queries per work-group
constexpr int kSubF = 8;            // pending keys per lane quarter
constexpr int kBufF = 4 * kSubF;    // pending keys per query
constexpr uint32_t kMaxDimMfma = 512;

__device__ __forceinline__ void fwave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// |x_r|^2 in FP32, one wave per row (lanes over the dimensions, then a tree).
__global__ __launch_bounds__(256) void sq_norms_kernel(const float* __restrict__ x, uint32_t n,
                                                       uint32_t d, float* __restrict__ out) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t r = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= n) return;
  const float* xr = x + (size_t)r * d;
  float s = 0.f;
  for (uint32_t k = lane; k < d; k += 64) s += xr[k] * xr[k];
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) s += __shfl_xor(s, m, 64);
  if (lane == 0) out[r] = s;
}

// s_waitcnt for at most n outstanding vector-memory operations, nothing else
// (gfx9 encoding: vmcnt in bits 3:0 and 15:14).
#define FKNN_WAIT_VMCNT(n) \
  __builtin_amdgcn_s_waitcnt(((n) & 15) | (((n) >> 4) << 14) | (7 << 4) | (15 << 8))

// One 16-byte-per-lane copy from global memory straight into LDS: lane l's 16
// bytes land at LDS address lds + 16 l (lds is wave-uniform, in M0). Written
// as inline assembly so the compiler does not track it; its completion is
// waited for explicitly (vector-memory counter) before the barrier that hands
// the buffer to the other waves. It has no register destination.
#pragma clang diagnostic push
#pragma clang diagnostic ignored "-Winline-asm"  // m0 is clobbered on purpose
__device__ __forceinline__ void dma16_lds(const void* gptr, uint32_t lds) {
  asm volatile(
      "s_mov_b32 m0, %1\n\t"
      "s_nop 0\n\t"
      "global_load_lds_dwordx4 %0, off"
      :
      : "v"(gptr), "s"(lds)
      : "memory", "m0");
}
#pragma clang diagnostic pop

__device__ __forceinline__ uint64_t fkey(float dist, uint32_t idx) {
  return ((uint64_t)__float_as_uint(dist) << 32) | idx;
}

template <int NR>
__device__ __forceinline__ float list_kth(const uint64_t (&R)[NR], uint32_t K) {
  uint64_t k = kNone64;
#pragma unroll
  for (int r = 0; r < NR; ++r)
    if ((uint32_t)r == (K - 1) / 64) {
      const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(R[r] >> 32), (K - 1) & 63);
      const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)R[r], (K - 1) & 63);
      k = ((uint64_t)hi << 32) | lo;
    }
  return k == kNone64 ? INFINITY : __uint_as_float((uint32_t)(k >> 32));
}

// Work-group: 64 queries (4 waves of 16) against base rows [c0, c1) of split
// blockIdx.y. NT4 = dimension chunks of 16 held per query (d <= 16 NT4),
// NR = list registers per lane (K <= 64 NR).
template <int NT4, int NR>
__global__ __launch_bounds__(256) void fknn_mfma_kernel(
    const float* __restrict__ Q, uint32_t nq, const float* __restrict__ Y, uint32_t d,
    const float* __restrict__ qn, const float* __restrict__ yn, const int32_t* __restrict__ exclude,
    uint32_t K, uint32_t nb, uint32_t chunk, uint64_t* __restrict__ part,
    uint32_t* __restrict__ out_idx, float* __restrict__ out_dist) {
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr int SV = NT4 * 64;  // float4 of one staged group
  static_assert(NT4 % kWaves == 0, "each wave copies whole slices");
  v4f* stage = reinterpret_cast<v4f*>(smem);                           // [2][SV]
  uint64_t* lists = reinterpret_cast<uint64_t*>(smem + 2 * SV * 16);   // [4][16][K]
  uint64_t* bufs = lists + (size_t)kWaves * kQW * K;                   // [4][16 * 32 + 64]

  const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6;
  const uint32_t i16 = lane & 15u, kq = lane >> 4;
  const uint32_t c0 = blockIdx.y * chunk;
  const uint32_t c1 = nb - c0 < chunk ? nb : c0 + chunk;
  const uint32_t qw0 = blockIdx.x * kQB + wave * kQW;  // first query of the wave
  const uint32_t qi = qw0 + i16;                       // this lane's query
  const bool qvalid = qi < nq;

  v4f bq[NT4];
#pragma unroll
  for (int t = 0; t < NT4; ++t) {
    const uint32_t dim = 16 * t + 4 * kq;
    bq[t] = (qvalid && dim < d) ? *reinterpret_cast<const v4f*>(Q + (size_t)qi * d + dim)
                                : v4f{0.f, 0.f, 0.f, 0.f};
  }
  const float qq = qvalid ? qn[qi] : 0.f;
  const int32_t ex = (qvalid && exclude) ? exclude[qi] : -1;
  float thr = qvalid ? INFINITY : -1.f;  // an absent query never admits
  uint32_t csub = 0;                     // keys in this lane's sub-buffer
  uint64_t* list_w = lists + (size_t)wave * kQW * K;
  uint64_t* buf_w = bufs + (size_t)wave * (kQW * kBufF + 64);
  const uint32_t discard = kQW * kBufF + lane;
  for (uint32_t p = lane; p < kQW * K; p += 64) list_w[p] = kNone64;

  // Stage copies, straight from global memory into LDS: slice t of group g
  // (1 KB) is one copy by one wave, lane l fetching row 16 g + l % 16,
  // dimensions 16 t + 4 (l / 16) .. + 3 into the 16 bytes at l. Rows past the
  // split and dimensions past d read a valid address instead (row c1 - 1,
  // dimension 0): their products are either never admitted (rows) or
  // multiplied by a zero query component (dimensions).
  const uint32_t lds_stage = (uint32_t)(uintptr_t)(__attribute__((address_space(3))) void*)stage;
  auto load_group = [&](uint32_t g, uint32_t buf) {
    uint32_t row = c0 + 16 * g + i16;
    row = row < c1 ? row : c1 - 1;
#pragma unroll
    for (int i = 0; i < NT4 / kWaves; ++i) {
      const uint32_t t = wave + kWaves * i;
      const uint32_t dim = 16 * t + 4 * kq;
      const float* src = Y + (size_t)row * d + (dim < d ? dim : 0u);
      dma16_lds(src, __builtin_amdgcn_readfirstlane(lds_stage + (buf * SV + t * 64) * 16));
    }
  };

  // Merge the pending keys of the queries flagged in m (a ballot over lanes)
  // into their lists; refresh those queries' thresholds.
  auto flush = [&](uint64_t m) {
    uint32_t qm = (uint32_t)(m | (m >> 16) | (m >> 32) | (m >> 48)) & 0xFFFFu;
    fwave_sync();
    while (qm) {
      const uint32_t i = __builtin_ctz(qm);
      qm &= qm - 1;
      // lanes 0..31 hold the query's pending slots (sub-buffer lane / 8)
      uint32_t cnt[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) cnt[t] = __builtin_amdgcn_readlane(csub, i + 16 * t);
      const uint32_t t = lane >> 3;
      const uint32_t ct = t == 0 ? cnt[0] : (t == 1 ? cnt[1] : (t == 2 ? cnt[2] : cnt[3]));
      const uint64_t x = (lane < 32u && (lane & 7u) < ct) ? buf_w[i * kBufF + lane] : kNone64;
      uint64_t R[NR];
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        const uint32_t p = 64 * r + lane;
        R[r] = p < K ? list_w[i * K + p] : kNone64;
      }
      merge64_into<NR>(R, x, lane);
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        const uint32_t p = 64 * r + lane;
        if (p < K) list_w[i * K + p] = R[r];
      }
      const float nt = list_kth<NR>(R, K);
      if (i16 == i) {
        thr = nt;
        csub = 0;
      }
      fwave_sync();
    }
  };

  const uint32_t ng = c1 > c0 ? (c1 - c0 + 15) / 16 : 0;
  if (ng > 0) load_group(0, 0);
  FKNN_WAIT_VMCNT(0);
  __syncthreads();
  for (uint32_t g = 0; g < ng; ++g) {
    const uint32_t buf = g & 1u;
    // the next group lands in the other buffer while this one's products run
    // (that buffer was last read in group g - 1, before the barrier below)
    if (g + 1 < ng) load_group(g + 1, buf ^ 1u);
    const v4f* sb = stage + buf * SV;
    // four accumulator chains (chunks t, t + 1, t + 2, t + 3), the next four
    // chunks' operands read from LDS while these are contracted
    v4f acc[4];
#pragma unroll
    for (int c4 = 0; c4 < 4; ++c4) acc[c4] = v4f{0.f, 0.f, 0.f, 0.f};
    v4f cur[4], nxt[4];
#pragma unroll
    for (int c4 = 0; c4 < 4; ++c4) cur[c4] = sb[c4 * 64 + lane];
#pragma unroll
    for (int t = 0; t < NT4; t += 4) {
      if (t + 4 < NT4) {
#pragma unroll
        for (int c4 = 0; c4 < 4; ++c4) nxt[c4] = sb[(t + 4 + c4) * 64 + lane];
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int c4 = 0; c4 < 4; ++c4)
          acc[c4] = __builtin_amdgcn_mfma_f32_16x16x4f32(cur[c4][s], bq[t + c4][s], acc[c4], 0, 0, 0);
      __builtin_amdgcn_sched_barrier(0);
      if (t + 4 < NT4) {
#pragma unroll
        for (int c4 = 0; c4 < 4; ++c4) cur[c4] = nxt[c4];
      }
    }
    // lane (i16, kq) holds <q_i16, y_r> for rows r = 16 g + 4 kq + 0..3
    const uint32_t rb = c0 + 16 * g + 4 * kq;
    float dd[4];
    uint32_t pass[4], c = 0;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const uint32_t row = rb + r;
      const float dot = (acc[0][r] + acc[1][r]) + (acc[2][r] + acc[3][r]);
      const float yy = row < c1 ? yn[row] : 0.f;
      dd[r] = fmaxf(qq + yy - 2.f * dot, 0.f);
      pass[r] = (row < c1 && (int32_t)row != ex && dd[r] < thr) ? 1u : 0u;
      c += pass[r];
    }
    if (__any(c > 0)) {
      const uint64_t over = __ballot(csub + c > (uint32_t)kSubF);
      if (over) {
        flush(over);
#pragma unroll
        for (int r = 0; r < 4; ++r) pass[r] = pass[r] && dd[r] < thr;  // tighter now
        c = pass[0] + pass[1] + pass[2] + pass[3];
      }
      uint32_t pos = i16 * kBufF + kq * kSubF + csub;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        buf_w[pass[r] ? pos : discard] = fkey(dd[r], rb + r);
        pos += pass[r];
      }
      csub += c;
    }
    FKNN_WAIT_VMCNT(0);  // this wave's copies of group g + 1 have landed
    __syncthreads();
  }
  const uint64_t m = __ballot(csub > 0);
  if (m) flush(m);
  fwave_sync();
  for (uint32_t p = lane; p < kQW * K; p += 64) {
    const uint32_t q = qw0 + p / K;
    if (q >= nq) break;
    const uint64_t key = list_w[p];
    const size_t o = (size_t)q * K + p % K;
    if (part) {
      part[(size_t)blockIdx.y * nq * K + o] = key;
    } else {
      out_idx[o] = key == kNone64 ? 0xFFFFFFFFu : (uint32_t)key;
      out_dist[o] = key == kNone64 ? INFINITY : __uint_as_float((uint32_t)(key >> 32));
    }
  }
}

// Top-K of the union of the splits' lists (disjoint index ranges), one wave
// per query.
template <int NR>
__global__ __launch_bounds__(256) void fknn_merge_kernel(const uint64_t* __restrict__ part,
                                                         uint32_t nsplit, uint32_t nq, uint32_t K,
                                                         uint32_t* __restrict__ out_idx,
                                                         float* __restrict__ out_dist) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t q = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (q >= nq) return;
  uint64_t R[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const uint32_t p = 64 * r + lane;
    R[r] = p < K ? part[(size_t)q * K + p] : kNone64;
  }
  for (uint32_t s = 1; s < nsplit; ++s)
    for (uint32_t c = 0; c < K; c += 64) {
      const uint32_t p = c + lane;
      merge64_into<NR>(R, p < K ? part[((size_t)s * nq + q) * K + p] : kNone64, lane);
    }
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const uint32_t p = 64 * r + lane;
    if (p < K) {
      const size_t o = (size_t)q * K + p;
      out_idx[o] = R[r] == kNone64 ? 0xFFFFFFFFu : (uint32_t)R[r];
      out_dist[o] = R[r] == kNone64 ? INFINITY : __uint_as_float((uint32_t)(R[r] >> 32));
    }
  }
}

// Other shapes (d not a multiple of 4, or d > 512): one wave per query, one
// base row per lane, distances by direct sums in FP32 over the dimensions in
// order; the same key order and strict threshold.
template <int NR>
__global__ __launch_bounds__(256) void fknn_valu_kernel(const float* __restrict__ Q, uint32_t nq,
                                                        const float* __restrict__ Y, uint32_t nb,
                                                        uint32_t d, const int32_t* __restrict__ exclude,
                                                        uint32_t K, uint32_t* __restrict__ out_idx,
                                                        float* __restrict__ out_dist) {
  __shared__ uint64_t pend[4][64];
  const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
  const uint32_t q = blockIdx.x * 4 + wave;
  if (q >= nq) return;
  uint64_t* buf = pend[wave];
  const float* qr = Q + (size_t)q * d;
  const int32_t ex = exclude ? exclude[q] : -1;
  uint64_t R[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) R[r] = kNone64;
  float thr = INFINITY;
  uint32_t cnt = 0;
  for (uint32_t j0 = 0; j0 < nb; j0 += 64) {
    const uint32_t j = j0 + lane;
    float dist = INFINITY;
    if (j < nb && (int32_t)j != ex) {
      const float* yr = Y + (size_t)j * d;
      float s = 0.f;
      for (uint32_t k = 0; k < d; ++k) {
        const float t = qr[k] - yr[k];
        s += t * t;
      }
      dist = s;
    }
    bool pass = dist < thr;
    uint64_t m = __ballot(pass);
    if (!m) continue;
    uint32_t c = (uint32_t)__popcll(m);
    if (cnt + c > 64) {
      fwave_sync();
      merge64_into<NR>(R, lane < cnt ? buf[lane] : kNone64, lane);
      cnt = 0;
      thr = list_kth<NR>(R, K);
      pass = dist < thr;
      m = __ballot(pass);
      c = (uint32_t)__popcll(m);
    }
    if (pass) {
      const uint32_t below =
          __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
      buf[cnt + below] = fkey(dist, j);
    }
    cnt += c;
    fwave_sync();
  }
  if (cnt) merge64_into<NR>(R, lane < cnt ? buf[lane] : kNone64, lane);
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const uint32_t p = 64 * r + lane;
    if (p < K) {
      const size_t o = (size_t)q * K + p;
      out_idx[o] = R[r] == kNone64 ? 0xFFFFFFFFu : (uint32_t)R[r];
      out_dist[o] = R[r] == kNone64 ? INFINITY : __uint_as_float((uint32_t)(R[r] >> 32));
    }
  }
}

size_t mfma_lds_bytes(int nt4, uint32_t K) {
  return (size_t)2 * nt4 * 64 * 16 + (size_t)kWaves * kQW * K * 8 +
         (size_t)kWaves * (kQW * kBufF + 64) * 8;
}

template <int NT4, int NR>
hipError_t launch_mfma(const float* Q, uint32_t nq, const float* Y, uint32_t nb, uint32_t d,
                       const float* qn, const float* yn, const int32_t* ex, uint32_t K,
                       uint32_t nsplit, uint32_t chunk, uint64_t* part, uint32_t* out_idx,
                       float* out_dist, hipStream_t s) {
  auto kern = fknn_mfma_kernel<NT4, NR>;
  const size_t lds = mfma_lds_bytes(NT4, K);
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  dim3 grid((nq + kQB - 1) / kQB, nsplit);
  hipLaunchKernelGGL(kern, grid, dim3(256), lds, s, Q, nq, Y, d, qn, yn, ex, K, nb, chunk,
                     nsplit > 1 ? part : nullptr, out_idx, out_dist);
  return hipGetLastError();
}

template <int NR>
hipError_t launch_mfma_nt4(int nt4, const float* Q, uint32_t nq, const float* Y, uint32_t nb,
                           uint32_t d, const float* qn, const float* yn, const int32_t* ex,
                           uint32_t K, uint32_t nsplit, uint32_t chunk, uint64_t* part,
                           uint32_t* oi, float* od, hipStream_t s) {
  switch (nt4) {
    case 4: return launch_mfma<4, NR>(Q, nq, Y, nb, d, qn, yn, ex, K, nsplit, chunk, part, oi, od, s);
    case 8: return launch_mfma<8, NR>(Q, nq, Y, nb, d, qn, yn, ex, K, nsplit, chunk, part, oi, od, s);
    case 16: return launch_mfma<16, NR>(Q, nq, Y, nb, d, qn, yn, ex, K, nsplit, chunk, part, oi, od, s);
    case 32: return launch_mfma<32, NR>(Q, nq, Y, nb, d, qn, yn, ex, K, nsplit, chunk, part, oi, od, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace
}  // namespace bdg

extern "C" {

int bdg_float_knn(const float* queries, uint32_t nq, const float* base, uint32_t nb, uint32_t d,
                  uint32_t K, const int32_t* exclude, uint32_t* out_idx, float* out_dist,
                  void* stream) {
  using namespace bdg;
  api_clear_error();
  if (K == 0 || K > 128) return api_error(BDG_EUNSUPPORTED, "K must be 1..128");
  if (d == 0) return api_error(BDG_EINVAL, "d must be >= 1");
  if (nq == 0) return BDG_OK;
  if (!queries || !base || !out_idx || !out_dist) return api_error(BDG_EINVAL, "null pointer");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const int NR = K <= 64 ? 1 : 2;
  (void)hipGetLastError();
  hipError_t e = hipSuccess;
  if (d % 4 != 0 || d > kMaxDimMfma) {
    dim3 grid((nq + 3) / 4);
    if (NR == 1)
      hipLaunchKernelGGL(fknn_valu_kernel<1>, grid, dim3(256), 0, s, queries, nq, base, nb, d,
                         exclude, K, out_idx, out_dist);
    else
      hipLaunchKernelGGL(fknn_valu_kernel<2>, grid, dim3(256), 0, s, queries, nq, base, nb, d,
                         exclude, K, out_idx, out_dist);
    e = hipGetLastError();
    return e == hipSuccess ? BDG_OK : api_device_error(e, "float kNN");
  }
  const int nt4 = d <= 64 ? 4 : (d <= 128 ? 8 : (d <= 256 ? 16 : 32));
  // Splits of the base: one work-group per CU runs at a time (its LDS), so
  // the launch is cut into whole rounds of CUs. The fewest splits whose
  // rounds are at least 97 % full (at least 4,096 base rows a split, at most
  // 64 splits); failing that, the fullest.
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess)
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  const uint32_t nqb = (nq + kQB - 1) / kQB;
  uint32_t max_split = nb / 4096 > 0 ? nb / 4096 : 1;
  if (max_split > 64) max_split = 64;
  uint32_t nsplit = 1;
  double best = 0.0;
  for (uint32_t sp = 1; sp <= max_split; ++sp) {
    const double wgs = (double)nqb * sp;
    const double fill = wgs / (ceil(wgs / cus) * cus);
    if (fill > best + 1e-9) {
      best = fill;
      nsplit = sp;
    }
    if (fill >= 0.97) break;
  }
  uint32_t chunk = nb ? (nb + nsplit - 1) / nsplit : 0;
  chunk = (chunk + 15) & ~15u;
  if (chunk == 0) chunk = 16;
  nsplit = nb ? (nb + chunk - 1) / chunk : 1;
  const size_t nbytes = ((size_t)nq + nb + 64) * 4;
  const size_t pbytes = nsplit > 1 ? (size_t)nsplit * nq * K * 8 : 0;
  void* ws = nullptr;
  e = hipMallocAsync(&ws, nbytes + pbytes + 256, s);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return api_error(BDG_ENOMEM, "float kNN workspace of %zu bytes", nbytes + pbytes);
  }
  uint64_t* part = static_cast<uint64_t*>(ws);
  float* qn = reinterpret_cast<float*>(static_cast<char*>(ws) + ((pbytes + 255) & ~size_t(255)));
  float* yn = qn + ((nq + 63) & ~63u);
  hipLaunchKernelGGL(sq_norms_kernel, dim3((nq + 3) / 4), dim3(256), 0, s, queries, nq, d, qn);
  if (nb) hipLaunchKernelGGL(sq_norms_kernel, dim3((nb + 3) / 4), dim3(256), 0, s, base, nb, d, yn);
  e = hipGetLastError();
  if (e == hipSuccess)
    e = NR == 1 ? launch_mfma_nt4<1>(nt4, queries, nq, base, nb, d, qn, yn, exclude, K, nsplit,
                                     chunk, part, out_idx, out_dist, s)
                : launch_mfma_nt4<2>(nt4, queries, nq, base, nb, d, qn, yn, exclude, K, nsplit,
                                     chunk, part, out_idx, out_dist, s);
  if (e == hipSuccess && nsplit > 1) {
    dim3 grid((nq + 3) / 4);
    if (NR == 1)
      hipLaunchKernelGGL(fknn_merge_kernel<1>, grid, dim3(256), 0, s, part, nsplit, nq, K, out_idx,
                         out_dist);
    else
      hipLaunchKernelGGL(fknn_merge_kernel<2>, grid, dim3(256), 0, s, part, nsplit, nq, K, out_idx,
                         out_dist);
    e = hipGetLastError();
  }
  hipError_t f = hipFreeAsync(ws, s);
  if (e == hipSuccess) e = f;
  return e == hipSuccess ? BDG_OK : api_device_error(e, "float kNN");
}

}  // extern "C"
