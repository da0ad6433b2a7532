// Binarisers and the real-valued ground truth (gfx950).
//
// The paper maps real-valued CNN features to binary codes that preserve their
// locality (Sec. 3.1, learned hashing), and measures recall against
// real-valued brute force (Sec. 4.2, Eq. 3). This file holds the GPU side of
// that part of the path:
//   * sign-of-random-projection encoding on the FP32 matrix cores, with the
//     sign and the bit packing fused (the plain binariser);
//   * a small MLP encoder (d -> h -> bits, tanh) whose products are BF16
//     matrix-core contractions with FP32 accumulation, its backward pass, a
//     triplet loss on relaxed Hamming distances, and Adam;
// (the exact squared-L2 kNN in FP32 that measures recall is in fknn.hip).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "bdg.h"
#include "kernels.h"

namespace bdg {
int api_error(int status, const char* fmt, ...);
int api_device_error(hipError_t e, const char* what);
void api_clear_error();

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

__device__ __forceinline__ uint16_t to_bf16(float f) {  // round to nearest even
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// -------------------------------------------------------------- SRP encode --

// Codes of 64 rows per work-group (16 per wave), one 64-bit word (64
// projections) per pass: acc[t] = rows x projections [16 t, 16 t + 16) of the
// word, by v_mfma_f32_16x16x4_f32 over d in chunks of 16. Lane (i, q) holds
// row i's x[k0 + 4 q .. + 4) (one 16-byte load) and feeds k-step s with element
// s; the projection chunk (16 x 64 floats) is staged in LDS and read with the
// same k map (row 4 q + s). Bit j = [<x, w_j> > 0].
__global__ __launch_bounds__(256) void srp_encode_kernel(const float* __restrict__ x, uint32_t n,
                                                         uint32_t d, const float* __restrict__ proj,
                                                         uint32_t bits,
                                                         uint64_t* __restrict__ out) {
  __shared__ float pc[16][64];
  const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6;
  const uint32_t i = lane & 15u, q = lane >> 4;
  const uint32_t row0 = blockIdx.x * 64 + wave * 16;
  const uint32_t row = row0 + i;
  const float* xr = x + (size_t)(row < n ? row : n - 1) * d;
  const uint32_t W = bits / 64;
  for (uint32_t w = 0; w < W; ++w) {
    v4f acc[4] = {{0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}};
    for (uint32_t k0 = 0; k0 < d; k0 += 16) {
      __syncthreads();
      {
        const uint32_t r = tid >> 4, c = (tid & 15u) * 4;  // 16 rows x 64 columns
        const float4 v = *reinterpret_cast<const float4*>(proj + (size_t)(k0 + r) * bits +
                                                          64 * w + c);
        pc[r][c] = v.x;
        pc[r][c + 1] = v.y;
        pc[r][c + 2] = v.z;
        pc[r][c + 3] = v.w;
      }
      __syncthreads();
      const float4 a = *reinterpret_cast<const float4*>(xr + k0 + 4 * q);
      const float av[4] = {a.x, a.y, a.z, a.w};
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int t = 0; t < 4; ++t)
          acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[s], pc[4 * q + s][16 * t + i], acc[t],
                                                        0, 0, 0);
    }
    // lane (i, q) holds rows 4 q + r, projection 16 t + i: pack row words
    uint64_t word = 0;  // lanes 0..15: row (lane) of the wave
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const uint64_t m = __ballot(acc[t][r] > 0.0f);
        // row 4 g + r sits in lanes [16 g, 16 g + 16) of m
        const uint32_t g = lane >> 2;
        if ((lane & 3u) == (uint32_t)r && lane < 16)
          word |= ((m >> (16 * g)) & 0xFFFFull) << (16 * t);
      }
    if (lane < 16 && row0 + lane < n) out[(size_t)(row0 + lane) * W + w] = word;
  }
}

// Sign of a real matrix, packed: bit j of row r = [z[r][j] > 0].
__global__ __launch_bounds__(256) void pack_signs_kernel(const float* __restrict__ z, uint32_t n,
                                                         uint32_t bits,
                                                         uint64_t* __restrict__ out) {
  const size_t t = (size_t)blockIdx.x * 256 + threadIdx.x;
  const uint32_t W = bits / 64;
  if (t >= (size_t)n * W) return;
  const float* zr = z + (t / W) * bits + (t % W) * 64;
  uint64_t word = 0;
  for (int j = 0; j < 64; ++j) word |= (uint64_t)(zr[j] > 0.0f) << j;
  out[t] = word;
}

// ------------------------------------------------------------ BF16 GEMM NT --

enum EpiKind { kEpiF32 = 0, kEpiBiasTanh = 1, kEpiBiasTanh2 = 2, kEpiDTanh = 3, kEpiBias = 4 };

struct Epi {
  int kind;
  float* f0;            // f32 output [M][N] (ldc)
  float* f1;            // second f32 output [M][N] (ldc)
  uint16_t* b0;         // bf16 output [M][N] (ldc)
  uint16_t* bt;         // bf16 transposed output [N][M] (ldt)
  uint32_t ldt;
  const float* bias;    // [N]
  const float* aux;     // [M][N] (ldc): tanh output whose derivative multiplies
  float* gbias;         // [N]: column sums of the result (atomic)
};

// C[m][n] = sum_k A[m][k] B[n][k] (both operands k-contiguous, bf16), FP32
// accumulation on v_mfma_f32_16x16x32_bf16; a 64 x 64 tile per work-group,
// 32 x 32 per wave (2 x 2 blocks). K % 32 == 0, lda and ldb multiples of 8.
__global__ __launch_bounds__(256) void gemm_nt_bf16_kernel(const uint16_t* __restrict__ A,
                                                           uint32_t lda,
                                                           const uint16_t* __restrict__ B,
                                                           uint32_t ldb, uint32_t M, uint32_t N,
                                                           uint32_t K, uint32_t ldc, Epi e) {
  const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6;
  const uint32_t i = lane & 15u, q = lane >> 4;
  const uint32_t mb = blockIdx.y * 64 + (wave >> 1) * 32;
  const uint32_t nb = blockIdx.x * 64 + (wave & 1) * 32;
  const uint16_t* ap[2];
  const uint16_t* bp[2];
  bool av[2], bv[2];
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const uint32_t m = mb + 16 * t + i, n = nb + 16 * t + i;
    av[t] = m < M;
    bv[t] = n < N;
    ap[t] = A + (size_t)(av[t] ? m : 0) * lda + 8 * q;
    bp[t] = B + (size_t)(bv[t] ? n : 0) * ldb + 8 * q;
  }
  v4f acc[2][2] = {{{0, 0, 0, 0}, {0, 0, 0, 0}}, {{0, 0, 0, 0}, {0, 0, 0, 0}}};
  const v8bf zero = {};
  v8bf a[2], b[2];
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    a[t] = av[t] ? *reinterpret_cast<const v8bf*>(ap[t]) : zero;
    b[t] = bv[t] ? *reinterpret_cast<const v8bf*>(bp[t]) : zero;
  }
  for (uint32_t k0 = 0; k0 < K; k0 += 32) {
    v8bf an[2], bn[2];
    const bool more = k0 + 32 < K;
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      an[t] = (av[t] && more) ? *reinterpret_cast<const v8bf*>(ap[t] + k0 + 32) : zero;
      bn[t] = (bv[t] && more) ? *reinterpret_cast<const v8bf*>(bp[t] + k0 + 32) : zero;
    }
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y)
        acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[x], b[y], acc[x][y], 0, 0, 0);
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      a[t] = an[t];
      b[t] = bn[t];
    }
  }
  // lane (i, q) holds C[mb + 16 x + 4 q + r][nb + 16 y + i]
#pragma unroll
  for (int y = 0; y < 2; ++y) {
    const uint32_t n = nb + 16 * y + i;
    float colsum = 0.f;
#pragma unroll
    for (int x = 0; x < 2; ++x) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const uint32_t m = mb + 16 * x + 4 * q + r;
        if (m >= M || n >= N) continue;
        const size_t o = (size_t)m * ldc + n;
        float v = acc[x][y][r];
        switch (e.kind) {
          case kEpiF32:
            e.f0[o] = v;
            break;
          case kEpiBias:
            e.f0[o] = v + e.bias[n];
            break;
          case kEpiBiasTanh: {
            v = tanhf(v + e.bias[n]);
            if (e.f0) e.f0[o] = v;
            if (e.b0) e.b0[o] = to_bf16(v);
            if (e.bt) e.bt[(size_t)n * e.ldt + m] = to_bf16(v);
            break;
          }
          case kEpiBiasTanh2:
            v += e.bias[n];
            e.f0[o] = v;
            e.f1[o] = tanhf(v);
            break;
          case kEpiDTanh: {
            const float h = e.aux[o];
            v *= 1.0f - h * h;
            if (e.bt) e.bt[(size_t)n * e.ldt + m] = to_bf16(v);
            colsum += v;
            break;
          }
        }
      }
    }
    if (e.kind == kEpiDTanh) {
      colsum += __shfl_xor(colsum, 16, 64);
      colsum += __shfl_xor(colsum, 32, 64);
      if (q == 0 && n < N) atomicAdd(e.gbias + n, colsum);
    }
  }
}

// -------------------------------------------------------- loss and helpers --

__global__ void zero_f32_kernel(float* p, size_t count) {
  const size_t t = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (t < count) p[t] = 0.f;
}

// mu[j] = mean over the rows of H[:, j]; loss = lam_b * sum mu^2 (one block,
// one thread per column).
__global__ __launch_bounds__(1024) void column_mean_kernel(const float* __restrict__ H,
                                                           uint32_t rows, uint32_t bits,
                                                           float lam_b, float* __restrict__ mu,
                                                           float* __restrict__ loss) {
  __shared__ float part[1024];
  const uint32_t j = threadIdx.x;
  float m = 0.f;
  if (j < bits) {
    for (uint32_t r = 0; r < rows; ++r) m += H[(size_t)r * bits + j];
    m /= (float)rows;
    mu[j] = m;
  }
  part[j] = j < bits ? m * m : 0.f;
  __syncthreads();
  for (uint32_t s = 512; s > 0; s >>= 1) {
    if (j < s) part[j] += part[j + s];
    __syncthreads();
  }
  if (j == 0) *loss = lam_b * part[0];
}

struct LossArgs {
  uint32_t T, bits, rows_pad;
  float margin, tau, lam_q, lam_b;
};

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

// One wave per triplet t (rows t, T + t, 2T + t of H). Writes dZ2 = dL/dZ2
// (bf16, row-major [rows_pad][bits] and transposed [bits][rows_pad]), adds
// the column sums of dZ2 to gb2 and the loss terms to *loss.
__global__ __launch_bounds__(256) void triplet_loss_kernel(const float* __restrict__ H,
                                                           const float* __restrict__ mu, LossArgs a,
                                                           uint16_t* __restrict__ dz,
                                                           uint16_t* __restrict__ dzt,
                                                           float* __restrict__ gb2,
                                                           float* __restrict__ loss) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t t = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (t >= a.T) return;  // wave-uniform
  const uint32_t B = a.bits, T = a.T;
  const float R = 3.f * (float)T;
  const float* ha = H + (size_t)t * B;
  const float* hp = H + (size_t)(T + t) * B;
  const float* hn = H + (size_t)(2 * T + t) * B;
  float sap = 0.f, san = 0.f, q = 0.f;
  for (uint32_t j = lane; j < B; j += 64) {
    sap += ha[j] * hp[j];
    san += ha[j] * hn[j];
    const float e1 = fabsf(ha[j]) - 1.f, e2 = fabsf(hp[j]) - 1.f, e3 = fabsf(hn[j]) - 1.f;
    q += e1 * e1 + e2 * e2 + e3 * e3;
  }
  sap = wave_sum(sap);
  san = wave_sum(san);
  q = wave_sum(q);
  const float dap = 0.5f * ((float)B - sap), dan = 0.5f * ((float)B - san);
  const float z = (dap - dan + a.margin) / a.tau;
  const float sp = fmaxf(z, 0.f) + log1pf(expf(-fabsf(z)));
  const float g = 1.f / (1.f + expf(-z)) / (a.tau * (float)T);
  if (lane == 0) atomicAdd(loss, sp / (float)T + a.lam_q * q / (R * (float)B));
  const float cq = a.lam_q * 2.f / (R * (float)B), cb = a.lam_b * 2.f / R;
  const uint32_t rows[3] = {t, T + t, 2 * T + t};
  for (uint32_t j = lane; j < B; j += 64) {
    const float va = ha[j], vp = hp[j], vn = hn[j];
    const float bal = cb * mu[j];
    float dh[3];
    dh[0] = g * (0.5f * vn - 0.5f * vp);
    dh[1] = -g * 0.5f * va;
    dh[2] = g * 0.5f * va;
    const float hv[3] = {va, vp, vn};
    float col = 0.f;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const float h = hv[k];
      const float sg = h > 0.f ? 1.f : (h < 0.f ? -1.f : 0.f);
      const float d = (dh[k] + cq * (fabsf(h) - 1.f) * sg + bal) * (1.f - h * h);
      dz[(size_t)rows[k] * B + j] = to_bf16(d);
      dzt[(size_t)j * a.rows_pad + rows[k]] = to_bf16(d);
      col += d;
    }
    atomicAdd(gb2 + j, col);
  }
}

// Zero rows [from, rows_pad) of dZ2 (both layouts): padding rows of a batch.
__global__ void zero_rows_kernel(uint16_t* dz, uint16_t* dzt, uint32_t from, uint32_t rows_pad,
                                 uint32_t bits) {
  const size_t t = (size_t)blockIdx.x * 256 + threadIdx.x;
  const size_t cnt = (size_t)(rows_pad - from) * bits;
  if (t >= cnt) return;
  const uint32_t r = from + (uint32_t)(t / bits), j = (uint32_t)(t % bits);
  dz[(size_t)r * bits + j] = 0;
  dzt[(size_t)j * rows_pad + r] = 0;
}

// Rows idx[r] of X (scaled) as bf16, row-major and (optionally) transposed;
// idx == 0xFFFFFFFF gives a zero row.
__global__ void gather_rows_kernel(const float* __restrict__ X, uint32_t d,
                                   const uint32_t* __restrict__ idx, uint32_t row0,
                                   uint32_t rows, uint32_t rows_pad, float scale,
                                   uint16_t* __restrict__ xb, uint16_t* __restrict__ xt) {
  const size_t t = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= (size_t)rows_pad * d) return;
  const uint32_t r = (uint32_t)(t / d), k = (uint32_t)(t % d);
  float v = 0.f;
  if (r < rows) {
    const uint32_t src = idx ? idx[r] : row0 + r;
    if (src != 0xFFFFFFFFu) v = X[(size_t)src * d + k] * scale;
  }
  const uint16_t b = to_bf16(v);
  xb[t] = b;
  if (xt) xt[(size_t)k * rows_pad + r] = b;
}

__global__ void adam_kernel(float* __restrict__ p, const float* __restrict__ g,
                            float* __restrict__ m, float* __restrict__ v, size_t count, float lr,
                            float b1, float b2, float eps, float c1, float c2) {
  const size_t t = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= count) return;
  const float gt = g[t];
  const float mt = b1 * m[t] + (1.f - b1) * gt;
  const float vt = b2 * v[t] + (1.f - b2) * gt * gt;
  m[t] = mt;
  v[t] = vt;
  p[t] -= lr * (mt / c1) / (sqrtf(vt / c2) + eps);
}

// bf16 copies of a [rows][cols] matrix: row-major and/or transposed.
__global__ void to_bf16_kernel(const float* __restrict__ w, uint32_t rows, uint32_t cols,
                               uint16_t* __restrict__ b, uint16_t* __restrict__ bt) {
  const size_t t = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= (size_t)rows * cols) return;
  const uint32_t r = (uint32_t)(t / cols), c = (uint32_t)(t % cols);
  const uint16_t v = to_bf16(w[t]);
  if (b) b[t] = v;
  if (bt) bt[(size_t)c * rows + r] = v;
}


unsigned blocks_for(size_t count) { return (unsigned)((count + 255) / 256); }

hipError_t gemm(const uint16_t* A, uint32_t lda, const uint16_t* B, uint32_t ldb, uint32_t M,
                uint32_t N, uint32_t K, uint32_t ldc, const Epi& e, hipStream_t s) {
  dim3 grid((N + 63) / 64, (M + 63) / 64);
  hipLaunchKernelGGL(gemm_nt_bf16_kernel, grid, dim3(256), 0, s, A, lda, B, ldb, M, N, K, ldc, e);
  return hipGetLastError();
}

Epi epi(int kind) {
  Epi e;
  e.kind = kind;
  e.f0 = e.f1 = nullptr;
  e.b0 = e.bt = nullptr;
  e.ldt = 0;
  e.bias = e.aux = nullptr;
  e.gbias = nullptr;
  return e;
}

}  // namespace
}  // namespace bdg

using namespace bdg;

extern "C" {

int bdg_encode(const float* x, uint32_t n, uint32_t d, const float* proj, uint32_t bits,
               uint64_t* out_codes, void* stream) {
  api_clear_error();
  if (bits == 0 || bits % 64 != 0 || bits > BDG_MAX_BITS)
    return api_error(BDG_EINVAL, "bits must be a multiple of 64, at most %u", BDG_MAX_BITS);
  if (d == 0 || d % 16 != 0) return api_error(BDG_EINVAL, "d must be a positive multiple of 16");
  if (n == 0) return BDG_OK;
  if (!x || !proj || !out_codes) return api_error(BDG_EINVAL, "null device pointer");
  (void)hipGetLastError();
  hipLaunchKernelGGL(srp_encode_kernel, dim3((n + 63) / 64), dim3(256), 0,
                     reinterpret_cast<hipStream_t>(stream), x, n, d, proj, bits, out_codes);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? BDG_OK : api_device_error(e, "encode launch");
}

int bdg_pack_signs(const float* z, uint32_t n, uint32_t bits, uint64_t* out_codes, void* stream) {
  api_clear_error();
  if (bits == 0 || bits % 64 != 0) return api_error(BDG_EINVAL, "bits must be a multiple of 64");
  if (n == 0) return BDG_OK;
  if (!z || !out_codes) return api_error(BDG_EINVAL, "null device pointer");
  (void)hipGetLastError();
  hipLaunchKernelGGL(pack_signs_kernel, dim3(blocks_for((size_t)n * (bits / 64))), dim3(256), 0,
                     reinterpret_cast<hipStream_t>(stream), z, n, bits, out_codes);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? BDG_OK : api_device_error(e, "pack launch");
}

int bdg_gemm_nt_bf16(const uint16_t* A, uint32_t lda, const uint16_t* B, uint32_t ldb, uint32_t M,
                     uint32_t N, uint32_t K, float* C, uint32_t ldc, void* stream) {
  api_clear_error();
  if (K % 32 != 0 || lda % 8 != 0 || ldb % 8 != 0 || lda < K || ldb < K || ldc < N)
    return api_error(BDG_EINVAL, "K %% 32, lda %% 8, ldb %% 8 must be 0; lda, ldb >= K; ldc >= N");
  if (!M || !N || !K) return BDG_OK;
  if (!A || !B || !C) return api_error(BDG_EINVAL, "null device pointer");
  (void)hipGetLastError();
  Epi e = epi(kEpiF32);
  e.f0 = C;
  hipError_t err = gemm(A, lda, B, ldb, M, N, K, ldc, e, reinterpret_cast<hipStream_t>(stream));
  return err == hipSuccess ? BDG_OK : api_device_error(err, "gemm launch");
}

static int mlp_check(const bdg_mlp_params* p, const bdg_mlp_acts* a) {
  if (!p || !a) return api_error(BDG_EINVAL, "params or activations are NULL");
  if (p->d % 32 || p->h % 64 || p->bits % 64 || !p->d || !p->h || !p->bits || p->bits > 1024)
    return api_error(BDG_EINVAL, "d %% 32, h %% 64, bits %% 64 must be 0 (bits <= 1024)");
  if (a->rows_pad % 32 || a->rows > a->rows_pad)
    return api_error(BDG_EINVAL, "rows_pad must be a multiple of 32 and >= rows");
  return BDG_OK;
}

int bdg_mlp_gather(const float* X, uint32_t d, const uint32_t* idx, uint32_t rows, float scale,
                   bdg_mlp_acts* a, void* stream) {
  api_clear_error();
  if (!a || !X || !a->Xb) return api_error(BDG_EINVAL, "null pointer");
  if (a->rows_pad % 32 || rows > a->rows_pad)
    return api_error(BDG_EINVAL, "rows_pad must be a multiple of 32 and >= rows");
  a->rows = rows;
  (void)hipGetLastError();
  hipLaunchKernelGGL(gather_rows_kernel, dim3(blocks_for((size_t)a->rows_pad * d)), dim3(256), 0,
                     reinterpret_cast<hipStream_t>(stream), X, d, idx, 0u, rows, a->rows_pad,
                     scale, a->Xb, a->Xt);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? BDG_OK : api_device_error(e, "gather launch");
}

int bdg_mlp_forward(const bdg_mlp_params* p, bdg_mlp_acts* a, void* stream) {
  api_clear_error();
  int st = mlp_check(p, a);
  if (st != BDG_OK) return st;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  (void)hipGetLastError();
  Epi e1 = epi(kEpiBiasTanh);
  e1.f0 = a->H1;
  e1.b0 = a->H1b;
  e1.bt = a->H1t;
  e1.ldt = a->rows_pad;
  e1.bias = p->b1;
  hipError_t err = gemm(a->Xb, p->d, p->W1b, p->d, a->rows_pad, p->h, p->d, p->h, e1, s);
  if (err == hipSuccess) {
    Epi e2 = epi(a->H ? kEpiBiasTanh2 : kEpiBias);
    e2.f0 = a->Z2;
    e2.f1 = a->H;
    e2.bias = p->b2;
    err = gemm(a->H1b, p->h, p->W2b, p->h, a->rows_pad, p->bits, p->h, p->bits, e2, s);
  }
  return err == hipSuccess ? BDG_OK : api_device_error(err, "forward launch");
}

int bdg_triplet_loss(const bdg_mlp_acts* a, uint32_t bits, uint32_t T, const bdg_loss_opts* o,
                     float* mu, float* gb2, float* loss, void* stream) {
  api_clear_error();
  if (!a || !o || !mu || !gb2 || !loss || !a->H || !a->dZ2b || !a->dZ2t)
    return api_error(BDG_EINVAL, "null pointer");
  if (bits % 64 || bits > 1024 || 3 * T > a->rows_pad || T == 0)
    return api_error(BDG_EINVAL, "bits %% 64 must be 0 (<= 1024) and 3 T <= rows_pad");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  (void)hipGetLastError();
  hipLaunchKernelGGL(zero_f32_kernel, dim3(blocks_for(bits)), dim3(256), 0, s, gb2, (size_t)bits);
  hipLaunchKernelGGL(column_mean_kernel, dim3(1), dim3(1024), 0, s, a->H, 3 * T, bits, o->lam_b,
                     mu, loss);
  LossArgs la;
  la.T = T;
  la.bits = bits;
  la.rows_pad = a->rows_pad;
  la.margin = o->margin;
  la.tau = o->tau;
  la.lam_q = o->lam_q;
  la.lam_b = o->lam_b;
  hipLaunchKernelGGL(triplet_loss_kernel, dim3((T + 3) / 4), dim3(256), 0, s, a->H, mu, la,
                     a->dZ2b, a->dZ2t, gb2, loss);
  if (3 * T < a->rows_pad)
    hipLaunchKernelGGL(zero_rows_kernel, dim3(blocks_for((size_t)(a->rows_pad - 3 * T) * bits)),
                       dim3(256), 0, s, a->dZ2b, a->dZ2t, 3 * T, a->rows_pad, bits);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? BDG_OK : api_device_error(e, "loss launch");
}

int bdg_mlp_backward(const bdg_mlp_params* p, const bdg_mlp_acts* a, bdg_mlp_grads* g,
                     void* stream) {
  api_clear_error();
  int st = mlp_check(p, a);
  if (st != BDG_OK) return st;
  if (!g || !g->W1 || !g->b1 || !g->W2) return api_error(BDG_EINVAL, "null gradient pointer");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  (void)hipGetLastError();
  const uint32_t R = a->rows_pad;
  hipLaunchKernelGGL(zero_f32_kernel, dim3(blocks_for(p->h)), dim3(256), 0, s, g->b1,
                     (size_t)p->h);
  Epi w2 = epi(kEpiF32);  // dW2 [bits][h] = dZ2^T H1
  w2.f0 = g->W2;
  hipError_t e = gemm(a->dZ2t, R, a->H1t, R, p->bits, p->h, R, p->h, w2, s);
  if (e == hipSuccess) {  // dZ1 = (dZ2 W2) * (1 - H1^2), stored transposed; db1
    Epi d1 = epi(kEpiDTanh);
    d1.aux = a->H1;
    d1.bt = a->dZ1t;
    d1.ldt = R;
    d1.gbias = g->b1;
    e = gemm(a->dZ2b, p->bits, p->W2bt, p->bits, R, p->h, p->bits, p->h, d1, s);
  }
  if (e == hipSuccess) {  // dW1 [h][d] = dZ1^T X
    Epi w1 = epi(kEpiF32);
    w1.f0 = g->W1;
    e = gemm(a->dZ1t, R, a->Xt, R, p->h, p->d, R, p->d, w1, s);
  }
  return e == hipSuccess ? BDG_OK : api_device_error(e, "backward launch");
}

int bdg_adam_step(float* param, const float* grad, float* m, float* v, size_t count, uint32_t t,
                  float lr, float beta1, float beta2, float eps, void* stream) {
  api_clear_error();
  if (t == 0) return api_error(BDG_EINVAL, "step t counts from 1");
  if (!count) return BDG_OK;
  if (!param || !grad || !m || !v) return api_error(BDG_EINVAL, "null device pointer");
  const float c1 = 1.f - powf(beta1, (float)t), c2 = 1.f - powf(beta2, (float)t);
  (void)hipGetLastError();
  hipLaunchKernelGGL(adam_kernel, dim3(blocks_for(count)), dim3(256), 0,
                     reinterpret_cast<hipStream_t>(stream), param, grad, m, v, count, lr, beta1,
                     beta2, eps, c1, c2);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? BDG_OK : api_device_error(e, "adam launch");
}

int bdg_mlp_refresh(const bdg_mlp_params* p, void* stream) {
  api_clear_error();
  if (!p || !p->W1 || !p->W2 || !p->W1b || !p->W2b || !p->W2bt)
    return api_error(BDG_EINVAL, "null pointer");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  (void)hipGetLastError();
  hipLaunchKernelGGL(to_bf16_kernel, dim3(blocks_for((size_t)p->h * p->d)), dim3(256), 0, s,
                     p->W1, p->h, p->d, p->W1b, (uint16_t*)nullptr);
  hipLaunchKernelGGL(to_bf16_kernel, dim3(blocks_for((size_t)p->bits * p->h)), dim3(256), 0, s,
                     p->W2, p->bits, p->h, p->W2b, p->W2bt);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? BDG_OK : api_device_error(e, "refresh launch");
}

int bdg_mlp_encode(const bdg_mlp_params* p, const float* X, uint32_t n, float scale,
                   uint64_t* out_codes, void* stream) {
  api_clear_error();
  if (!p || !X || !out_codes) return api_error(BDG_EINVAL, "null pointer");
  if (p->d % 32 || p->h % 64 || p->bits % 64 || p->bits > 1024)
    return api_error(BDG_EINVAL, "d %% 32, h %% 64, bits %% 64 must be 0");
  if (n == 0) return BDG_OK;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const uint32_t chunk = 32768;
  const size_t xb = (size_t)chunk * p->d * 2, hb = (size_t)chunk * p->h * 2,
               zb = (size_t)chunk * p->bits * 4;
  void* ws = nullptr;
  hipError_t e = hipMallocAsync(&ws, xb + hb + zb, s);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return api_error(BDG_ENOMEM, "encode workspace");
  }
  uint16_t* Xb = static_cast<uint16_t*>(ws);
  uint16_t* H1b = reinterpret_cast<uint16_t*>(static_cast<char*>(ws) + xb);
  float* Z2 = reinterpret_cast<float*>(static_cast<char*>(ws) + xb + hb);
  for (uint32_t r0 = 0; r0 < n && e == hipSuccess; r0 += chunk) {
    const uint32_t rows = n - r0 < chunk ? n - r0 : chunk;
    const uint32_t rp = (rows + 31) & ~31u;
    hipLaunchKernelGGL(gather_rows_kernel, dim3(blocks_for((size_t)rp * p->d)), dim3(256), 0, s,
                       X, p->d, (const uint32_t*)nullptr, r0, rows, rp, scale, Xb,
                       (uint16_t*)nullptr);
    Epi e1 = epi(kEpiBiasTanh);
    e1.b0 = H1b;
    e1.bias = p->b1;
    e = gemm(Xb, p->d, p->W1b, p->d, rp, p->h, p->d, p->h, e1, s);
    if (e != hipSuccess) break;
    Epi e2 = epi(kEpiBias);
    e2.f0 = Z2;
    e2.bias = p->b2;
    e = gemm(H1b, p->h, p->W2b, p->h, rp, p->bits, p->h, p->bits, e2, s);
    if (e != hipSuccess) break;
    hipLaunchKernelGGL(pack_signs_kernel, dim3(blocks_for((size_t)rows * (p->bits / 64))),
                       dim3(256), 0, s, Z2, rows, p->bits, out_codes + (size_t)r0 * (p->bits / 64));
    e = hipGetLastError();
  }
  hipError_t e2 = hipFreeAsync(ws, s);
  if (e == hipSuccess) e = e2;
  return e == hipSuccess ? BDG_OK : api_device_error(e, "encode");
}

}  // extern "C"
