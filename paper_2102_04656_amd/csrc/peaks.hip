// Rate probes for the roofline denominators of the two Hamming tiles: the
// sustained rate of 32-bit integer vector instructions (the popcount path's
// unit: XOR, popcount-accumulate, add) and of the int8 matrix cores with the
// operand bytes the matrix tile uses ({0, 1} candidates against +-1 queries,
// random). Each probe is a fixed loop of independent instructions over the
// whole chip, timed with events; nothing here belongs to the paper's method.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bdg.h"

namespace bdg {
int api_error(int status, const char* fmt, ...);
int api_device_error(hipError_t e, const char* what);
void api_clear_error();

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));

constexpr int kValuAcc = 8;     // independent accumulators per lane
constexpr int kValuIters = 1 << 18;
constexpr int kMfmaIters = 1 << 20;

// Per iteration and accumulator: v_xor_b32, v_bcnt_u32_b32 (popcount plus
// accumulate), v_add_u32 -- three 32-bit vector instructions.
__global__ __launch_bounds__(256) void valu_probe_kernel(uint32_t seed, uint32_t* out) {
  uint32_t x[kValuAcc], acc[kValuAcc];
  const uint32_t y = (threadIdx.x + seed) * 2654435761u;
#pragma unroll
  for (int j = 0; j < kValuAcc; ++j) {
    x[j] = threadIdx.x + 977u * j + seed;
    acc[j] = 0;
  }
  for (int i = 0; i < kValuIters; ++i) {
#pragma unroll
    for (int j = 0; j < kValuAcc; ++j) {
      acc[j] = __builtin_popcount(x[j] ^ y) + acc[j];
      x[j] += acc[j];
    }
  }
  uint32_t s = 0;
#pragma unroll
  for (int j = 0; j < kValuAcc; ++j) s += acc[j] + x[j];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__device__ __forceinline__ uint32_t mix(uint32_t h) {
  h ^= h >> 16;
  h *= 0x7feb352du;
  h ^= h >> 15;
  h *= 0x846ca68bu;
  return h ^ (h >> 16);
}

// Eight independent v_mfma_i32_16x16x64_i8 products per iteration: A operands
// random {0, 1} bytes, B operands random +-1 bytes, both fixed in registers.
__global__ __launch_bounds__(512) void mfma_probe_kernel(uint32_t seed, int* out) {
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  v4i a[4], b[2];
#pragma unroll
  for (int k = 0; k < 4; ++k)
#pragma unroll
    for (int e = 0; e < 4; ++e) a[k][e] = (int)(mix(t * 16 + k * 4 + e + seed) & 0x01010101u);
#pragma unroll
  for (int k = 0; k < 2; ++k)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const uint32_t r = mix(~t * 16 + k * 4 + e + seed) & 0x01010101u;
      b[k][e] = (int)((r * 0xFEu) ^ 0xFFFFFFFFu);  // set bit -> 0x01, clear -> 0xFF
    }
  v4i c[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) c[j] = v4i{j, 0, 0, 0};
  for (int i = 0; i < kMfmaIters; ++i) {
#pragma unroll
    for (int j = 0; j < 8; ++j)
      c[j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[j & 3], b[j >> 2], c[j], 0, 0, 0);
  }
  int s = 0;
#pragma unroll
  for (int j = 0; j < 8; ++j) s += c[j][0] + c[j][1] + c[j][2] + c[j][3];
  out[t] = s;
}

}  // namespace
}  // namespace bdg

extern "C" {

int bdg_probe_peak(int unit, double* ops_per_second, void* stream) {
  using namespace bdg;
  api_clear_error();
  if (!ops_per_second) return api_error(BDG_EINVAL, "ops_per_second is NULL");
  if (unit != BDG_PEAK_VALU_INT32 && unit != BDG_PEAK_MFMA_INT8)
    return api_error(BDG_EINVAL, "unknown unit %d", unit);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  int dev = 0, cus = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return api_device_error(e, "device query");
  // VALU: 8 work-groups of 4 waves per CU (8 waves per SIMD); matrix cores:
  // one work-group of 8 waves per CU (2 waves per SIMD)
  const bool valu = unit == BDG_PEAK_VALU_INT32;
  const dim3 grid(valu ? cus * 8 : cus), block(valu ? 256 : 512);
  const size_t threads = (size_t)grid.x * block.x;
  void* out = nullptr;
  e = hipMallocAsync(&out, threads * 4, s);
  if (e != hipSuccess) return api_error(BDG_ENOMEM, "probe output");
  hipEvent_t e0 = nullptr, e1 = nullptr;
  e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  float ms = 0.f;
  for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {  // the first run warms up
    if (e == hipSuccess) e = hipEventRecord(e0, s);
    if (valu)
      hipLaunchKernelGGL(valu_probe_kernel, grid, block, 0, s, (uint32_t)rep,
                         static_cast<uint32_t*>(out));
    else
      hipLaunchKernelGGL(mfma_probe_kernel, grid, block, 0, s, (uint32_t)rep,
                         static_cast<int*>(out));
    if (e == hipSuccess) e = hipGetLastError();
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  hipError_t f = hipFreeAsync(out, s);
  if (e == hipSuccess) e = f;
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return api_device_error(e, "probe");
  const double ops = valu ? 3.0 * kValuAcc * kValuIters * (double)threads
                          : 2.0 * 16384.0 * 8 * kMfmaIters * (double)(threads / 64);
  *ops_per_second = ops / (ms * 1e-3);
  return BDG_OK;
}

}  // extern "C"
