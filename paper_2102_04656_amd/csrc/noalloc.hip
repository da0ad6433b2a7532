// The build of bdg_build_knn_ex without any allocation: for callers that
// cannot allocate device memory (code under HIP graph capture, tight serving
// loops, harnesses that forbid allocation). Its workspace (operand fragments
// and the persistent launch's control words) is a file-scope device array of
// fixed size; each device the library runs on holds its own copy until the
// process ends. Every call on a device shares that device's copy, which keeps
// the last call's contents: the launch clears the control words itself (a
// fill kernel), and calls that overlap on one device race.
#include <hip/hip_runtime.h>
#include <string.h>

#include <mutex>

#include "bdg.h"
#include "kernels.h"

namespace bdg {
int api_error(int status, const char* fmt, ...);
int api_device_error(hipError_t e, const char* what);
void api_clear_error();
}  // namespace bdg

namespace {

constexpr size_t kScratchBytes = (size_t)BDG_NOALLOC_SCRATCH_MB << 20;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_ptr[kMaxDevices];  // device address of `scratch` on each device (set once)

// The device address of this device's copy of `scratch`. In host code the
// array's name is only a stand-in for the symbol, never a device address.
int scratch_ptr(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return bdg::api_device_error(e, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices)
    return bdg::api_error(BDG_EUNSUPPORTED, "device %d beyond the %d the library tracks", dev,
                          kMaxDevices);
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      return bdg::api_device_error(e != hipSuccess ? e : hipErrorInvalidSymbol,
                                   "hipGetSymbolAddress(scratch)");
    }
    g_ptr[dev] = p;
  }
  *out = g_ptr[dev];
  return BDG_OK;
}

}  // namespace

extern "C" {

int bdg_build_knn_noalloc(const uint64_t* codes, uint32_t n, uint32_t bits, uint32_t K,
                          uint32_t* out_idx, uint16_t* out_dist, void* stream) {
  bdg::api_clear_error();
  bdg_knn_opts o;
  memset(&o, 0, sizeof o);
  o.struct_size = sizeof o;
  o.path = BDG_PATH_MFMA;
  size_t need = 0;
  int st = bdg_build_knn_workspace_size(n, bits, K, &o, &need);
  if (st != BDG_OK) return st;
  if (need > kScratchBytes)
    return bdg::api_error(BDG_EUNSUPPORTED,
                          "n=%u bits=%u needs %zu bytes of scratch, more than the %zu of the "
                          "static workspace",
                          n, bits, need, kScratchBytes);
  if (n == 0) return BDG_OK;
  if (!codes || !out_idx || !out_dist) return bdg::api_error(BDG_EINVAL, "null device pointer");
  void* ws = nullptr;
  st = scratch_ptr(&ws);
  if (st != BDG_OK) return st;
  o.workspace = ws;
  o.workspace_bytes = kScratchBytes;
  return bdg_build_knn_ex(codes, n, bits, K, out_idx, out_dist, &o, stream);
}

}  // extern "C"
