// Allocation-free variant of the Tucker operator (cgl_tucker_noalloc) for
// callers that cannot allocate device memory: its intermediates live in a
// fixed file-scope device array instead of plan-owned buffers.
//
// The array is a device symbol: its host-side name is not a device address.
// Its address on each device is looked up once (hipGetSymbolAddress, with
// that device current) and kept; only that address is handed to kernels.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>

#include "../../include/cgl.h"
#include "plan_internal.hpp"

namespace {

// two intermediates of at most kScratchBytes / 2 each
constexpr size_t kScratchBytes = size_t(32) << 20;
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

void* g_scratch[kMaxDevices] = {};
std::mutex g_mu;

// device address of this device's copy of the scratch array
int scratch_address(void** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return CGL_EDEVICE;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_scratch[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return CGL_EDEVICE;
    g_scratch[dev] = ptr;
  }
  *out = g_scratch[dev];
  return CGL_OK;
}

}  // namespace

extern "C" int cgl_tucker_noalloc(cgl_plan_t p, int which, const void* in_dev, void* out_dev) {
  cgl::PlanInfo pi;
  const int st = cgl::plan_info(p, &pi);
  if (st != CGL_OK) return st;
  if (pi.batch > 0 || !in_dev || !out_dev) return CGL_EINVAL;
  int64_t N = 1;
  for (int mu = 0; mu < pi.d; ++mu) N *= pi.n[mu];
  const size_t bytes = static_cast<size_t>(N) * (pi.precision == CGL_FP64 ? 16 : 8);
  if (bytes > kScratchBytes / 2) return CGL_ESCRATCH;
  void* base = nullptr;
  const int sa = scratch_address(&base);
  if (sa != CGL_OK) return sa;
  char* s = static_cast<char*>(base);
  return cgl::tucker_with_scratch(p, which, in_dev, out_dev, s, s + kScratchBytes / 2);
}
