// cola_density_noalloc: the mean-1 CIC density of cola_density with its particle
// binning buffers in a file-scope device array instead of a caller workspace, for
// callers that cannot allocate device memory.
//
// The array `scratch` exists once per GPU (module globals are per device).  Host code
// never passes its name to a kernel: the name is a host-side stand-in, not a device
// address.  On the first call on a device, with that device current, its address is
// taken with hipGetSymbolAddress and kept per device; every later call on that device
// passes that pointer to the deposit's kernels, as the workspace entry point passes
// its buffer.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/cola.h"
#include "internal.hpp"

namespace {

constexpr size_t kScratchBytes = size_t(256) << 20;   // 256 MiB per GPU
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this GPU's array (taken once per device, current device).
int scratch_address(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return cola::record_hip(e);
  if (dev < 0 || dev >= kMaxDevices) return COLA_ERR_DEVICE;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) return cola::record_hip(e != hipSuccess ? e : hipErrorInvalidSymbol);
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return COLA_OK;
}

}  // namespace

extern "C" int cola_density_noalloc(cola_plan plan, const float* s, float* rho, void* stream) {
  if (!plan || !s || !rho) return COLA_ERR_INVALID;
  if (cola::plan_bin_bytes(plan) > kScratchBytes) return COLA_ERR_WORKSPACE;
  void* base = nullptr;
  const int rc = scratch_address(&base);
  if (rc != COLA_OK) return rc;
  return cola::density_with_bins(plan, s, rho, base, static_cast<hipStream_t>(stream));
}
