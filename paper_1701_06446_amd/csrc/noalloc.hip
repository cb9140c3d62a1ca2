// Fixed device array behind cum_update_noalloc: the staging buffer that
// cum_update allocates on demand for host inputs, here in a file-scope device
// array of NOALLOC_STAGE_BYTES that every call on a device shares.
//
// In host code `scratch` names a host-side stand-in, not device memory; the
// device address comes from hipGetSymbolAddress, looked up once per device
// (with that device current) and kept in a per-device table.
#include <hip/hip_runtime.h>

#include <mutex>

#include "noalloc.h"

namespace cum {

static __device__ __align__(256) char scratch[NOALLOC_STAGE_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

}  // namespace

hipError_t noalloc_stage(void** ptr) {
  *ptr = nullptr;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_ptr[dev] = p;
  }
  *ptr = g_ptr[dev];
  return hipSuccess;
}

}  // namespace cum
