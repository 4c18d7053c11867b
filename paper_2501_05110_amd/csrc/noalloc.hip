// Allocation-free form of vfp_apply_adjoint for callers that cannot allocate
// device memory (code under stream capture, serving loops, harnesses that
// forbid hipMalloc).  The call's one scratch vector, M^{-1} in, lives in a
// fixed device array of this file instead of a caller's buffer; everything
// else is vfp_apply_adjoint itself (same kernels, same results to the bit).
#include <hip/hip_runtime.h>

#include <mutex>

#include "internal.hpp"
#include "vfp.h"

namespace {

// One copy per device, held until the process ends.  Host code never passes
// this name to a kernel: it is a host-side stand-in, and the device address
// comes from hipGetSymbolAddress (per device) below.
static __device__ __align__(256) double scratch[VFP_NOALLOC_MAX_NDOFS];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
double* g_scratch[kMaxDevices] = {};

// Device address of `scratch` on device dev (which must be current).
int scratch_on(int dev, double** out) {
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return vfp::api_fail(VFP_EDEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", dev,
                           hipGetErrorString(e));
    g_scratch[dev] = static_cast<double*>(p);
  }
  *out = g_scratch[dev];
  return VFP_OK;
}

}  // namespace

extern "C" int vfp_apply_adjoint_noalloc(vfp_ctx* c, const double* in, double* out, void* stream) {
  int64_t n = 0;
  if (int e = vfp_ndofs(c, &n)) return e;
  if (n > (int64_t)VFP_NOALLOC_MAX_NDOFS)
    return vfp::api_fail(VFP_EINVAL, "ndofs %lld exceeds the allocation-free limit of %lld doubles",
                         (long long)n, (long long)VFP_NOALLOC_MAX_NDOFS);
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
    return vfp::api_fail(VFP_EDEVICE, "no current HIP device");
  const int cdev = vfp::ctx_device(c);
  if (cdev >= 0 && cdev != dev)
    return vfp::api_fail(VFP_EINVAL, "context lives on device %d but device %d is current", cdev, dev);
  double* work = nullptr;
  if (int e = scratch_on(dev, &work)) return e;
  return vfp_apply_adjoint(c, in, out, work, stream);
}
