// Launch dispatch over the I/O storage types (host code).
#include <hip/hip_runtime.h>

#include <mutex>

#include "fc_internal.h"

namespace fcx {

hipError_t launch_kernel_io0(int, int, const LaunchArgs&, int, size_t, hipStream_t);
hipError_t launch_kernel_io1(int, int, const LaunchArgs&, int, size_t, hipStream_t);
hipError_t launch_kernel_io2(int, int, const LaunchArgs&, int, size_t, hipStream_t);
hipError_t launch_zero_io0(void*, int64_t, hipStream_t);
hipError_t launch_zero_io1(void*, int64_t, hipStream_t);
hipError_t launch_zero_io2(void*, int64_t, hipStream_t);
hipError_t lds_limits_io0(size_t);
hipError_t lds_limits_io1(size_t);
hipError_t lds_limits_io2(size_t);

hipError_t launch_kernel(int cls, int size, const LaunchArgs& a, int aux, size_t lds, hipStream_t s) {
  switch (a.io) {
    case IO_C64: return launch_kernel_io0(cls, size, a, aux, lds, s);
    case IO_F16: return launch_kernel_io1(cls, size, a, aux, lds, s);
    case IO_BF16: return launch_kernel_io2(cls, size, a, aux, lds, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_zero(void* out, int64_t n, int io, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  switch (io) {
    case IO_C64: return launch_zero_io0(out, n, s);
    case IO_F16: return launch_zero_io1(out, n, s);
    case IO_BF16: return launch_zero_io2(out, n, s);
    default: return hipErrorInvalidValue;
  }
}

// The dynamic-LDS limit is a property of each kernel function, shared by
// every plan in the process: it is only ever raised (per device, under a
// lock), so a plan that needs less never lowers the limit for the launches
// of a plan that needs more.
hipError_t set_lds_limits(size_t bytes) {
  static std::mutex mu;
  static size_t granted[64] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (bytes <= granted[dev]) return hipSuccess;
  hipError_t a = lds_limits_io0(bytes), b = lds_limits_io1(bytes), c = lds_limits_io2(bytes);
  e = a != hipSuccess ? a : (b != hipSuccess ? b : c);
  if (e == hipSuccess) granted[dev] = bytes;
  return e;
}

}  // namespace fcx
