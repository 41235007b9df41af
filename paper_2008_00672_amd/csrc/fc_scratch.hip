// Fixed device scratch of the no-allocation weight gradient
// (fc_tx_weight_grad_noalloc): a file-scope device array of
// FC_NOALLOC_SCRATCH_BYTES, one copy per GPU the library runs on, held until
// the process ends.
//
// In host code the array's name is only a stand-in for the device symbol, not
// a device address. Its address on a device is looked up once, with that
// device current, by hipGetSymbolAddress; that pointer (different on every
// device) is what the kernels receive, exactly as they receive the
// plan-owned scratch of fc_tx_weight_grad.
#include <hip/hip_runtime.h>

#include <mutex>

#include "fc.h"

namespace fcx {

static __device__ __align__(256) float scratch[FC_NOALLOC_SCRATCH_BYTES / sizeof(float)];

constexpr int kMaxDevices = 64;

// Device address of this device's scratch array (the current device must be
// `device`). The first call per device looks it up; later calls return it.
hipError_t noalloc_scratch(int device, float** ptr) {
  static std::mutex mu;
  static float* addr[kMaxDevices] = {};
  if (device < 0 || device >= kMaxDevices || !ptr) return hipErrorInvalidValue;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    addr[device] = static_cast<float*>(p);
  }
  *ptr = addr[device];
  return hipSuccess;
}

}  // namespace fcx
