// One translation unit per I/O storage type (FC_IO = 0 c64, 1 f16, 2 bf16):
// instantiates the kernels of fc_device.h for that type and exports its
// launch entry points. Built three times in parallel.
#include "fc_device.h"

#ifndef FC_IO
#error "FC_IO must be defined"
#endif

#define FC_CAT2(a, b) a##b
#define FC_CAT(a, b) FC_CAT2(a, b)

namespace fcx {

hipError_t FC_CAT(launch_kernel_io, FC_IO)(int cls, int size, const LaunchArgs& a, int aux, size_t lds,
                                           hipStream_t s) {
  return launch_io<FC_IO>(cls, size, a, aux, lds, s);
}

hipError_t FC_CAT(launch_zero_io, FC_IO)(void* out, int64_t n, hipStream_t s) {
  return launch_zero_io<FC_IO>(out, n, s);
}

hipError_t FC_CAT(lds_limits_io, FC_IO)(size_t bytes) { return lds_limits_io<FC_IO>(bytes); }

}  // namespace fcx
