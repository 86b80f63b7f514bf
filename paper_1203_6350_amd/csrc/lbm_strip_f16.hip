// lbm_strip_f16.hip -- multi-step strip kernels for FP16 storage.
#include "lbm_strip.h"

namespace lbm {

hipError_t launch_multi_f16(const StepConfig &c, int k, const void *src, void *dst,
                          hipStream_t stream) {
  return launch_multi_storage<__half>(c, k, src, dst, stream);
}

}  // namespace lbm
