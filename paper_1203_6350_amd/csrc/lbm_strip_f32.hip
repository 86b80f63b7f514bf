// lbm_strip_f32.hip -- multi-step strip kernels for FP32 storage.
#include "lbm_strip.h"

namespace lbm {

hipError_t launch_multi_f32(const StepConfig &c, int k, const void *src, void *dst,
                          hipStream_t stream) {
  return launch_multi_storage<float>(c, k, src, dst, stream);
}

}  // namespace lbm
