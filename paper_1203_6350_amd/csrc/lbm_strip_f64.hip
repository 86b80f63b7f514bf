// lbm_strip_f64.hip -- multi-step strip kernels for FP64 storage.
#include "lbm_strip.h"

namespace lbm {

hipError_t launch_multi_f64(const StepConfig &c, int k, const void *src, void *dst,
                          hipStream_t stream) {
  return launch_multi_storage<double>(c, k, src, dst, stream);
}

}  // namespace lbm
