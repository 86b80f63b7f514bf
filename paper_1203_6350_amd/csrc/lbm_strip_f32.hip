// lbm_strip_f32.hip -- multi-step strip kernels for FP32 storage.
#include "lbm_strip.h"

namespace lbm {

hipError_t launch_multi_f32(const StepConfig &c, int k, const void *src, void *dst,
                          hipStream_t stream) {
  return launch_multi_storage<float>(c, k, src, dst, stream);
}

hipError_t launch_batch_multi_f32(int k, int nw, bool def, const BatchDomain *doms,
                                const int4 *items, const int *nitems, int grid, int j,
                                hipStream_t stream) {
  return launch_batch_multi_storage<float>(k, nw, def, doms, items, nitems, grid, j, stream);
}

int batch_multi_per_cu_f32(int k, int nw, bool def) { return batch_multi_per_cu<float>(k, nw, def); }

}  // namespace lbm
