// lbm_strip_f64.hip -- multi-step strip kernels for F64 storage. The
// build compiles this file once per step count K (LBM_STRIP_ONLY_K = 2, 3,
// 4), each object exporting the K-suffixed entry points that
// launch_multi_steps and the batch dispatch call.
#include "lbm_strip.h"

#ifndef LBM_STRIP_ONLY_K
#error "compile with -DLBM_STRIP_ONLY_K=2, 3 or 4"
#endif

#define LBM_CAT2(a, b) a##b
#define LBM_CAT(a, b) LBM_CAT2(a, b)

namespace lbm {

hipError_t LBM_CAT(launch_multi_f64_k, LBM_STRIP_ONLY_K)(const StepConfig &c, const void *src,
                                                          void *dst, hipStream_t stream) {
  return launch_multi_storage<double>(c, LBM_STRIP_ONLY_K, src, dst, stream);
}

hipError_t LBM_CAT(launch_batch_multi_f64_k, LBM_STRIP_ONLY_K)(int nw, int form,
                                                                const BatchDomain *doms,
                                                                const int4 *items,
                                                                int *nitems, int grid,
                                                                int j, hipStream_t stream) {
  return launch_batch_multi_storage<double>(LBM_STRIP_ONLY_K, nw, form, doms, items, nitems, grid,
                                           j, stream);
}

int LBM_CAT(batch_multi_per_cu_f64_k, LBM_STRIP_ONLY_K)(int nw, int form) {
  return batch_multi_per_cu<double>(LBM_STRIP_ONLY_K, nw, form);
}

}  // namespace lbm
