// Learned control variate (not in the paper): placeholder entry points until
// the network kernels land.
#include <hip/hip_runtime.h>

#include "../../include/mrip.h"
#include "context.hpp"

extern "C" {

mrip_status mrip_mlp_forward(const float *, const float *, uint64_t, float *, void *) {
  return MRIP_E_UNSUPPORTED;
}
mrip_status mrip_mlp_grad(const float *, const float *, const float *, uint64_t, float *, float *,
                          void *) {
  return MRIP_E_UNSUPPORTED;
}
mrip_status mrip_adam_step(float *, float *, float *, const float *, uint64_t, uint64_t, float,
                           float, float, float, void *) {
  return MRIP_E_UNSUPPORTED;
}
mrip_status mrip_cv_train(mrip_ctx, const mrip_plan_item *, uint64_t, const float *,
                          const mrip_cv_hparams *, uint64_t, void *) {
  return MRIP_E_UNSUPPORTED;
}
mrip_status mrip_cv_model(mrip_ctx, float *, float *, float *, float *) { return MRIP_E_UNSUPPORTED; }
mrip_status mrip_cv_apply(mrip_ctx, const mrip_plan_item *, uint64_t, const mrip_plan_item *,
                          uint64_t, uint64_t, void *) {
  return MRIP_E_UNSUPPORTED;
}
mrip_status mrip_cv_stats(mrip_ctx, uint32_t, double, mrip_stats_t *, mrip_stats_t *) {
  return MRIP_E_UNSUPPORTED;
}
mrip_status mrip_cv_times(mrip_ctx, float *, float *, float *) { return MRIP_E_UNSUPPORTED; }
}
