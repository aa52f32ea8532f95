// The library context behind the opaque mrip_ctx handle: parameters, launch
// shape and every device buffer the context owns.
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/mrip.h"

namespace mrip {

// A device allocation owned by the context; grows on demand, freed with it.
struct DevBuf {
  void *p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf &) = delete;
  DevBuf &operator=(const DevBuf &) = delete;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
  hipError_t ensure(size_t n) {
    if (n <= bytes && p) return hipSuccess;
    if (p) {
      (void)hipFree(p);
      p = nullptr;
      bytes = 0;
    }
    hipError_t e = hipMalloc(&p, n ? n : 1);
    if (e == hipSuccess) bytes = n;
    return e;
  }
  template <class T>
  T *as() const {
    return (T *)p;
  }
};

enum RunKind { RUN_NONE = 0, RUN_UNIFORM = 1, RUN_PLAN = 2 };

// State of the learned control variate.
struct CvState {
  bool trained = false, applied = false;
  DevBuf theta;             // fp32 master weights (MRIP_MLP_PARAMS)
  DevBuf adam_m, adam_v;    // Adam moments
  DevBuf grad, loss;        // gradient and loss of the last step
  DevBuf partial;           // per-workgroup gradient partials
  DevBuf xn, y;             // normalised training features and targets
  DevBuf norm;              // feature mean[10], std[10]
  DevBuf work;              // apply: features, predictions, per-dp sums
  std::vector<float> mean, std_;
  float final_loss = 0.f;
  float beta = 1.0f;
  // apply results, per design point (host)
  std::vector<uint32_t> dp_ids;
  std::vector<double> cv_nmv, plain_nmv;  // n, mean, var-of-mean, dof
  float full_ms = 0.f, prefix_ms = 0.f, infer_ms = 0.f;
};

}  // namespace mrip

struct mrip_ctx_s {
  mrip_model model;
  mrip_mapping mapping;
  mrip_rw_params rw;
  mrip_mm1_params mm1;
  mrip_ff_params ff;
  uint32_t rpw = 1, wg = 256;

  mrip::DevBuf out[4];
  mrip::DevBuf scratch;
  mrip::DevBuf stats;  // 3 doubles per scalar output
  mrip::RunKind last = mrip::RUN_NONE;
  uint64_t last_n = 0;
  hipStream_t last_stream = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;  // around the last simulation kernel
  // event pairs of the last RING simulation-kernel launches (run history)
  static constexpr uint32_t RING = 256;
  hipEvent_t ring0[RING] = {}, ring1[RING] = {};
  uint64_t launches = 0;
  std::string err;

  // plan
  uint64_t n_items = 0;
  mrip::DevBuf it_dp, it_rep, it_n, it_lambda, it_mu, it_order, queue, dp_index, dp_offsets,
      dp_stats;
  std::vector<uint32_t> dp_ids;

  // learned control variate
  mrip::CvState cv;

  ~mrip_ctx_s() {
    if (ev0) (void)hipEventDestroy(ev0);
    if (ev1) (void)hipEventDestroy(ev1);
    for (uint32_t i = 0; i < RING; ++i) {
      if (ring0[i]) (void)hipEventDestroy(ring0[i]);
      if (ring1[i]) (void)hipEventDestroy(ring1[i]);
    }
  }
};
