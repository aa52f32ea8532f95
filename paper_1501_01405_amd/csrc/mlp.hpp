// Control-variate network: constants of the flat parameter layout and the
// launchers of mlp.hip.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mrip {

constexpr int MLP_DIN = 10, MLP_H = 128;
// flat fp32 parameters: W1[128x10] b1[128] W2[128x128] b2[128] W3[1x128] b3[1]
constexpr int MLP_OFF_W1 = 0;
constexpr int MLP_OFF_B1 = MLP_OFF_W1 + MLP_H * MLP_DIN;  // 1280
constexpr int MLP_OFF_W2 = MLP_OFF_B1 + MLP_H;            // 1408
constexpr int MLP_OFF_B2 = MLP_OFF_W2 + MLP_H * MLP_H;    // 17792
constexpr int MLP_OFF_W3 = MLP_OFF_B2 + MLP_H;            // 17920
constexpr int MLP_OFF_B3 = MLP_OFF_W3 + MLP_H;            // 18048
constexpr int MLP_NPARAMS = MLP_OFF_B3 + 1;               // 18049
constexpr int MLP_PSTRIDE = 18056;  // partial-gradient row: params, loss, padding

struct AdamArgs {
  float lr, beta1, beta2, eps;
  float bc1, bc2;  // 1 - beta^step, bias corrections
};

// rows of partial gradients mlp_grad writes for n samples (one per 64)
size_t mlp_partial_rows(uint64_t n);

// y[i] = out_shift + out_scale * g(x_i)
hipError_t launch_mlp_forward(const float *theta, const float *x, uint64_t n, float *y,
                              float out_scale, float out_shift, hipStream_t s);
hipError_t launch_mlp_grad(const float *theta, const float *x, const float *y, uint64_t n,
                           float *partial, hipStream_t s);
// Fixed-order sum of the partial rows into grad / loss (either nullable);
// with theta non-null, also one Adam step on theta, m, v.
hipError_t launch_grad_reduce(const float *partial, uint32_t n_wg, uint64_t n, float *grad,
                              float *loss, float *theta, float *m, float *v, const AdamArgs &ad,
                              hipStream_t s);
hipError_t launch_adam(float *theta, float *m, float *v, const float *grad, uint64_t n,
                       const AdamArgs &ad, hipStream_t s);

}  // namespace mrip

namespace mrip {
// cvk.hip
hipError_t launch_col_stats(const float *m, uint64_t n, uint32_t cols, double *out,
                            hipStream_t s);
hipError_t launch_normalize(const float *src, uint64_t n, uint32_t cols, const float *mean,
                            const float *inv_std, float *dst, hipStream_t s);
hipError_t launch_axpy(const float *y, const float *g, float beta, uint64_t n, float *d,
                       hipStream_t s);
hipError_t launch_gather_normalize(const float *src, const uint32_t *perm, uint64_t n,
                                   uint32_t cols, const float *mean, const float *inv_std,
                                   float *dst, hipStream_t s);
hipError_t launch_center(const float *y, const uint32_t *group, const double *nmv, uint64_t n,
                         float *t, hipStream_t s);
}  // namespace mrip
