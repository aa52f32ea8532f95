// Control-variate network: constants of the flat parameter layout and the
// launchers of mlp.hip.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace mrip {

constexpr int MLP_DIN = 10, MLP_H = 128, MLP_DOUT = 4;
// flat fp32 parameters: W1[128x10] b1[128] W2[128x128] b2[128] W3[4x128] b3[4]
constexpr int MLP_OFF_W1 = 0;
constexpr int MLP_OFF_B1 = MLP_OFF_W1 + MLP_H * MLP_DIN;   // 1280
constexpr int MLP_OFF_W2 = MLP_OFF_B1 + MLP_H;             // 1408
constexpr int MLP_OFF_B2 = MLP_OFF_W2 + MLP_H * MLP_H;     // 17792
constexpr int MLP_OFF_W3 = MLP_OFF_B2 + MLP_H;             // 17920
constexpr int MLP_OFF_B3 = MLP_OFF_W3 + MLP_DOUT * MLP_H;  // 18432
constexpr int MLP_NPARAMS = MLP_OFF_B3 + MLP_DOUT;         // 18436
constexpr int MLP_PSTRIDE = 18440;  // partial-gradient row: params, loss, padding
// Bytes of the weights' image the gradient kernel stages (bf16 W2, W1
// padded to 32 features, fp32 b1, b2, bf16-rounded W3, b3, then bf16 W2^T,
// rows padded to 136), 16-byte aligned.
constexpr size_t MLP_IMAGE_BYTES = 82960;

struct AdamArgs {
  float lr, beta1, beta2, eps;
  float bc1, bc2;  // 1 - beta^step, bias corrections
};

// rows of partial gradients mlp_grad writes for n samples (one per 64)
size_t mlp_partial_rows(uint64_t n);

// theta (16-byte aligned) everywhere below
// y[4i..4i+3] = g(x_i), the network's four outputs
hipError_t launch_mlp_forward(const float *theta, const float *x, uint64_t n, float *y,
                              hipStream_t s);
// Coefficients per bin of rho of the control-variate estimator: the
// network's control h, then the four prefix controls.
constexpr int CV_NCOEF = 5;
// Per-sample inputs and outputs of the fused control-variate inference.
struct CvInferArgs {
  const float *mean, *inv_std;  // feature z-scores (10 each)
  const float *ctl;             // n x 8 raw controls (after the prefix, then over it)
  const uint64_t *customers;    // n run lengths
  const float *mu;              // n service rates
  const uint32_t *bin;          // n rows of the coefficient table
  const float *coef;            // table rows of CV_NCOEF
  const float *y;               // n responses
  float *g;                     // n x 4 network outputs (nullable), 16-byte aligned
  float *h, *d;                 // n network controls, n residuals
};
// g = net((x - mean) * inv_std), h = sum_{k<4} g_k z_k and
// d = y - coef[bin] . (h, z_4..z_7) with z the multipliers of the controls
hipError_t launch_cv_infer(const float *theta, const float *x, uint64_t n, const CvInferArgs &a,
                           hipStream_t s);
// img (MLP_IMAGE_BYTES, 16-byte aligned) = the image of theta
hipError_t launch_mlp_pack(const float *theta, void *img, hipStream_t s);
// Partial gradients of mean((sum_k g_k(x_i) z_ik - y_i)^2) at the weights
// whose image is img: one row per 64 samples. z: n x 4 per-sample
// multipliers, nullptr for z_i = e_0 (the first output alone).
hipError_t launch_mlp_grad(const void *img, const float *x, const float *z, const float *y,
                           uint64_t n, float *partial, hipStream_t s);
// Fixed-order sum of the partial rows into grad / loss (either nullable);
// with theta non-null, also one Adam step on theta, m, v, and with img
// non-null the image of the updated theta.
hipError_t launch_grad_reduce(const float *partial, uint32_t n_wg, uint64_t n, float *grad,
                              float *loss, float *theta, float *m, float *v, const AdamArgs &ad,
                              void *img, hipStream_t s);
hipError_t launch_adam(float *theta, float *m, float *v, const float *grad, uint64_t n,
                       const AdamArgs &ad, hipStream_t s);

}  // namespace mrip

namespace mrip {
// cvk.hip
hipError_t launch_col_stats(const float *m, uint64_t n, uint32_t cols, double *out,
                            hipStream_t s);
hipError_t launch_normalize(const float *src, uint64_t n, uint32_t cols, const float *mean,
                            const float *inv_std, float *dst, hipStream_t s);
hipError_t launch_gather_normalize(const float *src, const uint32_t *perm, uint64_t n,
                                   uint32_t cols, const float *mean, const float *inv_std,
                                   float *dst, hipStream_t s);
// z (n x 8) = the eight controls' multipliers; with group non-null also the
// standardised target t (n) and the network's multipliers zt (n x 4) from
// the groups' (n, mean, var) triples nmv.
hipError_t launch_multipliers(const float *ctl, const uint64_t *customers, const float *mu,
                              uint64_t n, float *z, const float *y, const uint32_t *group,
                              const double *nmv, float *t, float *zt, hipStream_t s);

}  // namespace mrip
