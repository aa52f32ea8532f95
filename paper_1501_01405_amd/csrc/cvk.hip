// Small kernels around the control-variate network: per-column fp64 mean
// and standard deviation, z-score normalisation, and the controls'
// per-sample multipliers with the training target.
#include <hip/hip_runtime.h>

#include "mlp.hpp"

namespace mrip {

namespace {

constexpr int CB = 256;

// Column j of a row-major n x cols fp32 matrix: out[2j] = mean,
// out[2j+1] = population std, fp64, two passes, fixed order.
__global__ void col_stats_kernel(const float *m, uint64_t n, uint32_t cols, double *out) {
  __shared__ double sh[CB];
  const uint32_t j = blockIdx.x;
  double s = 0.0;
  for (uint64_t i = threadIdx.x; i < n; i += CB) s += (double)m[i * cols + j];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = CB / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  const double mean = sh[0] / (double)n;
  __syncthreads();
  double ss = 0.0;
  for (uint64_t i = threadIdx.x; i < n; i += CB) {
    const double d = (double)m[i * cols + j] - mean;
    ss += d * d;
  }
  sh[threadIdx.x] = ss;
  __syncthreads();
  for (int w = CB / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[2 * j] = mean;
    out[2 * j + 1] = sqrt(sh[0] / (double)n);
  }
}

// dst[i][j] = (src[i][j] - mean[j]) * inv_std[j]
__global__ void normalize_kernel(const float *src, uint64_t n, uint32_t cols, const float *mean,
                                 const float *inv_std, float *dst) {
  const uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * cols) return;
  const uint32_t j = (uint32_t)(e % cols);
  dst[e] = (src[e] - mean[j]) * inv_std[j];
}

// dst[j][c] = (src[perm[j]][c] - mean[c]) * inv_std[c]  (row gather + z-score)
__global__ void gather_normalize_kernel(const float *src, const uint32_t *perm, uint64_t n,
                                        uint32_t cols, const float *mean, const float *inv_std,
                                        float *dst) {
  const uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * cols) return;
  const uint64_t j = e / cols;
  const uint32_t c = (uint32_t)(e % cols);
  dst[e] = (src[(uint64_t)perm[j] * cols + c] - mean[c]) * inv_std[c];
}

// Per replication i of N_i customers at service rate mu_i: the multipliers
// z = (c0, c1, c2 / m, c3 / m, c4, c5, c6 / m, c7 / m) / N_i of its eight
// controls c (after the prefix, then over it), with m = (float)(1 / mu_i)
// the service scale (every z_k is a time per customer). With `group` set
// (training): also t = (y - mean_g) / sd_g and zt = z_{0..3} / sd_g for the
// replication's design point g (both 0 where sd_g = 0), the standardised
// target and the multipliers of the network's four coefficients.
__global__ void multipliers_kernel(const float *ctl, const uint64_t *customers, const float *mu,
                                   uint64_t n, float *z, const float *y, const uint32_t *group,
                                   const double *nmv, float *t, float *zt) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double N = (double)customers[i];
  const double m = (double)(float)(1.0 / (double)mu[i]);
  const double sc[4] = {1.0 / N, 1.0 / N, (1.0 / m) / N, (1.0 / m) / N};
  double zk[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    zk[k] = (double)ctl[8 * i + k] * sc[k & 3];
    z[8 * i + k] = (float)zk[k];
  }
  if (!group) return;
  const uint32_t g = group[i];
  const double sd = sqrt(nmv[3 * g + 2]);
  t[i] = sd > 0.0 ? (float)(((double)y[i] - nmv[3 * g + 1]) / sd) : 0.0f;
#pragma unroll
  for (int k = 0; k < 4; ++k) zt[4 * i + k] = sd > 0.0 ? (float)(zk[k] / sd) : 0.0f;
}

}  // namespace

hipError_t launch_col_stats(const float *m, uint64_t n, uint32_t cols, double *out,
                            hipStream_t s) {
  hipLaunchKernelGGL(col_stats_kernel, dim3(cols), dim3(CB), 0, s, m, n, cols, out);
  return hipGetLastError();
}

hipError_t launch_normalize(const float *src, uint64_t n, uint32_t cols, const float *mean,
                            const float *inv_std, float *dst, hipStream_t s) {
  const uint64_t total = n * cols;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(normalize_kernel, dim3((uint32_t)((total + 255) / 256)), dim3(256), 0, s,
                     src, n, cols, mean, inv_std, dst);
  return hipGetLastError();
}

hipError_t launch_gather_normalize(const float *src, const uint32_t *perm, uint64_t n,
                                   uint32_t cols, const float *mean, const float *inv_std,
                                   float *dst, hipStream_t s) {
  const uint64_t total = n * cols;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(gather_normalize_kernel, dim3((uint32_t)((total + 255) / 256)), dim3(256), 0,
                     s, src, perm, n, cols, mean, inv_std, dst);
  return hipGetLastError();
}

hipError_t launch_multipliers(const float *ctl, const uint64_t *customers, const float *mu,
                              uint64_t n, float *z, const float *y, const uint32_t *group,
                              const double *nmv, float *t, float *zt, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(multipliers_kernel, dim3((uint32_t)((n + 255) / 256)), dim3(256), 0, s, ctl,
                     customers, mu, n, z, y, group, nmv, t, zt);
  return hipGetLastError();
}

}  // namespace mrip
