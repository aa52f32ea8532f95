// Small kernels around the control-variate network: per-column fp64 mean
// and standard deviation, z-score normalisation, and D = Y - beta * G.
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

// t[i] = (y[i] - mean_g) / sd_g for the design point g = group[i], from the
// (n, mean, var) triples of the groups; 0 where sd_g = 0.
__global__ void center_kernel(const float *y, const uint32_t *group, const double *nmv,
                              uint64_t n, float *t) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t g = group[i];
  const double sd = sqrt(nmv[3 * g + 2]);
  t[i] = sd > 0.0 ? (float)(((double)y[i] - nmv[3 * g + 1]) / sd) : 0.0f;
}

__global__ void axpy_kernel(const float *y, const float *g, float beta, uint64_t n, float *d) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) d[i] = y[i] - beta * g[i];
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

hipError_t launch_center(const float *y, const uint32_t *group, const double *nmv, uint64_t n,
                         float *t, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(center_kernel, dim3((uint32_t)((n + 255) / 256)), dim3(256), 0, s, y, group,
                     nmv, n, t);
  return hipGetLastError();
}

hipError_t launch_axpy(const float *y, const float *g, float beta, uint64_t n, float *d,
                       hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(axpy_kernel, dim3((uint32_t)((n + 255) / 256)), dim3(256), 0, s, y, g, beta,
                     n, d);
  return hipGetLastError();
}

}  // namespace mrip
