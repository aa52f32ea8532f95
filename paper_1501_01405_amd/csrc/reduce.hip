// MRIP statistics on the device (paper section 1: a confidence interval from
// independent replications): per segment of per-replication outputs, the
// count, the mean and the unbiased variance, in fp64, two passes. The
// summation order is fixed (thread-strided partial sums, then a fixed tree),
// so results are reproducible run to run. int32 outputs are summed exactly
// in int64 for the mean.
#include "device.hpp"
#include "kernels.hpp"
#include "reduce_dev.hpp"
#include "taus.hpp"

namespace mrip {

namespace {

constexpr int RB = 256;  // threads per segment

__device__ __forceinline__ double load_x(const void *x, int dtype, uint64_t i) {
  return dtype == 0 ? (double)((const int32_t *)x)[i] : (double)((const float *)x)[i];
}

__device__ double block_sum(double v, double *sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int w = RB / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

__device__ long long block_sum_ll(long long v, long long *sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int w = RB / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  const long long r = sh[0];
  __syncthreads();
  return r;
}

// Segment blockIdx.x of x (blockIdx.y = 0) or of x1, a second fp32 array
// reduced alongside in the same launch (blockIdx.y = 1, into out1).
__global__ void reduce_kernel(const void *x, int dtype, const uint32_t *index,
                              const uint64_t *offsets, uint64_t n, double *out, const float *x1,
                              double *out1) {
  __shared__ double shd[RB];
  __shared__ long long shl[RB];
  const uint32_t g = blockIdx.x;
  if (blockIdx.y == 1) {
    x = x1;
    dtype = 1;
    out = out1;
  }
  const uint64_t begin = offsets ? offsets[g] : 0;
  const uint64_t end = offsets ? offsets[g + 1] : n;
  const uint64_t cnt = end - begin;
  double mean;
  if (dtype == 0) {
    long long s = 0;
    for (uint64_t j = begin + threadIdx.x; j < end; j += RB)
      s += ((const int32_t *)x)[index ? index[j] : j];
    mean = (double)block_sum_ll(s, shl) / (double)cnt;
  } else {
    double s = 0.0;
    for (uint64_t j = begin + threadIdx.x; j < end; j += RB)
      s += load_x(x, dtype, index ? index[j] : j);
    mean = block_sum(s, shd) / (double)cnt;
  }
  double ss = 0.0;
  for (uint64_t j = begin + threadIdx.x; j < end; j += RB) {
    const double d = load_x(x, dtype, index ? index[j] : j) - mean;
    ss += d * d;
  }
  ss = block_sum(ss, shd);
  if (threadIdx.x == 0) {
    out[3 * g + 0] = (double)cnt;
    out[3 * g + 1] = cnt > 0 ? mean : 0.0;
    out[3 * g + 2] = cnt > 1 ? ss / (double)(cnt - 1) : 0.0;
  }
}

// One workgroup per output: the same fixed-order two-pass reduction.
__global__ void reduce_multi_kernel(ReduceSet set, uint64_t n, double *out) {
  __shared__ RedShared sh;
  const uint32_t o = blockIdx.x;
  reduce_output(set.x[o], set.dtype[o], n, out + 3 * o, sh);
}

__global__ void philox_dump_kernel(uint64_t seed, const uint32_t *ctr, uint64_t n,
                                   uint32_t *out) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const Block4 b = philox(ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3],
                          (uint32_t)seed, (uint32_t)(seed >> 32));
  out[4 * i + 0] = b.x;
  out[4 * i + 1] = b.y;
  out[4 * i + 2] = b.z;
  out[4 * i + 3] = b.w;
}

__global__ void taus_dump_kernel(uint64_t seed, uint32_t model, uint32_t dp, uint32_t rep,
                                 uint64_t skip, uint64_t n, const uint32_t *tables, uint32_t *out) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  Taus t = taus_seed(model, dp, rep, (uint32_t)seed, (uint32_t)(seed >> 32));
  taus_skip(t, skip + i, tables);
  out[i] = taus_next(t);
}

}  // namespace

hipError_t launch_reduce_f64(const void *x, int dtype, uint64_t n, const uint64_t *offsets,
                             uint32_t n_segments, double *out, hipStream_t s) {
  hipLaunchKernelGGL(reduce_kernel, dim3(n_segments), dim3(RB), 0, s, x, dtype, nullptr, offsets,
                     n, out, (const float *)nullptr, (double *)nullptr);
  return hipGetLastError();
}

hipError_t launch_reduce_f64_gather(const void *x, int dtype, const uint32_t *index,
                                    const uint64_t *offsets, uint32_t n_segments, double *out,
                                    hipStream_t s) {
  hipLaunchKernelGGL(reduce_kernel, dim3(n_segments), dim3(RB), 0, s, x, dtype, index, offsets,
                     (uint64_t)0, out, (const float *)nullptr, (double *)nullptr);
  return hipGetLastError();
}

hipError_t launch_reduce_f64_gather2(const float *x0, const float *x1, const uint32_t *index,
                                     const uint64_t *offsets, uint32_t n_segments, double *out0,
                                     double *out1, hipStream_t s) {
  hipLaunchKernelGGL(reduce_kernel, dim3(n_segments, 2), dim3(RB), 0, s, (const void *)x0, 1,
                     index, offsets, (uint64_t)0, out0, x1, out1);
  return hipGetLastError();
}

hipError_t launch_reduce_f64_multi(const ReduceSet &set, uint32_t n_outputs, uint64_t n,
                                   double *out, hipStream_t s) {
  hipLaunchKernelGGL(reduce_multi_kernel, dim3(n_outputs), dim3(RB), 0, s, set, n, out);
  return hipGetLastError();
}

hipError_t launch_taus_dump(uint64_t seed, uint32_t model, uint32_t dp, uint32_t rep, uint64_t skip,
                            uint64_t n, const uint32_t *tables, uint32_t *out, hipStream_t s) {
  const uint64_t blocks = (n + 255) / 256;
  hipLaunchKernelGGL(taus_dump_kernel, dim3((uint32_t)blocks), dim3(256), 0, s, seed, model, dp,
                     rep, skip, n, tables, out);
  return hipGetLastError();
}

hipError_t launch_philox_dump(uint64_t seed, const uint32_t *ctr, uint64_t n, uint32_t *out,
                              hipStream_t s) {
  if (n == 0) return hipSuccess;
  const uint64_t blocks = (n + 255) / 256;
  hipLaunchKernelGGL(philox_dump_kernel, dim3((uint32_t)blocks), dim3(256), 0, s, seed, ctr, n,
                     out);
  return hipGetLastError();
}

}  // namespace mrip
