// The fixed-order fp64 two-pass reduction of one output (count, mean,
// unbiased variance) by one 256-thread workgroup, shared by the reduction
// kernels and the simulation kernel that reduces the previous run's
// outputs in an extra workgroup: both give the same bits.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mrip {

constexpr int RED_THREADS = 256;

struct RedShared {
  double d[RED_THREADS];
  long long l[RED_THREADS];
};

__device__ __forceinline__ double red_load(const void *x, int dtype, uint64_t i) {
  return dtype == 0 ? (double)((const int32_t *)x)[i] : (double)((const float *)x)[i];
}

template <class T>
__device__ __forceinline__ T red_block_sum(T v, T *sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int w = RED_THREADS / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  const T r = sh[0];
  __syncthreads();
  return r;
}

// out[0..2] = (n, mean, variance) of x[0..n) (dtype 0: int32, summed
// exactly in int64 for the mean; 1: fp32). Every thread of a 256-thread
// workgroup calls it; thread 0 writes.
__device__ __forceinline__ void reduce_output(const void *x, int dtype, uint64_t n, double *out,
                                              RedShared &sh) {
  double mean;
  if (dtype == 0) {
    long long s = 0;
    for (uint64_t j = threadIdx.x; j < n; j += RED_THREADS) s += ((const int32_t *)x)[j];
    mean = (double)red_block_sum(s, sh.l) / (double)n;
  } else {
    double s = 0.0;
    for (uint64_t j = threadIdx.x; j < n; j += RED_THREADS) s += red_load(x, dtype, j);
    mean = red_block_sum(s, sh.d) / (double)n;
  }
  double ss = 0.0;
  for (uint64_t j = threadIdx.x; j < n; j += RED_THREADS) {
    const double d = red_load(x, dtype, j) - mean;
    ss += d * d;
  }
  ss = red_block_sum(ss, sh.d);
  if (threadIdx.x == 0) {
    out[0] = (double)n;
    out[1] = n > 0 ? mean : 0.0;
    out[2] = n > 1 ? ss / (double)(n - 1) : 0.0;
  }
}

}  // namespace mrip
