// Monte Carlo pi replication engines (paper section 5.1, first model).
//
// Point i of replication r is the pair of words 2(i&1), 2(i&1)+1 of Philox
// block (i>>1, 0, r, TAG_PI); a word's top 24 bits X give u = (X + 1/2)
// 2^-24 and the point is inside the quarter disc iff
// (2X+1)^2 + (2Y+1)^2 <= 2^50, an exact test on two v_mad_u64_u32.
//
// WAVE: one replication per wavefront, the lanes take interleaved blocks
// (four per lane per iteration) and sum their counts at the end. SIMT: one
// replication per lane (STRIDE 1) or per wavefront's first lane (STRIDE 64,
// the paper's WLP form).
//
// On taus88 streams point i takes outputs 2i and 2i+1 of the replication's
// stream; in the WAVE form lane l takes the contiguous run of points
// [l B, (l+1) B), B = ceil(points / 64), after jumping 2 l B outputs.
//
// With few replications a wavefront each leaves the chip idle, so
// pi_wide_kernel<X> gives a replication X wavefronts (a workgroup); the hit
// count is an integer sum, identical however the points are shared out.
#include "device.hpp"
#include "kernels.hpp"
#include "taus.hpp"

namespace mrip {

namespace {

__device__ __forceinline__ uint32_t inside(uint32_t wx, uint32_t wy) {
  const uint64_t a = 2u * (wx >> 8) + 1u, b = 2u * (wy >> 8) + 1u;
  return a * a + b * b <= (1ull << 50) ? 1u : 0u;
}

// hits of the two points of block k (the second only if it exists)
__device__ __forceinline__ uint32_t block_hits(uint64_t k, uint64_t points, uint32_t rep,
                                               uint32_t k0, uint32_t k1) {
  const Block4 b = philox((uint32_t)k, 0u, rep, TAG_PI, k0, k1);
  return inside(b.x, b.y) + ((2 * k + 1 < points) ? inside(b.z, b.w) : 0u);
}

__global__ void pi_wave_kernel(PiArgs a) {
  const int lane = threadIdx.x & 63;
  const uint64_t r = (uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (r >= a.n_reps) return;  // wave-uniform
  const uint32_t k0 = (uint32_t)a.seed, k1 = (uint32_t)(a.seed >> 32);
  const uint64_t blocks = (a.points + 1) / 2;
  uint32_t hits = 0;
  uint64_t k = lane;
  // four blocks per lane per iteration while all of them exist
  for (; k + 192 < blocks; k += 256) {
    hits += block_hits(k, a.points, (uint32_t)r, k0, k1);
    hits += block_hits(k + 64, a.points, (uint32_t)r, k0, k1);
    hits += block_hits(k + 128, a.points, (uint32_t)r, k0, k1);
    hits += block_hits(k + 192, a.points, (uint32_t)r, k0, k1);
  }
  for (; k < blocks; k += 64) hits += block_hits(k, a.points, (uint32_t)r, k0, k1);
  const int total = group_sum_i((int)hits, 64);
  if (lane == 0) {
    a.hits[r] = total;
    a.estimate[r] = (float)(4.0 * (double)total / (double)a.points);
  }
}

template <int STRIDE>
__global__ void pi_simt_kernel(PiArgs a) {
  if (threadIdx.x % STRIDE) return;
  const uint64_t r = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / STRIDE;
  if (r >= a.n_reps) return;
  const uint32_t k0 = (uint32_t)a.seed, k1 = (uint32_t)(a.seed >> 32);
  const uint64_t blocks = (a.points + 1) / 2;
  uint32_t hits = 0;
  for (uint64_t k = 0; k < blocks; ++k) hits += block_hits(k, a.points, (uint32_t)r, k0, k1);
  a.hits[r] = (int32_t)hits;
  a.estimate[r] = (float)(4.0 * (double)hits / (double)a.points);
}

__global__ void pi_wave_taus_kernel(PiArgs a) {
  const int lane = threadIdx.x & 63;
  const uint64_t r = (uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (r >= a.n_reps) return;  // wave-uniform
  const uint32_t k0 = (uint32_t)a.seed, k1 = (uint32_t)(a.seed >> 32);
  const uint64_t per = (a.points + 63) / 64;
  const uint64_t p0 = min(a.points, (uint64_t)lane * per), p1 = min(a.points, p0 + per);
  Taus t = taus_seed(TAG_PI, 0u, (uint32_t)r, k0, k1);
  taus_skip(t, 2 * p0, a.taus);
  uint32_t hits = 0;
  uint64_t i = p0;
  for (; i + 2 <= p1; i += 2) {
    const uint32_t x0 = taus_next(t), y0 = taus_next(t);
    const uint32_t x1 = taus_next(t), y1 = taus_next(t);
    hits += inside(x0, y0) + inside(x1, y1);
  }
  if (i < p1) {
    const uint32_t x0 = taus_next(t), y0 = taus_next(t);
    hits += inside(x0, y0);
  }
  const int total = group_sum_i((int)hits, 64);
  if (lane == 0) {
    a.hits[r] = total;
    a.estimate[r] = (float)(4.0 * (double)total / (double)a.points);
  }
}

template <int STRIDE>
__global__ void pi_simt_taus_kernel(PiArgs a) {
  if (threadIdx.x % STRIDE) return;
  const uint64_t r = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / STRIDE;
  if (r >= a.n_reps) return;
  const uint32_t k0 = (uint32_t)a.seed, k1 = (uint32_t)(a.seed >> 32);
  Taus t = taus_seed(TAG_PI, 0u, (uint32_t)r, k0, k1);
  uint32_t hits = 0;
  for (uint64_t i = 0; i < a.points; ++i) {
    const uint32_t x = taus_next(t), y = taus_next(t);
    hits += inside(x, y);
  }
  a.hits[r] = (int32_t)hits;
  a.estimate[r] = (float)(4.0 * (double)hits / (double)a.points);
}

template <int X, int RNG>
__global__ __launch_bounds__(64 * X) void pi_wide_kernel(PiArgs a) {
  constexpr uint32_t L = 64 * X;  // lanes per replication
  __shared__ uint32_t sh[X];
  const uint32_t tid = threadIdx.x;
  const uint64_t r = blockIdx.x;
  const uint32_t k0 = (uint32_t)a.seed, k1 = (uint32_t)(a.seed >> 32);
  uint32_t hits = 0;
  if (RNG == RNG_TAUS88) {
    const uint64_t per = (a.points + L - 1) / L;
    const uint64_t p0 = min(a.points, (uint64_t)tid * per), p1 = min(a.points, p0 + per);
    Taus t = taus_seed(TAG_PI, 0u, (uint32_t)r, k0, k1);
    taus_skip(t, 2 * p0, a.taus);
    uint64_t i = p0;
    for (; i + 2 <= p1; i += 2) {
      const uint32_t x0 = taus_next(t), y0 = taus_next(t);
      const uint32_t x1 = taus_next(t), y1 = taus_next(t);
      hits += inside(x0, y0) + inside(x1, y1);
    }
    if (i < p1) {
      const uint32_t x0 = taus_next(t), y0 = taus_next(t);
      hits += inside(x0, y0);
    }
  } else {
    const uint64_t blocks = (a.points + 1) / 2;
    uint64_t k = tid;
    for (; k + 3 * L < blocks; k += 4 * L) {
      hits += block_hits(k, a.points, (uint32_t)r, k0, k1);
      hits += block_hits(k + L, a.points, (uint32_t)r, k0, k1);
      hits += block_hits(k + 2 * L, a.points, (uint32_t)r, k0, k1);
      hits += block_hits(k + 3 * L, a.points, (uint32_t)r, k0, k1);
    }
    for (; k < blocks; k += L) hits += block_hits(k, a.points, (uint32_t)r, k0, k1);
  }
  const int wave_total = group_sum_i((int)hits, 64);
  if ((tid & 63) == 0) sh[tid >> 6] = (uint32_t)wave_total;
  __syncthreads();
  if (tid == 0) {
    uint32_t total = 0;
    for (int w = 0; w < X; ++w) total += sh[w];
    a.hits[r] = (int32_t)total;
    a.estimate[r] = (float)(4.0 * (double)total / (double)a.points);
  }
}

template <int X>
hipError_t wide_launch(const PiArgs &a, hipStream_t s) {
  if (a.rng == RNG_TAUS88)
    hipLaunchKernelGGL((pi_wide_kernel<X, RNG_TAUS88>), dim3((uint32_t)a.n_reps), dim3(64 * X),
                       0, s, a);
  else
    hipLaunchKernelGGL((pi_wide_kernel<X, RNG_PHILOX>), dim3((uint32_t)a.n_reps), dim3(64 * X),
                       0, s, a);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_pi_wave(const PiArgs &a, uint32_t wg, hipStream_t s) {
  // aim at about 4096 wavefronts (four per SIMD) when replications are few
  // and long enough to share out
  if (a.n_reps < 4096 && a.points >= 65536) {
    const uint64_t x = 4096 / a.n_reps;
    if (x >= 16) return wide_launch<16>(a, s);
    if (x >= 8) return wide_launch<8>(a, s);
    if (x >= 4) return wide_launch<4>(a, s);
    if (x >= 2) return wide_launch<2>(a, s);
  }
  const uint32_t wpb = wg / 64;
  const uint64_t blocks = (a.n_reps + wpb - 1) / wpb;
  if (a.rng == RNG_TAUS88)
    hipLaunchKernelGGL(pi_wave_taus_kernel, dim3((uint32_t)blocks), dim3(wg), 0, s, a);
  else
    hipLaunchKernelGGL(pi_wave_kernel, dim3((uint32_t)blocks), dim3(wg), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_pi_simt(const PiArgs &a, bool one_lane, hipStream_t s) {
  const uint32_t wg = 64;
  const uint64_t threads = a.n_reps * (one_lane ? 64 : 1);
  const uint64_t blocks = (threads + wg - 1) / wg;
  const dim3 g((uint32_t)blocks), b(wg);
  if (a.rng == RNG_TAUS88) {
    if (one_lane) hipLaunchKernelGGL(pi_simt_taus_kernel<64>, g, b, 0, s, a);
    else hipLaunchKernelGGL(pi_simt_taus_kernel<1>, g, b, 0, s, a);
  } else {
    if (one_lane) hipLaunchKernelGGL(pi_simt_kernel<64>, g, b, 0, s, a);
    else hipLaunchKernelGGL(pi_simt_kernel<1>, g, b, 0, s, a);
  }
  return hipGetLastError();
}

}  // namespace mrip
