// Lattice random-walk replication engines (paper section 5.1, third model).
//
// WAVE mapping: one replication per wavefront, lane w = walker w. The
// replication's visited-site bitmap (grid^2 bits, 512 B at 64x64) lives in
// LDS and every move sets its bit with an LDS atomic or; at the end the
// lanes popcount the bitmap and sum squared displacements across the wave.
//
// SIMT mapping: one replication per lane; the lane walks its walkers one
// after the other and keeps the replication's bitmap in global memory, the
// per-thread state the paper's thread-per-replication form implies. The
// same kernel with one working lane per wavefront is the paper's own WLP.
//
// On taus88 streams (RNG = RNG_TAUS88) move t of walker w takes bits
// 2(t&15) of output w ceil(T/16) + (t>>4) of the replication's stream: each
// walker reads a contiguous run, so a WAVE lane jumps to its walker's run and
// a SIMT lane reads the stream in order, walker after walker.
#include "device.hpp"
#include "kernels.hpp"
#include "taus.hpp"

namespace mrip {

namespace {

__device__ __forceinline__ void step_delta(uint32_t d, int &dx, int &dy) {
  dx = (d == 0u) - (d == 1u);
  dy = (d == 2u) - (d == 3u);
}

// Set the visited bit of lattice site c (row-major) in an LDS bitmap.
__device__ __forceinline__ void mark(uint32_t *bm, int c) { atomicOr(&bm[c >> 5], 1u << (c & 31)); }

template <int GRID, bool LDS>
__device__ __forceinline__ void move1(uint32_t d, bool active, int &x, int &y, int &ux, int &uy,
                                      uint32_t *bm) {
  int dx, dy;
  step_delta(d, dx, dy);
  ux += dx;
  uy += dy;
  x = (x + dx) & (GRID - 1);
  y = (y + dy) & (GRID - 1);
  const int c = y * GRID + x;
  if (LDS) {
    if (active) mark(bm, c);
  } else {
    bm[c >> 5] |= 1u << (c & 31);
  }
}

// Up to 16 moves from one 32-bit word (2 bits each, lowest first): moves
// g .. min(g + 16, steps) - 1.
template <int GRID, bool LDS>
__device__ __forceinline__ void walk16(uint32_t word, uint32_t g, uint32_t steps, bool active,
                                       int &x, int &y, int &ux, int &uy, uint32_t *bm) {
  if (g + 16u <= steps) {
#pragma unroll
    for (int i = 0; i < 16; ++i) move1<GRID, LDS>((word >> (2 * i)) & 3u, active, x, y, ux, uy, bm);
  } else {
    for (uint32_t i = 0; g + i < steps; ++i)
      move1<GRID, LDS>((word >> (2 * i)) & 3u, active, x, y, ux, uy, bm);
  }
}

template <int GRID, int RNG>
__global__ void rw_wave_kernel(RwArgs a) {
  constexpr int WORDS = GRID * GRID / 32;
  extern __shared__ uint32_t lds[];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint64_t r = (uint64_t)blockIdx.x * (blockDim.x >> 6) + wave;
  const uint32_t k0 = (uint32_t)a.seed, k1 = (uint32_t)(a.seed >> 32);
  uint32_t *bm = lds + wave * WORDS;
  for (int i = lane; i < WORDS; i += 64) bm[i] = 0u;
  __syncthreads();

  const bool active = r < a.n_reps && (uint32_t)lane < a.walkers;
  const uint32_t w = (uint32_t)lane;
  int x = (int)(((w % 8u) * (GRID / 8) + GRID / 16) % GRID);
  int y = (int)(((w / 8u) * (GRID / 8) + GRID / 16) % GRID);
  int ux = 0, uy = 0;
  if (active) mark(bm, y * GRID + x);

  if (RNG == RNG_TAUS88) {
    Taus t = taus_seed(TAG_RW, 0u, (uint32_t)r, k0, k1);
    taus_skip(t, (uint64_t)w * ((a.steps + 15) / 16), a.taus);
    for (uint32_t g = 0; g < a.steps; g += 16)
      walk16<GRID, true>(taus_next(t), g, a.steps, active, x, y, ux, uy, bm);
  } else {
    for (uint32_t g = 0; g < a.steps; g += 64) {
      const Block4 b = philox(g >> 6, w, (uint32_t)r, TAG_RW, k0, k1);
      walk16<GRID, true>(b.x, g, a.steps, active, x, y, ux, uy, bm);
      walk16<GRID, true>(b.y, g + 16, a.steps, active, x, y, ux, uy, bm);
      walk16<GRID, true>(b.z, g + 32, a.steps, active, x, y, ux, uy, bm);
      walk16<GRID, true>(b.w, g + 48, a.steps, active, x, y, ux, uy, bm);
    }
  }
  __syncthreads();
  int cnt = 0;
  for (int i = lane; i < WORDS; i += 64) cnt += __popc(bm[i]);
  cnt = group_sum_i(cnt, 64);
  const int sd = active ? ux * ux + uy * uy : 0;
  const int ssd = group_sum_i(sd, 64);
  if (lane == 0 && r < a.n_reps) {
    a.ssd[r] = ssd;
    a.distinct[r] = cnt;
  }
}

// STRIDE = 1: one replication per lane. STRIDE = 64: one replication per
// wavefront with only its first lane working (the paper's WLP form, 63 of
// 64 lanes idle).
template <int GRID, int STRIDE, int RNG>
__global__ void rw_simt_kernel(RwArgs a) {
  constexpr int WORDS = GRID * GRID / 32;
  if (threadIdx.x % STRIDE) return;
  const uint64_t r = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / STRIDE;
  if (r >= a.n_reps) return;
  const uint32_t k0 = (uint32_t)a.seed, k1 = (uint32_t)(a.seed >> 32);
  uint32_t *bm = a.scratch_bitmaps + r * WORDS;
  for (int i = 0; i < WORDS; ++i) bm[i] = 0u;
  int ssd = 0;
  Taus t;
  if (RNG == RNG_TAUS88) t = taus_seed(TAG_RW, 0u, (uint32_t)r, k0, k1);
  for (uint32_t w = 0; w < a.walkers; ++w) {
    int x = (int)(((w % 8u) * (GRID / 8) + GRID / 16) % GRID);
    int y = (int)(((w / 8u) * (GRID / 8) + GRID / 16) % GRID);
    int ux = 0, uy = 0;
    bm[(y * GRID + x) >> 5] |= 1u << ((y * GRID + x) & 31);
    if (RNG == RNG_TAUS88) {
      for (uint32_t g = 0; g < a.steps; g += 16)
        walk16<GRID, false>(taus_next(t), g, a.steps, true, x, y, ux, uy, bm);
    } else {
      for (uint32_t g = 0; g < a.steps; g += 64) {
        const Block4 b = philox(g >> 6, w, (uint32_t)r, TAG_RW, k0, k1);
        walk16<GRID, false>(b.x, g, a.steps, true, x, y, ux, uy, bm);
        walk16<GRID, false>(b.y, g + 16, a.steps, true, x, y, ux, uy, bm);
        walk16<GRID, false>(b.z, g + 32, a.steps, true, x, y, ux, uy, bm);
        walk16<GRID, false>(b.w, g + 48, a.steps, true, x, y, ux, uy, bm);
      }
    }
    ssd += ux * ux + uy * uy;
  }
  int cnt = 0;
  for (int i = 0; i < WORDS; ++i) cnt += __popc(bm[i]);
  a.ssd[r] = ssd;
  a.distinct[r] = cnt;
}

template <int GRID>
hipError_t wave_launch(const RwArgs &a, uint32_t wg, hipStream_t s) {
  const uint32_t wpb = wg / 64;
  const uint64_t blocks = (a.n_reps + wpb - 1) / wpb;
  const size_t lds = (size_t)wpb * (GRID * GRID / 32) * sizeof(uint32_t);
  if (a.rng == RNG_TAUS88)
    hipLaunchKernelGGL((rw_wave_kernel<GRID, RNG_TAUS88>), dim3((uint32_t)blocks), dim3(wg), lds, s, a);
  else
    hipLaunchKernelGGL((rw_wave_kernel<GRID, RNG_PHILOX>), dim3((uint32_t)blocks), dim3(wg), lds, s, a);
  return hipGetLastError();
}

template <int GRID>
hipError_t simt_launch(const RwArgs &a, bool one_lane, hipStream_t s) {
  const uint32_t wg = 64;
  const uint64_t threads = a.n_reps * (one_lane ? 64 : 1);
  const uint64_t blocks = (threads + wg - 1) / wg;
  const dim3 g((uint32_t)blocks), b(wg);
  if (a.rng == RNG_TAUS88) {
    if (one_lane) hipLaunchKernelGGL((rw_simt_kernel<GRID, 64, RNG_TAUS88>), g, b, 0, s, a);
    else hipLaunchKernelGGL((rw_simt_kernel<GRID, 1, RNG_TAUS88>), g, b, 0, s, a);
  } else {
    if (one_lane) hipLaunchKernelGGL((rw_simt_kernel<GRID, 64, RNG_PHILOX>), g, b, 0, s, a);
    else hipLaunchKernelGGL((rw_simt_kernel<GRID, 1, RNG_PHILOX>), g, b, 0, s, a);
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_rw_wave(const RwArgs &a, uint32_t wg, hipStream_t s) {
  switch (a.grid) {
    case 16: return wave_launch<16>(a, wg, s);
    case 32: return wave_launch<32>(a, wg, s);
    case 64: return wave_launch<64>(a, wg, s);
    case 128: return wave_launch<128>(a, wg, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_rw_simt(const RwArgs &a, bool one_lane, hipStream_t s) {
  switch (a.grid) {
    case 16: return simt_launch<16>(a, one_lane, s);
    case 32: return simt_launch<32>(a, one_lane, s);
    case 64: return simt_launch<64>(a, one_lane, s);
    case 128: return simt_launch<128>(a, one_lane, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace mrip
