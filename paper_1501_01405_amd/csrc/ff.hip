// Forest-fire cellular automaton replication engines (Drossel-Schwabl,
// synchronous, torus, von Neumann neighbourhood).
//
// The grid is held as two bit planes, `tree` and `burning` (empty = neither),
// 32 cells per word, bit i of word k of a row = cell x = 32k + i. One step is
// then word-parallel logic:
//     nb      = burning shifted left/right (funnel shifts with wrap) | row above | row below
//     ignite  = tree & (nb | [u < TF])
//     grow    = empty & [u < TP]
//     burning' = ignite,  tree' = (tree & ~ignite) | grow,  burnt += popcount(ignite)
// and the random bits come one Philox block per 4 cells.
//
// WAVE mapping: one replication per wavefront. The whole 128x128 grid of a
// replication fits in 16 VGPRs per lane (2 rows x 2 planes x 4 words); row
// exchange with the lanes above and below goes through cross-lane shuffles,
// so the grid never leaves the register file during the 2000 steps.
//
// SIMT mapping: one replication per lane. A 4 KiB grid per lane cannot stay
// in registers; it lives in global memory laid out [plane][row][word][rep]
// so that the 64 lanes of a wave touch 64 consecutive words, and is updated
// in place one row at a time (old rows y-1 and 0 are kept in registers).
#include "device.hpp"
#include "kernels.hpp"

namespace mrip {

namespace {

// mask = 2 mask + [u < t]: the borrow of u - t shifts straight into the mask
// (v_sub_co_u32 then v_addc_co_u32), two instructions per bit where a
// compare, a select and a shift-or would take three.
__device__ __forceinline__ uint32_t shift_in_less(uint32_t mask, uint32_t u, uint32_t t) {
  uint32_t tmp;
  asm("v_sub_co_u32 %0, vcc, %2, %3\n\t"
      "v_addc_co_u32 %1, vcc, %1, %1, vcc"
      : "=&v"(tmp), "+v"(mask)
      : "v"(u), "v"(t)
      : "vcc");
  return mask;
}

// Bits [u < TP] and [u < TF] for the 32 cells of one word: cells
// 32k..32k+31 of row y use blocks q0..q0+7, word (cell & 3).
__device__ __forceinline__ void draw_masks(uint32_t t, uint32_t q0, uint32_t rep, uint32_t k0,
                                           uint32_t k1, uint32_t tp, uint32_t tf, uint32_t &ltp,
                                           uint32_t &ltf) {
  uint32_t mp = 0u, mf = 0u;
  // kept as a loop: eight inlined Philox blocks per word would stop the
  // callers' loops over the register-resident grid from unrolling
#pragma unroll 2
  for (int m = 7; m >= 0; --m) {
    const Block4 b = philox(t, q0 + (uint32_t)m, rep, TAG_FF, k0, k1);
    mp = shift_in_less(mp, b.w, tp);
    mf = shift_in_less(mf, b.w, tf);
    mp = shift_in_less(mp, b.z, tp);
    mf = shift_in_less(mf, b.z, tf);
    mp = shift_in_less(mp, b.y, tp);
    mf = shift_in_less(mf, b.y, tf);
    mp = shift_in_less(mp, b.x, tp);
    mf = shift_in_less(mf, b.x, tf);
  }
  ltp = mp;
  ltf = mf;
}

// bit x of the result = bit x-1 of the row (word k of DW, wrapping)
__device__ __forceinline__ uint32_t from_left(uint32_t cur, uint32_t prev_word) {
  return __builtin_amdgcn_alignbit(cur, prev_word, 31);
}
// bit x of the result = bit x+1 of the row
__device__ __forceinline__ uint32_t from_right(uint32_t next_word, uint32_t cur) {
  return __builtin_amdgcn_alignbit(next_word, cur, 1);
}

template <int GRID>
__global__ void ff_wave_kernel(FfArgs a) {
  constexpr int RPL = GRID / 64;  // rows per lane
  constexpr int DW = GRID / 32;   // words per row
  const int lane = threadIdx.x & 63;
  const uint64_t r = (uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (r >= a.n_reps) return;  // wave-uniform
  const uint32_t k0 = (uint32_t)a.seed, k1 = (uint32_t)(a.seed >> 32);
  const int up_lane = (lane + 63) & 63, dn_lane = (lane + 1) & 63;

  uint32_t T[RPL][DW], B[RPL][DW];
#pragma unroll
  for (int i = 0; i < RPL; ++i)
#pragma unroll
    for (int k = 0; k < DW; ++k) T[i][k] = B[i][k] = 0u;
  int burnt = 0;

  for (uint32_t t = 0; t < a.steps; ++t) {
    uint32_t up[DW], dn[DW];
#pragma unroll
    for (int k = 0; k < DW; ++k) {
      up[k] = (uint32_t)__shfl((int)B[RPL - 1][k], up_lane, 64);
      dn[k] = (uint32_t)__shfl((int)B[0][k], dn_lane, 64);
    }
    uint32_t nT[RPL][DW], nB[RPL][DW];
#pragma unroll
    for (int i = 0; i < RPL; ++i) {
      const uint32_t y = (uint32_t)lane * RPL + i;
#pragma unroll
      for (int k = 0; k < DW; ++k) {
        const uint32_t above = i == 0 ? up[k] : B[i - 1][k];
        const uint32_t below = i == RPL - 1 ? dn[k] : B[i + 1][k];
        const uint32_t nb = from_left(B[i][k], B[i][(k + DW - 1) % DW]) |
                            from_right(B[i][(k + 1) % DW], B[i][k]) | above | below;
        uint32_t ltp, ltf;
        draw_masks(t, (y * GRID + 32u * k) >> 2, (uint32_t)r, k0, k1, a.tp, a.tf, ltp, ltf);
        const uint32_t tree = T[i][k], burn = B[i][k];
        const uint32_t ign = tree & (nb | ltf);
        const uint32_t grow = ~(tree | burn) & ltp;
        nB[i][k] = ign;
        nT[i][k] = (tree & ~ign) | grow;
        burnt += __popc(ign);
      }
    }
#pragma unroll
    for (int i = 0; i < RPL; ++i)
#pragma unroll
      for (int k = 0; k < DW; ++k) {
        T[i][k] = nT[i][k];
        B[i][k] = nB[i][k];
      }
  }
  burnt = group_sum_i(burnt, 64);
  if (lane == 0) a.burnt[r] = burnt;
}

// STRIDE = 1: one replication per lane; 64: one working lane per wavefront
// (the paper's WLP form).
template <int GRID, int STRIDE>
__global__ void ff_simt_kernel(FfArgs a) {
  constexpr int DW = GRID / 32;
  if (threadIdx.x % STRIDE) return;
  const uint64_t r = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / STRIDE;
  if (r >= a.n_reps) return;
  const uint64_t R = a.n_reps;
  const uint32_t k0 = (uint32_t)a.seed, k1 = (uint32_t)(a.seed >> 32);
  // word (plane p, row y, word k) of replication r
  auto at = [&](int p, uint32_t y, int k) -> uint32_t * {
    return a.state + (((uint64_t)p * GRID + y) * DW + k) * R + r;
  };
  for (uint32_t y = 0; y < (uint32_t)GRID; ++y)
    for (int k = 0; k < DW; ++k) {
      *at(0, y, k) = 0u;
      *at(1, y, k) = 0u;
    }
  int burnt = 0;
  for (uint32_t t = 0; t < a.steps; ++t) {
    uint32_t first[DW], prev[DW], cur[DW];
    for (int k = 0; k < DW; ++k) {
      first[k] = *at(1, 0, k);
      cur[k] = first[k];
      prev[k] = *at(1, GRID - 1, k);
    }
    for (uint32_t y = 0; y < (uint32_t)GRID; ++y) {
      uint32_t nxt[DW];
      for (int k = 0; k < DW; ++k) nxt[k] = (y == GRID - 1) ? first[k] : *at(1, y + 1, k);
      for (int k = 0; k < DW; ++k) {
        const uint32_t nb = from_left(cur[k], cur[(k + DW - 1) % DW]) |
                            from_right(cur[(k + 1) % DW], cur[k]) | prev[k] | nxt[k];
        uint32_t ltp, ltf;
        draw_masks(t, (y * GRID + 32u * k) >> 2, (uint32_t)r, k0, k1, a.tp, a.tf, ltp, ltf);
        const uint32_t tree = *at(0, y, k), burn = cur[k];
        const uint32_t ign = tree & (nb | ltf);
        const uint32_t grow = ~(tree | burn) & ltp;
        *at(0, y, k) = (tree & ~ign) | grow;
        *at(1, y, k) = ign;
        burnt += __popc(ign);
      }
      for (int k = 0; k < DW; ++k) {
        prev[k] = cur[k];
        cur[k] = nxt[k];
      }
    }
  }
  a.burnt[r] = burnt;
}

template <int GRID>
hipError_t wave_launch(const FfArgs &a, uint32_t wg, hipStream_t s) {
  const uint32_t wpb = wg / 64;
  const uint64_t blocks = (a.n_reps + wpb - 1) / wpb;
  hipLaunchKernelGGL(ff_wave_kernel<GRID>, dim3((uint32_t)blocks), dim3(wg), 0, s, a);
  return hipGetLastError();
}

template <int GRID>
hipError_t simt_launch(const FfArgs &a, bool one_lane, hipStream_t s) {
  const uint32_t wg = 64;
  const uint64_t threads = a.n_reps * (one_lane ? 64 : 1);
  const uint64_t blocks = (threads + wg - 1) / wg;
  if (one_lane) hipLaunchKernelGGL((ff_simt_kernel<GRID, 64>), dim3((uint32_t)blocks), dim3(wg), 0, s, a);
  else hipLaunchKernelGGL((ff_simt_kernel<GRID, 1>), dim3((uint32_t)blocks), dim3(wg), 0, s, a);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_ff_wave(const FfArgs &a, uint32_t wg, hipStream_t s) {
  switch (a.grid) {
    case 64: return wave_launch<64>(a, wg, s);
    case 128: return wave_launch<128>(a, wg, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_ff_simt(const FfArgs &a, bool one_lane, hipStream_t s) {
  switch (a.grid) {
    case 32: return simt_launch<32>(a, one_lane, s);
    case 64: return simt_launch<64>(a, one_lane, s);
    case 96: return simt_launch<96>(a, one_lane, s);
    case 128: return simt_launch<128>(a, one_lane, s);
    case 160: return simt_launch<160>(a, one_lane, s);
    case 192: return simt_launch<192>(a, one_lane, s);
    case 224: return simt_launch<224>(a, one_lane, s);
    case 256: return simt_launch<256>(a, one_lane, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace mrip
