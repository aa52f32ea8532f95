// Device building blocks shared by the MRIP kernels (gfx950, wave64).
//
//  * Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11, section 3.2). The key
//    is the 64-bit seed and is wave-uniform, so the ten round keys stay in
//    scalar registers; the counter carries the logical ids (draw index,
//    entity, replication, model tag), never hardware lane numbers.
//  * Variates: u in (0, 1] from the top 24 bits (exact in fp32), the
//    exponential by inversion through the hardware log2.
//  * Cross-lane helpers: DPP row shifts for the 16-lane max-plus scan,
//    shuffles for end-of-replication reductions.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mrip {

enum : uint32_t { TAG_RW = 1, TAG_MM1 = 2, TAG_FF = 3, TAG_PI = 4 };

struct Block4 {
  uint32_t x, y, z, w;
};

// a ^ b ^ c in one gfx950 v_bitop3_b32 (truth table 0x96)
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
  return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

// One Philox4x32-10 block. The 32x32->64 products become one
// v_mad_u64_u32 each; the xor with the counter word and the round key is a
// single three-input bitop.
__device__ __forceinline__ Block4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                         uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t n0 = xor3((uint32_t)(p1 >> 32), c1, k0);
    const uint32_t n2 = xor3((uint32_t)(p0 >> 32), c3, k1);
    c1 = (uint32_t)p1;
    c3 = (uint32_t)p0;
    c0 = n0;
    c2 = n2;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return Block4{c0, c1, c2, c3};
}

__device__ __forceinline__ uint32_t word_of(const Block4 &b, uint32_t j) {
  return j == 0 ? b.x : j == 1 ? b.y : j == 2 ? b.z : b.w;
}

// Exponential variate: scale * log2(u) with scale = -(1/rate) * ln 2
// (computed on the host), u = ((x >> 8) + 1) * 2^-24 in (0, 1]. u is formed
// as fma(x & ~0xff, 2^-32, 2^-24): the masked word converts exactly (24
// significant bits), and the fused multiply-add is exact because its result
// k * 2^-24, k <= 2^24, is representable; one instruction fewer than shift,
// add, convert, scale.
__device__ __forceinline__ float log2_u01(uint32_t x) {
  const float u = __builtin_fmaf((float)(x & 0xFFFFFF00u), 0x1p-32f, 0x1p-24f);
  return __builtin_amdgcn_logf(u);
}
__device__ __forceinline__ float exp_variate(uint32_t x, float neg_mean_ln2) {
  return neg_mean_ln2 * log2_u01(x);
}

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// DPP: row_shr:n moves lane i-n -> i inside each row of 16 lanes; lanes
// whose source falls outside the row keep `identity`.
template <int N>
__device__ __forceinline__ float row_shr(float v, float identity) {
  return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(identity), __float_as_int(v),
                                                    0x110 + N, 0xF, 0xF, false));
}

__device__ __forceinline__ float readlane_f(float v, int lane) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

// Error-free transformation of a + b (Knuth's two-sum).
__device__ __forceinline__ void two_sum(float a, float b, float &s, float &e) {
  s = a + b;
  const float bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

// Kahan-compensated accumulator (sum - comp is the running total).
struct Kahan {
  float sum = 0.0f, comp = 0.0f;
  __device__ __forceinline__ void add(float x) {
    const float y = x - comp;
    const float t = sum + y;
    comp = (t - sum) - y;
    sum = t;
  }
  __device__ __forceinline__ float value() const { return sum - comp; }
};

// Sum of (hi, lo) float pairs over aligned groups of `width` lanes with a
// compensated butterfly; every lane of the group gets the total.
__device__ __forceinline__ float group_sum_compensated(float v, int width) {
  float hi = v, lo = 0.0f;
  for (int off = 1; off < width; off <<= 1) {
    const float ohi = __shfl_xor(hi, off, 64);
    const float olo = __shfl_xor(lo, off, 64);
    float s, e;
    two_sum(hi, ohi, s, e);
    hi = s;
    lo = lo + olo + e;
  }
  return hi + lo;
}

__device__ __forceinline__ float group_max(float v, int width) {
  for (int off = 1; off < width; off <<= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
  return v;
}

__device__ __forceinline__ int group_sum_i(int v, int width) {
  for (int off = 1; off < width; off <<= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ __forceinline__ long long group_sum_ll(long long v, int width) {
  for (int off = 1; off < width; off <<= 1) v += __shfl_xor(v, off, 64);
  return v;
}

}  // namespace mrip
