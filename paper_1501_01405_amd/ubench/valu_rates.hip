// Issue-rate microbenchmark for the VALU instructions the MRIP kernels are
// made of (gfx950). Each lane runs 8 independent dependency chains of one
// instruction for many iterations over a grid that fills every SIMD several
// times; the rate is lane-instructions per second, reported beside the
// full-rate figure 256 CU x 4 SIMD x 16 lanes x clock. Two timings per
// instruction: the best of 5 isolated launches (each after a host
// synchronisation), and the average of 20 back-to-back launches after
// 50 ms of continuous launches (the clock state a long run settles in).
//
// Usage: valu_rates [waves_per_simd ...]   (default: 4 8 16)
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <cstdlib>

#define ITERS 1024
#define CHAINS 8

#define CHECK(x)                                                                  \
  do {                                                                            \
    hipError_t e_ = (x);                                                          \
    if (e_ != hipSuccess) {                                                       \
      std::fprintf(stderr, "%s failed: %s\n", #x, hipGetErrorString(e_));          \
      std::exit(1);                                                               \
    }                                                                             \
  } while (0)

enum Op {
  MAD_U64, MUL_HI, MUL_LO, LOG, XOR, XOR3, ADD_F32, FMA_F32, ADD_U32, CVT_F32, FMA_F64,
  BFE_I32, AND_OR, LSHL_OR, LSHL_ADD, LSHLREV
};

template <int OP>
__global__ void rate_kernel(uint32_t *out, uint32_t seed) {
  const uint32_t t = threadIdx.x + blockIdx.x * blockDim.x;
  uint32_t u[CHAINS];
  uint64_t w[CHAINS];
  float f[CHAINS];
  double d[CHAINS];
#pragma unroll
  for (int c = 0; c < CHAINS; ++c) {
    u[c] = t * 2654435761u + seed + c;
    w[c] = u[c];
    f[c] = 1.0f + (float)(u[c] & 1023) * 1e-3f;
    d[c] = (double)f[c];
  }
  const uint32_t k = seed | 1u;
  const float fk = 0.999f;
  for (int i = 0; i < ITERS; ++i) {
#pragma unroll
    for (int c = 0; c < CHAINS; ++c) {
      if (OP == MAD_U64) {
        uint64_t carry;
        asm volatile("v_mad_u64_u32 %0, %1, %2, %3, %4"
                     : "=v"(w[c]), "=s"(carry)
                     : "v"(u[c]), "v"(k), "v"(w[c]));
        u[c] = (uint32_t)w[c];
      } else if (OP == MUL_HI) {
        asm volatile("v_mul_hi_u32 %0, %1, %2" : "=v"(u[c]) : "v"(u[c]), "v"(k));
      } else if (OP == MUL_LO) {
        asm volatile("v_mul_lo_u32 %0, %1, %2" : "=v"(u[c]) : "v"(u[c]), "v"(k));
      } else if (OP == LOG) {
        asm volatile("v_log_f32 %0, %1" : "=v"(f[c]) : "v"(f[c]));
      } else if (OP == XOR) {
        asm volatile("v_xor_b32 %0, %1, %2" : "=v"(u[c]) : "v"(u[c]), "v"(k));
      } else if (OP == XOR3) {
        asm volatile("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x96" : "=v"(u[c]) : "v"(u[c]), "v"(k), "v"(c));
      } else if (OP == ADD_F32) {
        asm volatile("v_add_f32 %0, %1, %2" : "=v"(f[c]) : "v"(f[c]), "v"(fk));
      } else if (OP == FMA_F32) {
        asm volatile("v_fma_f32 %0, %1, %2, %3" : "=v"(f[c]) : "v"(f[c]), "v"(fk), "v"(fk));
      } else if (OP == ADD_U32) {
        asm volatile("v_add_u32 %0, %1, %2" : "=v"(u[c]) : "v"(u[c]), "v"(k));
      } else if (OP == CVT_F32) {
        asm volatile("v_cvt_f32_u32 %0, %1" : "=v"(f[c]) : "v"(u[c]));
        u[c] += 1u;
      } else if (OP == BFE_I32) {
        asm volatile("v_bfe_i32 %0, %1, %2, 2" : "=v"(u[c]) : "v"(u[c]), "v"(k));
      } else if (OP == AND_OR) {
        asm volatile("v_and_or_b32 %0, %1, %2, %3" : "=v"(u[c]) : "v"(u[c]), "v"(k), "v"(c));
      } else if (OP == LSHL_OR) {
        asm volatile("v_lshl_or_b32 %0, %1, 2, %2" : "=v"(u[c]) : "v"(u[c]), "v"(k));
      } else if (OP == LSHL_ADD) {
        asm volatile("v_lshl_add_u32 %0, %1, 3, %2" : "=v"(u[c]) : "v"(u[c]), "v"(k));
      } else if (OP == LSHLREV) {
        asm volatile("v_lshlrev_b32 %0, %1, %2" : "=v"(u[c]) : "v"(k), "v"(u[c]));
      } else if (OP == FMA_F64) {
        asm volatile("v_fma_f64 %0, %1, %2, %3" : "=v"(d[c]) : "v"(d[c]), "v"((double)fk), "v"(d[c]));
      }
    }
  }
  uint32_t acc = 0;
#pragma unroll
  for (int c = 0; c < CHAINS; ++c)
    acc ^= u[c] ^ (uint32_t)w[c] ^ __float_as_uint(f[c]) ^ (uint32_t)__double_as_longlong(d[c]);
  out[t] = acc;
}

struct Rate {
  double isolated, sustained;        // lane-ops/s
  double isolated_ms, sustained_ms;  // per launch
};

template <int OP>
Rate measure(uint32_t *out, int blocks, int threads) {
  hipEvent_t a, b;
  CHECK(hipEventCreate(&a));
  CHECK(hipEventCreate(&b));
  hipLaunchKernelGGL(rate_kernel<OP>, dim3(blocks), dim3(threads), 0, 0, out, 1u);
  CHECK(hipGetLastError());
  CHECK(hipDeviceSynchronize());
  float best = 1e30f;
  for (int r = 0; r < 5; ++r) {
    CHECK(hipEventRecord(a, 0));
    hipLaunchKernelGGL(rate_kernel<OP>, dim3(blocks), dim3(threads), 0, 0, out, (uint32_t)r);
    CHECK(hipEventRecord(b, 0));
    CHECK(hipEventSynchronize(b));
    float ms;
    CHECK(hipEventElapsedTime(&ms, a, b));
    if (ms < best) best = ms;
  }
  // continuous launches for at least 50 ms (at most 4096), then 20 timed
  float warm = 0.0f;
  for (int k = 0; k < 64 && warm < 50.0f; ++k) {
    CHECK(hipEventRecord(a, 0));
    for (int r = 0; r < 64; ++r)
      hipLaunchKernelGGL(rate_kernel<OP>, dim3(blocks), dim3(threads), 0, 0, out, (uint32_t)r);
    CHECK(hipEventRecord(b, 0));
    CHECK(hipEventSynchronize(b));
    float ms;
    CHECK(hipEventElapsedTime(&ms, a, b));
    warm += ms;
  }
  CHECK(hipEventRecord(a, 0));
  for (int r = 0; r < 20; ++r)
    hipLaunchKernelGGL(rate_kernel<OP>, dim3(blocks), dim3(threads), 0, 0, out, (uint32_t)r);
  CHECK(hipEventRecord(b, 0));
  CHECK(hipEventSynchronize(b));
  float sus;
  CHECK(hipEventElapsedTime(&sus, a, b));
  CHECK(hipEventDestroy(a));
  CHECK(hipEventDestroy(b));
  const double lane_ops = (double)blocks * threads * ITERS * CHAINS;
  Rate r;
  r.isolated_ms = best;
  r.sustained_ms = sus / 20.0;
  r.isolated = lane_ops / (best * 1e-3);
  r.sustained = lane_ops / (r.sustained_ms * 1e-3);
  return r;
}

int main(int argc, char **argv) {
  int dev = 0, cus = 0, clock_khz = 0;
  CHECK(hipGetDevice(&dev));
  CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  CHECK(hipDeviceGetAttribute(&clock_khz, hipDeviceAttributeClockRate, dev));
  int wps_list[8] = {4, 8, 16};
  int n_wps = 3;
  if (argc > 1) {
    n_wps = 0;
    for (int i = 1; i < argc && n_wps < 8; ++i) wps_list[n_wps++] = std::atoi(argv[i]);
  }
  const int threads = 256;  // 4 waves per block, one per SIMD
  const double full = (double)cus * 4 * 16 * clock_khz * 1e3;
  for (int wi = 0; wi < n_wps; ++wi) {
  const int waves_per_simd = wps_list[wi];
  const int blocks = cus * waves_per_simd;
  uint32_t *out;
  CHECK(hipMalloc(&out, (size_t)blocks * threads * sizeof(uint32_t)));
  std::printf("cus %d clock_mhz %.0f waves_per_simd %d (16 lanes/SIMD/clk = %.4e lane-ops/s)\n",
              cus, clock_khz / 1e3, waves_per_simd, full);
  struct Row {
    const char *name;
    Rate (*fn)(uint32_t *, int, int);
  } rows[] = {
      {"v_mad_u64_u32", measure<MAD_U64>}, {"v_mul_hi_u32", measure<MUL_HI>},
      {"v_mul_lo_u32", measure<MUL_LO>},   {"v_log_f32", measure<LOG>},
      {"v_xor_b32", measure<XOR>},         {"v_bitop3_b32(xor3)", measure<XOR3>},
      {"v_add_f32", measure<ADD_F32>},     {"v_fma_f32", measure<FMA_F32>},
      {"v_add_u32", measure<ADD_U32>},     {"v_cvt_f32_u32(+add)", measure<CVT_F32>},
      {"v_fma_f64", measure<FMA_F64>},     {"v_bfe_i32", measure<BFE_I32>},
      {"v_and_or_b32", measure<AND_OR>},   {"v_lshl_or_b32", measure<LSHL_OR>},
      {"v_lshl_add_u32", measure<LSHL_ADD>}, {"v_lshlrev_b32", measure<LSHLREV>},
  };
  for (const Row &r : rows) {
    const Rate m = r.fn(out, blocks, threads);
    std::printf("%-22s isolated %.4e lane-ops/s %.3f of full rate (%.3f ms)  "
                "sustained %.4e lane-ops/s %.3f of full rate (%.3f ms)\n",
                r.name, m.isolated, m.isolated / full, m.isolated_ms, m.sustained,
                m.sustained / full, m.sustained_ms);
  }
  CHECK(hipFree(out));
  }
  return 0;
}
