// Control-variate network kernels: a 10-128-128-4 ReLU MLP with bfloat16
// operands and fp32 accumulation on the gfx950 matrix cores
// (v_mfma_f32_16x16x32_bf16), forward and backward, plus Adam. Its four
// outputs are the coefficients of four zero-mean controls; training fits
// sum_k g_k(x) z_k to a target with per-sample multipliers z.
//
// Layout. A workgroup of 4 wavefronts takes 64 samples, 16 per wave. Every
// layer is computed transposed, activations as [hidden][sample]:
//     Z1^T = W1 . X^T,  Z2^T = W2 . H1^T,  dH1^T = W2^T . dZ2^T
// so a layer's output tile (lane l holds rows 4(l/16)+i, column l%16) is
// already the next product's B operand up to a permutation of the
// contraction index. The permutation is applied to the A operand's loads
// instead (k-slot (g, i) of a 32-wide step j <-> hidden unit
// 32j + 4g + (i&3) + 16(i>>2)), so activations never leave registers between
// layers. Weight gradients contract over samples: dZ^T and the layer inputs
// are staged in LDS as [unit][sample] and multiplied with samples as K.
// The last layer (128 -> 4) is four VALU dot products.
//
// Every matrix product rounds both operands to bf16 (round to nearest even,
// v_cvt_pk_bf16_f32); biases, ReLU masks and the loss stay fp32.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/mrip.h"
#include "device.hpp"
#include "mlp.hpp"

namespace mrip {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int DIN = MLP_DIN, H = MLP_H, TS = 64;  // samples per workgroup
constexpr int SP = TS + 8;                       // padded row of the staging arrays

constexpr int DOUT = MLP_DOUT;

struct FwdLds {
  __bf16 w2[H][H + 8];   // W2[h2][h1]
  __bf16 w1[H][32 + 8];  // W1[h][f], f >= 10 zero
  float b1[H], b2[H], w3[DOUT][H];
};

struct BwdLds {
  FwdLds f;
  __bf16 w2t[H][H + 8];  // W2^T[h1][h2]
  __bf16 h1t[H][SP];     // H1^T[h1][s]
  __bf16 dz2t[H][SP];    // dZ2^T[h2][s]
  __bf16 dz1t[H][SP];    // dZ1^T[h1][s]
  __bf16 xt[16][SP];     // X^T[f][s], f < 16
  float red[2 + DOUT][4][H];  // per-wave sums of db1, db2, dW3[k]
  float red_s[1 + DOUT][4];   // per-wave sums of loss and db3[k]
};

__device__ __forceinline__ __bf16 bf(float v) { return (__bf16)v; }
__device__ __forceinline__ float bfr(float v) { return (float)(__bf16)v; }

__device__ __forceinline__ f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// A operand with the permuted contraction index: columns 32j+4g..+3 and
// 32j+16+4g..+3 of row `row`.
__device__ __forceinline__ bf16x8 load_perm(const __bf16 *row, int j, int g) {
  const bf16x4 lo = *(const bf16x4 *)(row + 32 * j + 4 * g);
  const bf16x4 hi = *(const bf16x4 *)(row + 32 * j + 16 + 4 * g);
  return bf16x8{lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
}

// Stage W1, W2 (bf16), b1, b2, bf16-rounded W3 into LDS.
__device__ void stage_weights(const float *theta, FwdLds &L, BwdLds *B) {
  const int tid = threadIdx.x;
  for (int e = tid; e < H * H; e += blockDim.x) {
    const int r = e / H, c = e % H;
    const __bf16 v = bf(theta[MLP_OFF_W2 + e]);
    L.w2[r][c] = v;
    if (B) B->w2t[c][r] = v;
  }
  for (int e = tid; e < H * 32; e += blockDim.x) {
    const int r = e / 32, f = e % 32;
    L.w1[r][f] = f < DIN ? bf(theta[MLP_OFF_W1 + r * DIN + f]) : bf(0.0f);
  }
  for (int e = tid; e < H; e += blockDim.x) {
    L.b1[e] = theta[MLP_OFF_B1 + e];
    L.b2[e] = theta[MLP_OFF_B2 + e];
  }
  for (int e = tid; e < DOUT * H; e += blockDim.x) L.w3[e / H][e % H] = bfr(theta[MLP_OFF_W3 + e]);
}

struct Out4 {
  float v[DOUT];
};

// Forward pass of the wave's 16 samples. On return z1, z2 hold the
// pre-activations of this lane's units (16t + 4g + i) for its sample, and
// the return value is the four outputs for the sample of column l%16.
__device__ Out4 forward_wave(const FwdLds &L, bf16x8 xb, const float *b3, float z1[8][4],
                             float z2[8][4]) {
  const int lane = threadIdx.x & 63, g = lane >> 4, c = lane & 15;
#pragma unroll
  for (int t = 0; t < 8; ++t) {
    const bf16x8 a = *(const bf16x8 *)&L.w1[16 * t + c][8 * g];
    const f32x4 acc = mfma(a, xb, f32x4{0.f, 0.f, 0.f, 0.f});
#pragma unroll
    for (int i = 0; i < 4; ++i) z1[t][i] = acc[i] + L.b1[16 * t + 4 * g + i];
  }
  bf16x8 hb[4];
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      hb[j][i] = bf(fmaxf(z1[2 * j][i], 0.0f));
      hb[j][4 + i] = bf(fmaxf(z1[2 * j + 1][i], 0.0f));
    }
#pragma unroll
  for (int t = 0; t < 8; ++t) {
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int j = 0; j < 4; ++j) acc = mfma(load_perm(&L.w2[16 * t + c][0], j, g), hb[j], acc);
#pragma unroll
    for (int i = 0; i < 4; ++i) z2[t][i] = acc[i] + L.b2[16 * t + 4 * g + i];
  }
  Out4 o;
#pragma unroll
  for (int k = 0; k < DOUT; ++k) {
    float part = 0.0f;
#pragma unroll
    for (int t = 0; t < 8; ++t)
#pragma unroll
      for (int i = 0; i < 4; ++i)
        part = fmaf(L.w3[k][16 * t + 4 * g + i], bfr(fmaxf(z2[t][i], 0.0f)), part);
    part += __shfl_xor(part, 16, 64);
    part += __shfl_xor(part, 32, 64);
    o.v[k] = part + b3[k];
  }
  return o;
}

__device__ __forceinline__ bf16x8 load_x(const float *x, uint64_t s, bool valid, int g) {
  bf16x8 xb;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int f = 8 * g + i;
    xb[i] = bf((valid && f < DIN) ? x[s * DIN + f] : 0.0f);
  }
  return xb;
}

__global__ __launch_bounds__(256) void mlp_forward_kernel(const float *theta, const float *x,
                                                          uint64_t n, float *y) {
  extern __shared__ __attribute__((aligned(16))) char smem[];
  FwdLds &L = *reinterpret_cast<FwdLds *>(smem);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, g = lane >> 4, c = lane & 15;
  const uint64_t s = (uint64_t)blockIdx.x * TS + 16 * w + c;
  const bool valid = s < n;
  stage_weights(theta, L, nullptr);
  const bf16x8 xb = load_x(x, s, valid, g);
  __syncthreads();
  float z1[8][4], z2[8][4];
  const Out4 yh = forward_wave(L, xb, theta + MLP_OFF_B3, z1, z2);
  if (g == 0 && valid) *(float4 *)(y + 4 * s) = float4{yh.v[0], yh.v[1], yh.v[2], yh.v[3]};
}

// Inference of the control variate, fused: z-score the raw features, the
// forward pass, then per sample (one lane each) the controls' multipliers,
// the network's control h = sum_k g_k z_k and the residual
// d = y - coef[bin] . (h, z_4..z_7), in fp64 (rounded once to fp32). The
// z-scores round as the standalone normalisation does ((x - mean) * inv_std
// in fp32, then bf16 for the product).
__global__ __launch_bounds__(256) void cv_infer_kernel(const float *theta, const float *x,
                                                       uint64_t n, CvInferArgs a) {
  extern __shared__ __attribute__((aligned(16))) char smem[];
  FwdLds &L = *reinterpret_cast<FwdLds *>(smem);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, g = lane >> 4, c = lane & 15;
  const uint64_t s = (uint64_t)blockIdx.x * TS + 16 * w + c;
  const bool valid = s < n;
  stage_weights(theta, L, nullptr);
  bf16x8 xb;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int f = 8 * g + i;
    xb[i] = bf((valid && f < DIN) ? (x[s * DIN + f] - a.mean[f]) * a.inv_std[f] : 0.0f);
  }
  __syncthreads();
  float z1[8][4], z2[8][4];
  const Out4 o = forward_wave(L, xb, theta + MLP_OFF_B3, z1, z2);
  if (g != 0 || !valid) return;
  if (a.g) *(float4 *)(a.g + 4 * s) = float4{o.v[0], o.v[1], o.v[2], o.v[3]};
  const double N = (double)a.customers[s];
  const double m = (double)(float)(1.0 / (double)a.mu[s]);
  const double sc[4] = {1.0 / N, 1.0 / N, (1.0 / m) / N, (1.0 / m) / N};
  const float *cl = a.ctl + 8 * s;
  double h = 0.0;
#pragma unroll
  for (int k = 0; k < 4; ++k) h += (double)o.v[k] * (double)(float)((double)cl[k] * sc[k]);
  const float *cf = a.coef + (uint64_t)a.bin[s] * CV_NCOEF;
  double f = (double)cf[0] * h;
#pragma unroll
  for (int k = 0; k < 4; ++k) f += (double)cf[1 + k] * (double)(float)((double)cl[4 + k] * sc[k]);
  a.h[s] = (float)h;
  a.d[s] = (float)((double)a.y[s] - f);
}

// Sum over the 16 lanes of a row (same g, every sample column).
__device__ __forceinline__ float row16_sum(float v) {
#pragma unroll
  for (int off = 1; off < 16; off <<= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Gradient of mean((sum_k g_k(x) z_k - y)^2) over n samples (z nullable:
// z = e_0): one partial row per workgroup (MLP_PSTRIDE floats: the
// MLP_NPARAMS gradients, then the loss sum). The output gradient
// dy_k = 2 (pred - y) z_k / n is formed in fp32 and enters the products as
// bf16.
__global__ __launch_bounds__(256) void mlp_grad_kernel(const float *theta, const float *x,
                                                       const float *z, const float *y, uint64_t n,
                                                       float inv_n, float *partial) {
  extern __shared__ __attribute__((aligned(16))) char smem[];
  BwdLds &B = *reinterpret_cast<BwdLds *>(smem);
  FwdLds &L = B.f;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, g = lane >> 4, c = lane & 15;
  const int sl = 16 * w + c;  // sample within the workgroup
  const uint64_t s = (uint64_t)blockIdx.x * TS + sl;
  const bool valid = s < n;
  stage_weights(theta, L, &B);
  const bf16x8 xb = load_x(x, s, valid, g);
  if (g < 2) {
#pragma unroll
    for (int i = 0; i < 8; ++i) B.xt[8 * g + i][sl] = xb[i];
  }
  __syncthreads();

  float z1[8][4], z2[8][4];
  const Out4 yh = forward_wave(L, xb, theta + MLP_OFF_B3, z1, z2);
  float zz[DOUT] = {1.0f, 0.0f, 0.0f, 0.0f};
  if (z && valid) {
    const float4 zv = *(const float4 *)(z + 4 * s);
    zz[0] = zv.x;
    zz[1] = zv.y;
    zz[2] = zv.z;
    zz[3] = zv.w;
  }
  float pred = 0.0f;
#pragma unroll
  for (int k = 0; k < DOUT; ++k) pred = fmaf(yh.v[k], zz[k], pred);
  const float err = valid ? pred - y[s] : 0.0f;
  const float e2 = 2.0f * err * inv_n;
  float dy[DOUT], dyb[DOUT];
#pragma unroll
  for (int k = 0; k < DOUT; ++k) {
    dy[k] = e2 * zz[k];
    dyb[k] = bfr(dy[k]);
  }

  // last layer: dW3[k] partial sums over the wave's samples, and the ReLU of
  // the second layer
  float dz2[8][4];
#pragma unroll
  for (int t = 0; t < 8; ++t)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int h = 16 * t + 4 * g + i;
      float d = 0.0f;
#pragma unroll
      for (int k = 0; k < DOUT; ++k) d = fmaf(L.w3[k][h], dyb[k], d);
      dz2[t][i] = z2[t][i] > 0.0f ? d : 0.0f;
      const float h2 = bfr(fmaxf(z2[t][i], 0.0f));
#pragma unroll
      for (int k = 0; k < DOUT; ++k) {
        const float v = row16_sum(dyb[k] * h2);
        if (c == 0) B.red[2 + k][w][h] = v;
      }
    }
  // dH1^T = W2^T . dZ2^T, then the ReLU of the first layer
  bf16x8 db[4];
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      db[j][i] = bf(dz2[2 * j][i]);
      db[j][4 + i] = bf(dz2[2 * j + 1][i]);
    }
  float dz1[8][4];
#pragma unroll
  for (int t = 0; t < 8; ++t) {
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int j = 0; j < 4; ++j) acc = mfma(load_perm(&B.w2t[16 * t + c][0], j, g), db[j], acc);
#pragma unroll
    for (int i = 0; i < 4; ++i) dz1[t][i] = z1[t][i] > 0.0f ? acc[i] : 0.0f;
  }

  // stage operands of the weight gradients ([unit][sample])
#pragma unroll
  for (int t = 0; t < 8; ++t)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int h = 16 * t + 4 * g + i;
      B.h1t[h][sl] = bf(fmaxf(z1[t][i], 0.0f));
      B.dz2t[h][sl] = bf(dz2[t][i]);
      B.dz1t[h][sl] = bf(dz1[t][i]);
    }
  // per-wave sums over samples of db1, db2, db3 and the loss
#pragma unroll
  for (int t = 0; t < 8; ++t)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int h = 16 * t + 4 * g + i;
      const float v1 = row16_sum(dz1[t][i]);
      const float v2 = row16_sum(dz2[t][i]);
      if (c == 0) {
        B.red[0][w][h] = v1;
        B.red[1][w][h] = v2;
      }
    }
  {
    const float l2 = row16_sum(g == 0 ? err * err : 0.0f);
    if (lane == 0) B.red_s[0][w] = l2;
#pragma unroll
    for (int k = 0; k < DOUT; ++k) {
      const float d3 = row16_sum(g == 0 ? dy[k] : 0.0f);
      if (lane == 0) B.red_s[1 + k][w] = d3;
    }
  }
  __syncthreads();

  float *out = partial + (uint64_t)blockIdx.x * MLP_PSTRIDE;
  // dW2[h2][h1] = sum_s dZ2^T[h2][s] H1^T[h1][s]: wave w owns h2 tiles 2w, 2w+1
#pragma unroll
  for (int tt = 0; tt < 2; ++tt) {
    const int t2 = 2 * w + tt;
#pragma unroll
    for (int t1 = 0; t1 < 8; ++t1) {
      f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const bf16x8 a = *(const bf16x8 *)&B.dz2t[16 * t2 + c][32 * j + 8 * g];
        const bf16x8 b = *(const bf16x8 *)&B.h1t[16 * t1 + c][32 * j + 8 * g];
        acc = mfma(a, b, acc);
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
        out[MLP_OFF_W2 + (16 * t2 + 4 * g + i) * H + 16 * t1 + c] = acc[i];
    }
  }
  // dW1[h1][f] = sum_s dZ1^T[h1][s] X^T[f][s]: wave w owns h1 tiles 2w, 2w+1
#pragma unroll
  for (int tt = 0; tt < 2; ++tt) {
    const int t1 = 2 * w + tt;
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const bf16x8 a = *(const bf16x8 *)&B.dz1t[16 * t1 + c][32 * j + 8 * g];
      const bf16x8 b = *(const bf16x8 *)&B.xt[c][32 * j + 8 * g];
      acc = mfma(a, b, acc);
    }
    if (c < DIN) {
#pragma unroll
      for (int i = 0; i < 4; ++i) out[MLP_OFF_W1 + (16 * t1 + 4 * g + i) * DIN + c] = acc[i];
    }
  }
  // fixed-order sums of the four waves' rows: db1, db2, then dW3[k]
  for (int e = tid; e < (2 + DOUT) * H; e += blockDim.x) {
    const int r = e / H, h = e % H;
    const float v = ((B.red[r][0][h] + B.red[r][1][h]) + B.red[r][2][h]) + B.red[r][3][h];
    const int off = r == 0 ? MLP_OFF_B1 + h : r == 1 ? MLP_OFF_B2 + h : MLP_OFF_W3 + (r - 2) * H + h;
    out[off] = v;
  }
  if (tid <= DOUT) {
    const float v = ((B.red_s[tid][0] + B.red_s[tid][1]) + B.red_s[tid][2]) + B.red_s[tid][3];
    out[tid == 0 ? MLP_NPARAMS : MLP_OFF_B3 + tid - 1] = v;
  }
}

// grad[p] = sum over workgroups of partial[wg][p] in a fixed order; the loss
// slot becomes the mean squared error. With `adam` set, also one Adam step.
__global__ void grad_reduce_kernel(const float *partial, uint32_t n_wg, float inv_n, float *grad,
                                   float *loss, float *theta, float *m, float *v, AdamArgs ad) {
  const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p > (uint32_t)MLP_NPARAMS) return;
  float s = 0.0f;
  for (uint32_t k = 0; k < n_wg; ++k) s += partial[(uint64_t)k * MLP_PSTRIDE + p];
  if (p == (uint32_t)MLP_NPARAMS) {
    if (loss) *loss = s * inv_n;
    return;
  }
  if (grad) grad[p] = s;
  if (theta) {
    const float mm = ad.beta1 * m[p] + (1.0f - ad.beta1) * s;
    const float vv = ad.beta2 * v[p] + (1.0f - ad.beta2) * s * s;
    m[p] = mm;
    v[p] = vv;
    theta[p] -= ad.lr * (mm / ad.bc1) / (sqrtf(vv / ad.bc2) + ad.eps);
  }
}

__global__ void adam_kernel(float *theta, float *m, float *v, const float *grad, uint64_t n,
                            AdamArgs ad) {
  const uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const float gr = grad[p];
  const float mm = ad.beta1 * m[p] + (1.0f - ad.beta1) * gr;
  const float vv = ad.beta2 * v[p] + (1.0f - ad.beta2) * gr * gr;
  m[p] = mm;
  v[p] = vv;
  theta[p] -= ad.lr * (mm / ad.bc1) / (sqrtf(vv / ad.bc2) + ad.eps);
}

template <class K>
hipError_t allow_lds(K kernel, size_t bytes) {
  static bool done = false;  // per kernel instantiation; idempotent
  if (done) return hipSuccess;
  hipError_t e = hipFuncSetAttribute((const void *)kernel,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e == hipSuccess) done = true;
  return e;
}

}  // namespace

size_t mlp_partial_rows(uint64_t n) { return (size_t)((n + TS - 1) / TS); }

hipError_t launch_mlp_forward(const float *theta, const float *x, uint64_t n, float *y,
                              hipStream_t s) {
  if (n == 0) return hipSuccess;
  const size_t lds = sizeof(FwdLds);
  hipError_t e = allow_lds(mlp_forward_kernel, lds);
  if (e != hipSuccess) return e;
  const uint64_t blocks = (n + TS - 1) / TS;
  hipLaunchKernelGGL(mlp_forward_kernel, dim3((uint32_t)blocks), dim3(256), lds, s, theta, x, n,
                     y);
  return hipGetLastError();
}

hipError_t launch_cv_infer(const float *theta, const float *x, uint64_t n, const CvInferArgs &a,
                           hipStream_t s) {
  if (n == 0) return hipSuccess;
  const size_t lds = sizeof(FwdLds);
  hipError_t e = allow_lds(cv_infer_kernel, lds);
  if (e != hipSuccess) return e;
  const uint64_t blocks = (n + TS - 1) / TS;
  hipLaunchKernelGGL(cv_infer_kernel, dim3((uint32_t)blocks), dim3(256), lds, s, theta, x, n, a);
  return hipGetLastError();
}

hipError_t launch_mlp_grad(const float *theta, const float *x, const float *z, const float *y,
                           uint64_t n, float *partial, hipStream_t s) {
  const size_t lds = sizeof(BwdLds);
  hipError_t e = allow_lds(mlp_grad_kernel, lds);
  if (e != hipSuccess) return e;
  const uint64_t blocks = (n + TS - 1) / TS;
  hipLaunchKernelGGL(mlp_grad_kernel, dim3((uint32_t)blocks), dim3(256), lds, s, theta, x, z, y,
                     n, 1.0f / (float)n, partial);
  return hipGetLastError();
}

hipError_t launch_grad_reduce(const float *partial, uint32_t n_wg, uint64_t n, float *grad,
                              float *loss, float *theta, float *m, float *v, const AdamArgs &ad,
                              hipStream_t s) {
  const uint32_t threads = 256, blocks = (MLP_NPARAMS + 1 + threads - 1) / threads;
  hipLaunchKernelGGL(grad_reduce_kernel, dim3(blocks), dim3(threads), 0, s, partial, n_wg,
                     1.0f / (float)n, grad, loss, theta, m, v, ad);
  return hipGetLastError();
}

hipError_t launch_adam(float *theta, float *m, float *v, const float *grad, uint64_t n,
                       const AdamArgs &ad, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const uint64_t blocks = (n + 255) / 256;
  hipLaunchKernelGGL(adam_kernel, dim3((uint32_t)blocks), dim3(256), 0, s, theta, m, v, grad, n,
                     ad);
  return hipGetLastError();
}

// ------------------------------------------------ gradient without allocation
// The partial-gradient rows of mrip_mlp_grad_noalloc live in a file-scope
// device array: each GPU the library runs on holds its own copy, at its own
// address, until the process ends. Host code reaches it only through the
// address hipGetSymbolAddress returns on that device (the array's name is a
// host-side stand-in there, not a device address).
namespace {

constexpr uint64_t NOALLOC_MAX_N = MRIP_MLP_GRAD_NOALLOC_MAX;
constexpr uint64_t NOALLOC_ROWS = NOALLOC_MAX_N / TS;
static_assert(NOALLOC_MAX_N % TS == 0, "whole partial rows");

__device__ __align__(256) float scratch[NOALLOC_ROWS * MLP_PSTRIDE];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
float *g_scratch_ptr[MAX_DEVICES] = {};

// The device address of this device's scratch, looked up on its first use
// with the device current.
hipError_t scratch_on_device(float **out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = (float *)p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

}  // namespace
}  // namespace mrip

extern "C" MRIP_API mrip_status mrip_mlp_grad_noalloc(const float *theta_dev, const float *x_dev,
                                                      const float *z_dev, const float *y_dev,
                                                      uint64_t n, float *grad_dev, float *loss_dev,
                                                      void *hip_stream) {
  using namespace mrip;
  if (n == 0 || !theta_dev || !x_dev || !y_dev || !grad_dev) return MRIP_E_INVAL;
  if (n > NOALLOC_MAX_N) return MRIP_E_INVAL;  // beyond the scratch array
  if (z_dev && ((uintptr_t)z_dev & 15u)) return MRIP_E_INVAL;
  float *part = nullptr;
  if (scratch_on_device(&part) != hipSuccess) return MRIP_E_HIP;
  hipStream_t s = (hipStream_t)hip_stream;
  const uint64_t rows = (n + TS - 1) / TS;
  // every row the reduction reads is written first by the gradient kernel
  if (launch_mlp_grad(theta_dev, x_dev, z_dev, y_dev, n, part, s) != hipSuccess) return MRIP_E_HIP;
  AdamArgs none{};
  if (launch_grad_reduce(part, (uint32_t)rows, n, grad_dev, loss_dev, nullptr, nullptr, nullptr,
                         none, s) != hipSuccess)
    return MRIP_E_HIP;
  return MRIP_OK;
}

