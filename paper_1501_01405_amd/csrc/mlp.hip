// Control-variate network kernels: a 10-128-128-1 ReLU MLP with bfloat16
// operands and fp32 accumulation on the gfx950 matrix cores
// (v_mfma_f32_16x16x32_bf16), forward and backward, plus Adam.
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
// The last layer (128 -> 1) is a VALU dot product.
//
// Every matrix product rounds both operands to bf16 (round to nearest even,
// v_cvt_pk_bf16_f32); biases, ReLU masks and the loss stay fp32.
#include <hip/hip_runtime.h>

#include "device.hpp"
#include "mlp.hpp"

namespace mrip {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int DIN = MLP_DIN, H = MLP_H, TS = 64;  // samples per workgroup
constexpr int SP = TS + 8;                       // padded row of the staging arrays

struct FwdLds {
  __bf16 w2[H][H + 8];   // W2[h2][h1]
  __bf16 w1[H][32 + 8];  // W1[h][f], f >= 10 zero
  float b1[H], b2[H], w3[H];
};

struct BwdLds {
  FwdLds f;
  __bf16 w2t[H][H + 8];  // W2^T[h1][h2]
  __bf16 h1t[H][SP];     // H1^T[h1][s]
  __bf16 dz2t[H][SP];    // dZ2^T[h2][s]
  __bf16 dz1t[H][SP];    // dZ1^T[h1][s]
  __bf16 xt[16][SP];     // X^T[f][s], f < 16
  float red[3][4][H];    // per-wave sums of db1, db2, dW3
  float red_s[2][4];     // per-wave sums of loss and db3
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
    L.w3[e] = bfr(theta[MLP_OFF_W3 + e]);
  }
}

// Forward pass of the wave's 16 samples. On return z1, z2 hold the
// pre-activations of this lane's units (16t + 4g + i) for its sample, and
// the return value is the prediction for the sample of column l%16.
__device__ float forward_wave(const FwdLds &L, bf16x8 xb, float b3, float z1[8][4],
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
  float part = 0.0f;
#pragma unroll
  for (int t = 0; t < 8; ++t)
#pragma unroll
    for (int i = 0; i < 4; ++i)
      part = fmaf(L.w3[16 * t + 4 * g + i], bfr(fmaxf(z2[t][i], 0.0f)), part);
  part += __shfl_xor(part, 16, 64);
  part += __shfl_xor(part, 32, 64);
  return part + b3;
}

__device__ __forceinline__ bf16x8 load_x(const float *x, int s, bool valid, int g) {
  bf16x8 xb;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int f = 8 * g + i;
    xb[i] = bf((valid && f < DIN) ? x[(uint64_t)s * DIN + f] : 0.0f);
  }
  return xb;
}

__global__ __launch_bounds__(256) void mlp_forward_kernel(const float *theta, const float *x,
                                                          uint64_t n, float *y, float out_scale,
                                                          float out_shift) {
  extern __shared__ __attribute__((aligned(16))) char smem[];
  FwdLds &L = *reinterpret_cast<FwdLds *>(smem);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, g = lane >> 4, c = lane & 15;
  const uint64_t s = (uint64_t)blockIdx.x * TS + 16 * w + c;
  const bool valid = s < n;
  stage_weights(theta, L, nullptr);
  const bf16x8 xb = load_x(x, (int)s, valid, g);
  __syncthreads();
  float z1[8][4], z2[8][4];
  const float yh = forward_wave(L, xb, theta[MLP_OFF_B3], z1, z2);
  if (g == 0 && valid) y[s] = out_shift + out_scale * yh;
}

// Sum over the 16 lanes of a row (same g, every sample column).
__device__ __forceinline__ float row16_sum(float v) {
#pragma unroll
  for (int off = 1; off < 16; off <<= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Gradient of mean((g(x) - y)^2) over n samples: one partial row per
// workgroup (MLP_PSTRIDE floats: the 18049 gradients, then the loss sum).
__global__ __launch_bounds__(256) void mlp_grad_kernel(const float *theta, const float *x,
                                                       const float *y, uint64_t n, float inv_n,
                                                       float *partial) {
  extern __shared__ __attribute__((aligned(16))) char smem[];
  BwdLds &B = *reinterpret_cast<BwdLds *>(smem);
  FwdLds &L = B.f;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, g = lane >> 4, c = lane & 15;
  const int sl = 16 * w + c;  // sample within the workgroup
  const uint64_t s = (uint64_t)blockIdx.x * TS + sl;
  const bool valid = s < n;
  stage_weights(theta, L, &B);
  const bf16x8 xb = load_x(x, (int)s, valid, g);
  if (g < 2) {
#pragma unroll
    for (int i = 0; i < 8; ++i) B.xt[8 * g + i][sl] = xb[i];
  }
  __syncthreads();

  float z1[8][4], z2[8][4];
  const float yh = forward_wave(L, xb, theta[MLP_OFF_B3], z1, z2);
  const float err = valid ? yh - y[s] : 0.0f;
  const float dy = 2.0f * err * inv_n;
  const float dyb = bfr(dy);

  // last layer and the ReLU of the second
  float dz2[8][4];
  float p3[8][4];
#pragma unroll
  for (int t = 0; t < 8; ++t)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int h = 16 * t + 4 * g + i;
      p3[t][i] = dyb * bfr(fmaxf(z2[t][i], 0.0f));
      dz2[t][i] = z2[t][i] > 0.0f ? L.w3[h] * dyb : 0.0f;
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
  // per-wave sums over samples of db1, db2, dW3
#pragma unroll
  for (int t = 0; t < 8; ++t)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int h = 16 * t + 4 * g + i;
      const float v1 = row16_sum(dz1[t][i]);
      const float v2 = row16_sum(dz2[t][i]);
      const float v3 = row16_sum(p3[t][i]);
      if (c == 0) {
        B.red[0][w][h] = v1;
        B.red[1][w][h] = v2;
        B.red[2][w][h] = v3;
      }
    }
  {
    float l2 = (g == 0) ? err * err : 0.0f;
    float d3 = (g == 0) ? dy : 0.0f;
    l2 = row16_sum(l2);
    d3 = row16_sum(d3);
    if (lane == 0) {
      B.red_s[0][w] = l2;
      B.red_s[1][w] = d3;
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
  if (tid < H) {
    const int h = tid;
    out[MLP_OFF_B1 + h] = ((B.red[0][0][h] + B.red[0][1][h]) + B.red[0][2][h]) + B.red[0][3][h];
    out[MLP_OFF_B2 + h] = ((B.red[1][0][h] + B.red[1][1][h]) + B.red[1][2][h]) + B.red[1][3][h];
    out[MLP_OFF_W3 + h] = ((B.red[2][0][h] + B.red[2][1][h]) + B.red[2][2][h]) + B.red[2][3][h];
  }
  if (tid == 0) {
    out[MLP_OFF_B3] = ((B.red_s[1][0] + B.red_s[1][1]) + B.red_s[1][2]) + B.red_s[1][3];
    out[MLP_NPARAMS] = ((B.red_s[0][0] + B.red_s[0][1]) + B.red_s[0][2]) + B.red_s[0][3];
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
                              float out_scale, float out_shift, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const size_t lds = sizeof(FwdLds);
  hipError_t e = allow_lds(mlp_forward_kernel, lds);
  if (e != hipSuccess) return e;
  const uint64_t blocks = (n + TS - 1) / TS;
  hipLaunchKernelGGL(mlp_forward_kernel, dim3((uint32_t)blocks), dim3(256), lds, s, theta, x, n,
                     y, out_scale, out_shift);
  return hipGetLastError();
}

hipError_t launch_mlp_grad(const float *theta, const float *x, const float *y, uint64_t n,
                           float *partial, hipStream_t s) {
  const size_t lds = sizeof(BwdLds);
  hipError_t e = allow_lds(mlp_grad_kernel, lds);
  if (e != hipSuccess) return e;
  const uint64_t blocks = (n + TS - 1) / TS;
  hipLaunchKernelGGL(mlp_grad_kernel, dim3((uint32_t)blocks), dim3(256), lds, s, theta, x, y, n,
                     1.0f / (float)n, partial);
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

}  // namespace mrip
