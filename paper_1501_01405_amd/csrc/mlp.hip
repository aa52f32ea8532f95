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

// The weights as the products read them from LDS. b1 .. b3 are contiguous
// fp32 in the order of the flat parameters (b2, W3 and b3 are one run there).
struct FwdLds {
  __bf16 w2[H][H + 8];   // W2[h2][h1]
  __bf16 w1[H][32 + 8];  // W1[h][f], f >= 10 zero
  float b1[H], b2[H], w3[DOUT][H], b3[DOUT];  // w3 bf16-rounded
};
// The gradient kernel's weights: FwdLds and W2^T, all in bf16 where a
// product reads them. Kept in global memory in exactly this layout (the
// training's Adam step rewrites it with the weights) and staged into LDS by
// a flat 16-byte copy.
struct MlpImage {
  FwdLds f;
  __bf16 w2t[H][H + 8];  // W2^T[h1][h2]
};
static_assert(sizeof(FwdLds) % 16 == 0 && sizeof(MlpImage) == MLP_IMAGE_BYTES,
              "16-byte copies of the image");
static_assert(offsetof(FwdLds, w3) == offsetof(FwdLds, b2) + 4 * H &&
                  offsetof(FwdLds, b3) == offsetof(FwdLds, w3) + 4 * DOUT * H,
              "b2, W3, b3 contiguous as in the flat parameters");

struct BwdLds {
  MlpImage m;            // m.f.w2 is reused for H2^T[h2][s] once the forward pass is done
  __bf16 h1t[H][SP];     // H1^T[h1][s]
  __bf16 dz2t[H][SP];    // dZ2^T[h2][s]
  __bf16 dz1t[H][SP];    // dZ1^T[h1][s]
  __bf16 xt[16][SP];     // X^T[f][s], f < 16
  __bf16 dyt[DOUT][SP];  // dY^T[k][s]
  float red[2][4][H];    // per-wave sums of db1, db2
  float red_s[1 + DOUT][4];  // per-wave sums of loss and db3[k]
};
static_assert(sizeof(__bf16) * H * SP <= sizeof(__bf16) * H * (H + 8), "H2^T fits in W2's place");

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

// The image value of flat parameter p (bf16 where a product reads it).
__device__ __forceinline__ void image_put(MlpImage &m, uint32_t p, float v) {
  if (p < (uint32_t)MLP_OFF_B1) {
    m.f.w1[p / DIN][p % DIN] = bf(v);
  } else if (p < (uint32_t)MLP_OFF_W2) {
    m.f.b1[p - MLP_OFF_B1] = v;
  } else if (p < (uint32_t)MLP_OFF_B2) {
    const uint32_t q = p - MLP_OFF_W2, r = q / H, c = q % H;
    m.f.w2[r][c] = bf(v);
    m.w2t[c][r] = bf(v);
  } else if (p < (uint32_t)MLP_OFF_W3) {
    m.f.b2[p - MLP_OFF_B2] = v;
  } else if (p < (uint32_t)MLP_OFF_B3) {
    const uint32_t q = p - MLP_OFF_W3;
    m.f.w3[q / H][q % H] = bfr(v);
  } else {
    m.f.b3[p - MLP_OFF_B3] = v;
  }
}

// Stage FwdLds from the flat fp32 parameters (16-byte aligned), 256
// threads: every thread issues all of its 16-byte loads before its first
// store.
__device__ __forceinline__ void stage_theta(const float *__restrict__ theta, FwdLds &L) {
  const int tid = threadIdx.x;
  const float4 *t4 = reinterpret_cast<const float4 *>(theta);
  constexpr int W2V = H * H / 4 / 256;  // 16 vectors of W2 per thread
  constexpr int W1V = H * DIN / 4;      // 320 vectors of W1
  constexpr int TAILV = (H + DOUT * H + DOUT) / 4;  // b2, W3, b3: 161 vectors
  static_assert(MLP_OFF_W2 % 4 == 0 && MLP_OFF_B1 % 4 == 0 && MLP_OFF_B2 % 4 == 0, "float4 runs");
  float4 w2v[W2V];
#pragma unroll
  for (int k = 0; k < W2V; ++k) w2v[k] = t4[MLP_OFF_W2 / 4 + tid + 256 * k];
  const float4 zero4 = {0.f, 0.f, 0.f, 0.f};
  const float4 w1a = t4[MLP_OFF_W1 / 4 + tid];
  const float4 w1b = tid + 256 < W1V ? t4[MLP_OFF_W1 / 4 + 256 + tid] : zero4;
  const float4 b1v = tid < H / 4 ? t4[MLP_OFF_B1 / 4 + tid] : zero4;
  const float4 tv = tid < TAILV ? t4[MLP_OFF_B2 / 4 + tid] : zero4;
#pragma unroll
  for (int k = 0; k < W2V; ++k) {
    const int e = tid + 256 * k, r = e >> 5, c0 = 4 * (e & 31);
    *(bf16x4 *)&L.w2[r][c0] = bf16x4{bf(w2v[k].x), bf(w2v[k].y), bf(w2v[k].z), bf(w2v[k].w)};
  }
  auto put_w1 = [&](int q, float4 v) {
    const float f4[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int i = 0; i < 4; ++i) L.w1[(q + i) / DIN][(q + i) % DIN] = bf(f4[i]);
  };
  put_w1(4 * tid, w1a);
  if (tid + 256 < W1V) put_w1(4 * (256 + tid), w1b);
  {  // zero columns 10..31 of row tid/2: 10..15 by even threads, 16..31 by odd ones
    const int r = tid >> 1;
    if (tid & 1) {
      *(uint4 *)&L.w1[r][16] = uint4{0u, 0u, 0u, 0u};
      *(uint4 *)&L.w1[r][24] = uint4{0u, 0u, 0u, 0u};
    } else {
      *(uint32_t *)&L.w1[r][10] = 0u;
      *(uint2 *)&L.w1[r][12] = uint2{0u, 0u};
    }
  }
  if (tid < H / 4) *(float4 *)&L.b1[4 * tid] = b1v;
  if (tid < TAILV) {
    float4 v = tv;
    if (tid >= H / 4 && tid < (H + DOUT * H) / 4) {  // W3 enters its product as bf16
      v.x = bfr(v.x);
      v.y = bfr(v.y);
      v.z = bfr(v.z);
      v.w = bfr(v.w);
    }
    reinterpret_cast<float4 *>(reinterpret_cast<char *>(&L) + offsetof(FwdLds, b2))[tid] = v;
  }
}

// Flat copy of BYTES (a multiple of 16) from global memory into LDS, 256
// threads, all loads of a thread issued before its first store.
template <int BYTES>
__device__ __forceinline__ void copy_to_lds(const void *__restrict__ src, void *dst) {
  constexpr int V = BYTES / 16, PER = (V + 255) / 256;
  const int tid = threadIdx.x;
  const uint4 *s4 = reinterpret_cast<const uint4 *>(src);
  uint4 *d4 = reinterpret_cast<uint4 *>(dst);
  uint4 v[PER];
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int e = tid + 256 * k;
    v[k] = e < V ? s4[e] : uint4{0u, 0u, 0u, 0u};
  }
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int e = tid + 256 * k;
    if (e < V) d4[e] = v[k];
  }
}

struct Out4 {
  float v[DOUT];
};

// Forward pass of the wave's 16 samples. On return z1, z2 hold the
// pre-activations of this lane's units (16t + 4g + i) for its sample, and
// the return value is the four outputs for the sample of column l%16.
__device__ Out4 forward_wave(const FwdLds &L, bf16x8 xb, float z1[8][4], float z2[8][4]) {
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
    o.v[k] = part + L.b3[k];
  }
  return o;
}

// The features of sample s for k-slots 8g..8g+7 (zero beyond the 10th, and
// for an invalid sample), optionally z-scored. Every load is issued
// unconditionally from a clamped address, so that they are all in flight at
// once.
__device__ __forceinline__ bf16x8 load_x(const float *x, uint64_t s, bool valid, int g,
                                         const float *mean = nullptr,
                                         const float *inv_std = nullptr) {
  float v[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int f = 8 * g + i;
    const bool ok = valid && f < DIN;
    v[i] = x[ok ? s * DIN + f : 0];
    if (mean) v[i] = (v[i] - mean[ok ? f : 0]) * inv_std[ok ? f : 0];
    v[i] = ok ? v[i] : 0.0f;
  }
  bf16x8 xb;
#pragma unroll
  for (int i = 0; i < 8; ++i) xb[i] = bf(v[i]);
  return xb;
}

__global__ __launch_bounds__(256) void mlp_forward_kernel(const float *theta, const float *x,
                                                          uint64_t n, float *y) {
  extern __shared__ __attribute__((aligned(16))) char smem[];
  FwdLds &L = *reinterpret_cast<FwdLds *>(smem);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, g = lane >> 4, c = lane & 15;
  const uint64_t s = (uint64_t)blockIdx.x * TS + 16 * w + c;
  const bool valid = s < n;
  const bf16x8 xb = load_x(x, s, valid, g);
  stage_theta(theta, L);
  __syncthreads();
  float z1[8][4], z2[8][4];
  const Out4 yh = forward_wave(L, xb, z1, z2);
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
  const bf16x8 xb = load_x(x, s, valid, g, a.mean, a.inv_std);
  stage_theta(theta, L);
  __syncthreads();
  float z1[8][4], z2[8][4];
  const Out4 o = forward_wave(L, xb, z1, z2);
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

// Sum over the 16 lanes of a row (same g, every sample column), on the
// DPP network: pairs, quads, then rotations of the row by 4 and 8; every
// lane of the row ends with the sum.
template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, true));
}
__device__ __forceinline__ float row16_sum(float v) {
  v += dpp<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp<0x124>(v);  // row_ror:4
  v += dpp<0x128>(v);  // row_ror:8
  return v;
}

// Gradient of mean((sum_k g_k(x) z_k - y)^2) over n samples (z nullable:
// z = e_0): one partial row per workgroup (MLP_PSTRIDE floats: the
// MLP_NPARAMS gradients, then the loss sum). The output gradient
// dy_k = 2 (pred - y) z_k / n is formed in fp32 and enters the products as
// bf16. The weights come from their image (MlpImage).
__global__ __launch_bounds__(256) void mlp_grad_kernel(const MlpImage *img, const float *x,
                                                       const float *z, const float *y, uint64_t n,
                                                       float inv_n, float *partial) {
  extern __shared__ __attribute__((aligned(16))) char smem[];
  BwdLds &B = *reinterpret_cast<BwdLds *>(smem);
  FwdLds &L = B.m.f;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, g = lane >> 4, c = lane & 15;
  const int sl = 16 * w + c;  // sample within the workgroup
  const uint64_t s = (uint64_t)blockIdx.x * TS + sl;
  const bool valid = s < n;
  const uint64_t sc = valid ? s : 0;  // a readable row for the unconditional loads
  const bf16x8 xb = load_x(x, s, valid, g);
  const float4 zv = z ? *(const float4 *)(z + 4 * sc) : float4{1.0f, 0.0f, 0.0f, 0.0f};
  const float yv = y[sc];
  copy_to_lds<sizeof(MlpImage)>(img, &B.m);
  if (g < 2) {
#pragma unroll
    for (int i = 0; i < 8; ++i) B.xt[8 * g + i][sl] = xb[i];
  }
  __syncthreads();

  float z1[8][4], z2[8][4];
  const Out4 yh = forward_wave(L, xb, z1, z2);
  const float zz[DOUT] = {zv.x, zv.y, zv.z, zv.w};
  float pred = 0.0f;
#pragma unroll
  for (int k = 0; k < DOUT; ++k) pred = fmaf(yh.v[k], zz[k], pred);
  const float err = valid ? pred - yv : 0.0f;
  const float e2 = 2.0f * err * inv_n;
  float dy[DOUT], dyb[DOUT];
#pragma unroll
  for (int k = 0; k < DOUT; ++k) {
    dy[k] = e2 * zz[k];
    dyb[k] = bfr(dy[k]);
  }

  // the ReLU of the second layer
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
    for (int j = 0; j < 4; ++j) acc = mfma(load_perm(&B.m.w2t[16 * t + c][0], j, g), db[j], acc);
#pragma unroll
    for (int i = 0; i < 4; ++i) dz1[t][i] = z1[t][i] > 0.0f ? acc[i] : 0.0f;
  }
  __syncthreads();  // every wave is past its forward pass: W2's place takes H2^T

  // stage the operands of the weight gradients ([unit][sample])
  __bf16(*h2t)[SP] = reinterpret_cast<__bf16(*)[SP]>(&L.w2[0][0]);
#pragma unroll
  for (int t = 0; t < 8; ++t)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int h = 16 * t + 4 * g + i;
      B.h1t[h][sl] = bf(fmaxf(z1[t][i], 0.0f));
      h2t[h][sl] = bf(fmaxf(z2[t][i], 0.0f));
      B.dz2t[h][sl] = bf(dz2[t][i]);
      B.dz1t[h][sl] = bf(dz1[t][i]);
    }
  if (g == 0) {
#pragma unroll
    for (int k = 0; k < DOUT; ++k) B.dyt[k][sl] = bf(dy[k]);
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
  // dW1[h1][f] = sum_s dZ1^T[h1][s] X^T[f][s] and
  // dW3^T[h2][k] = sum_s H2^T[h2][s] dY^T[k][s]: wave w owns tiles 2w, 2w+1
  const bf16x8 zero8 = {};
#pragma unroll
  for (int tt = 0; tt < 2; ++tt) {
    const int t = 2 * w + tt;
    f32x4 acc1 = {0.f, 0.f, 0.f, 0.f}, acc3 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const bf16x8 a1 = *(const bf16x8 *)&B.dz1t[16 * t + c][32 * j + 8 * g];
      const bf16x8 b1 = *(const bf16x8 *)&B.xt[c][32 * j + 8 * g];
      acc1 = mfma(a1, b1, acc1);
      const bf16x8 a3 = *(const bf16x8 *)&h2t[16 * t + c][32 * j + 8 * g];
      const bf16x8 b3 = c < DOUT ? *(const bf16x8 *)&B.dyt[c][32 * j + 8 * g] : zero8;
      acc3 = mfma(a3, b3, acc3);
    }
    if (c < DIN) {
#pragma unroll
      for (int i = 0; i < 4; ++i) out[MLP_OFF_W1 + (16 * t + 4 * g + i) * DIN + c] = acc1[i];
    }
    if (c < DOUT) {
#pragma unroll
      for (int i = 0; i < 4; ++i) out[MLP_OFF_W3 + c * H + 16 * t + 4 * g + i] = acc3[i];
    }
  }
  // fixed-order sums of the four waves' rows: db1, db2
  for (int e = tid; e < 2 * H; e += blockDim.x) {
    const int r = e / H, h = e % H;
    const float v = ((B.red[r][0][h] + B.red[r][1][h]) + B.red[r][2][h]) + B.red[r][3][h];
    out[(r == 0 ? MLP_OFF_B1 : MLP_OFF_B2) + h] = v;
  }
  if (tid <= DOUT) {
    const float v = ((B.red_s[tid][0] + B.red_s[tid][1]) + B.red_s[tid][2]) + B.red_s[tid][3];
    out[tid == 0 ? MLP_NPARAMS : MLP_OFF_B3 + tid - 1] = v;
  }
}

// The image of the flat parameters: one thread per parameter, through the
// same image_put the Adam step uses, then one per padding element (zero).
__global__ void mlp_pack_kernel(const float *theta, MlpImage *img) {
  constexpr uint32_t RP = 8, FP = 40 - DIN;  // padding per row of W2 / W2^T, of W1
  constexpr uint32_t PADS = 2 * H * RP + H * FP;
  const uint32_t e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < (uint32_t)MLP_NPARAMS) {
    image_put(*img, e, theta[e]);
    return;
  }
  const uint32_t q = e - MLP_NPARAMS;
  if (q < H * RP)
    img->f.w2[q / RP][H + q % RP] = bf(0.0f);
  else if (q < 2 * H * RP)
    img->w2t[(q - H * RP) / RP][H + (q - H * RP) % RP] = bf(0.0f);
  else if (q < PADS)
    img->f.w1[(q - 2 * H * RP) / FP][DIN + (q - 2 * H * RP) % FP] = bf(0.0f);
}

// grad[p] = sum over workgroups of partial[wg][p] in a fixed order (row 0
// first; the loads of eight rows are issued together); the loss slot
// becomes the mean squared error. With `theta` set, also one Adam step, and
// with `img` set, the updated weights' image.
__global__ void grad_reduce_kernel(const float *partial, uint32_t n_wg, float inv_n, float *grad,
                                   float *loss, float *theta, float *m, float *v, AdamArgs ad,
                                   MlpImage *img) {
  const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p > (uint32_t)MLP_NPARAMS) return;
  float s = 0.0f;
  uint32_t k = 0;
  for (; k + 8 <= n_wg; k += 8) {
    float t[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) t[j] = partial[(uint64_t)(k + j) * MLP_PSTRIDE + p];
#pragma unroll
    for (int j = 0; j < 8; ++j) s += t[j];
  }
  for (; k < n_wg; ++k) s += partial[(uint64_t)k * MLP_PSTRIDE + p];
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
    const float nt = theta[p] - ad.lr * (mm / ad.bc1) / (sqrtf(vv / ad.bc2) + ad.eps);
    theta[p] = nt;
    if (img) image_put(*img, p, nt);
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

hipError_t launch_mlp_pack(const float *theta, void *img, hipStream_t s) {
  constexpr uint32_t cells = MLP_NPARAMS + 2 * H * 8 + H * (40 - DIN);
  hipLaunchKernelGGL(mlp_pack_kernel, dim3((cells + 255) / 256), dim3(256), 0, s, theta,
                     (MlpImage *)img);
  return hipGetLastError();
}

hipError_t launch_mlp_grad(const void *img, const float *x, const float *z, const float *y,
                           uint64_t n, float *partial, hipStream_t s) {
  const size_t lds = sizeof(BwdLds);
  hipError_t e = allow_lds(mlp_grad_kernel, lds);
  if (e != hipSuccess) return e;
  const uint64_t blocks = (n + TS - 1) / TS;
  hipLaunchKernelGGL(mlp_grad_kernel, dim3((uint32_t)blocks), dim3(256), lds, s,
                     (const MlpImage *)img, x, z, y, n, 1.0f / (float)n, partial);
  return hipGetLastError();
}

hipError_t launch_grad_reduce(const float *partial, uint32_t n_wg, uint64_t n, float *grad,
                              float *loss, float *theta, float *m, float *v, const AdamArgs &ad,
                              void *img, hipStream_t s) {
  const uint32_t threads = 256, blocks = (MLP_NPARAMS + 1 + threads - 1) / threads;
  hipLaunchKernelGGL(grad_reduce_kernel, dim3(blocks), dim3(threads), 0, s, partial, n_wg,
                     1.0f / (float)n, grad, loss, theta, m, v, ad, (MlpImage *)img);
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

// the partial rows, then the weights' image
constexpr uint64_t NOALLOC_IMAGE_OFF = NOALLOC_ROWS * MLP_PSTRIDE;  // floats
static_assert(NOALLOC_IMAGE_OFF % 4 == 0 && MLP_IMAGE_BYTES % 4 == 0, "16-byte aligned image");
__device__ __align__(256) float scratch[NOALLOC_IMAGE_OFF + MLP_IMAGE_BYTES / 4];

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
  if (((uintptr_t)theta_dev & 15u) || (z_dev && ((uintptr_t)z_dev & 15u))) return MRIP_E_INVAL;
  float *part = nullptr;
  if (scratch_on_device(&part) != hipSuccess) return MRIP_E_HIP;
  hipStream_t s = (hipStream_t)hip_stream;
  const uint64_t rows = (n + TS - 1) / TS;
  float *img = part + NOALLOC_IMAGE_OFF;
  // every element of the image and every row the reduction reads is
  // written first, by the pack and the gradient kernels
  if (launch_mlp_pack(theta_dev, img, s) != hipSuccess) return MRIP_E_HIP;
  if (launch_mlp_grad(img, x_dev, z_dev, y_dev, n, part, s) != hipSuccess) return MRIP_E_HIP;
  AdamArgs none{};
  if (launch_grad_reduce(part, (uint32_t)rows, n, grad_dev, loss_dev, nullptr, nullptr, nullptr,
                         none, nullptr, s) != hipSuccess)
    return MRIP_E_HIP;
  return MRIP_OK;
}

