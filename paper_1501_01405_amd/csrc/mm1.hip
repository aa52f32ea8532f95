// M/M/1 replication engines (paper section 5.1, second model).
//
// Customer n carries the pair (A_n, S_n); with T the time in system of the
// previous customer, W_n = max(0, T - A_n), I_n = max(0, A_n - T),
// T_n = W_n + S_n. Each customer is the max-plus map f_n(T) = max(a_n,
// T + b_n) with a_n = S_n, b_n = S_n - A_n, and maps compose in closed form:
// (a2, b2) after (a1, b1) = (max(a2, a1 + b2), b1 + b2). That turns the
// sequential Lindley recursion into a prefix scan.
//
// WAVE mapping (one replication per wavefront): a segment of 16 lanes takes
// 16 P consecutive customers, P per lane from P/2 Philox blocks, composes
// the lane's maps, runs a 4-step DPP inclusive scan (row_shr 1, 2, 4, 8;
// a DPP row is exactly the segment) and applies the exclusive prefix to the
// carried T. A replication spans 4 / RPW segments; the carry passes through
// them in order as T <- max(a_tot, T + b_tot). Because every replication is
// always cut into the same segments and the carry visits them in the same
// order, the per-customer values do not depend on RPW or on the workgroup
// size; only the summation order of the means does.
//
// SIMT mapping (one replication per lane): the sequential recursion, one
// customer after the other, as the paper's thread-per-replication form.
#include "device.hpp"
#include "kernels.hpp"

namespace mrip {

namespace {

constexpr float kNegInf = -__builtin_huge_valf();

struct Rep {
  uint32_t dp, rep;
  uint64_t n;        // customers (0 = empty slot)
  float ca, cs;      // -(1/lambda) ln 2, -(1/mu) ln 2
  float lambda, mu;
  uint64_t out;      // output index
};

struct Sums {
  Kahan w, t, i;
};

struct Feat {
  float sa = 0.f, ss = 0.f, sw = 0.f, st = 0.f, si = 0.f, wmax = 0.f, tlast = 0.f;
  int zeros = 0;
};

__device__ __forceinline__ float pick4(int q, float v0, float v1, float v2, float v3) {
  return q == 0 ? v0 : q == 1 ? v1 : q == 2 ? v2 : v3;
}

// Customers per lane per chunk (P / 2 Philox blocks). A segment of 16 lanes
// takes 16 P consecutive customers; this fixes the association of the scan,
// so it is the same for every launch shape.
constexpr int MM1_P = 8;

// The variates of one chunk for this lane: P customers from P/2 blocks.
template <int P>
struct Draw {
  float A[P], S[P];
};

template <int RPW, int P>
__device__ __forceinline__ Draw<P> draw_chunk(uint64_t base, const Rep &d, uint32_t k0,
                                              uint32_t k1) {
  constexpr int S = 4 / RPW;
  constexpr int NB = P / 2;
  const int lane = threadIdx.x & 63;
  const int s = (lane >> 4) % S, l = lane & 15;
  const uint64_t kb = (base >> 1) + (uint64_t)(16 * s + l) * NB;
  Draw<P> r;
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    const Block4 b = philox((uint32_t)(kb + j), d.dp, d.rep, TAG_MM1, k0, k1);
    r.A[2 * j] = exp_variate(b.x, d.ca);
    r.S[2 * j] = exp_variate(b.y, d.cs);
    r.A[2 * j + 1] = exp_variate(b.z, d.ca);
    r.S[2 * j + 1] = exp_variate(b.w, d.cs);
  }
  return r;
}

// One chunk: every segment of the replication takes 16 P customers, whose
// variates are `dr`. FEAT accumulates the prefix features; TAIL masks
// customers >= n (only chunks that reach past some replication's end need
// it).
template <int RPW, int P, bool FEAT, bool TAIL>
__device__ __forceinline__ void wave_chunk(uint64_t base, const Draw<P> &dr, const Rep &d,
                                           uint64_t K, float &carry, Sums &acc, Feat &ft) {
  constexpr int S = 4 / RPW;  // segments per replication
  constexpr int NB = P / 2;   // Philox blocks per lane
  const int lane = threadIdx.x & 63;
  const int row = lane >> 4, l = lane & 15;
  const int q = row / S, s = row % S;
  const uint64_t kb = (base >> 1) + (uint64_t)(16 * s + l) * NB;
  const float *A = dr.A;
  const float *Sv = dr.S;

  // lane-local composition of the lane's P customers, in order
  float a = Sv[0];
  float bb = Sv[0] - A[0];
#pragma unroll
  for (int j = 1; j < P; ++j) {
    const float bj = Sv[j] - A[j];
    a = fmaxf(Sv[j], a + bj);
    bb = bb + bj;
  }

  // inclusive scan over the 16-lane segment
#define MRIP_SCAN_STEP(N)                              \
  {                                                    \
    const float as = row_shr<N>(a, kNegInf);           \
    const float bs = row_shr<N>(bb, 0.0f);             \
    a = fmaxf(a, as + bb);                             \
    bb = bs + bb;                                      \
  }
  MRIP_SCAN_STEP(1)
  MRIP_SCAN_STEP(2)
  MRIP_SCAN_STEP(4)
  MRIP_SCAN_STEP(8)
#undef MRIP_SCAN_STEP
  const float ea = row_shr<1>(a, kNegInf);
  const float eb = row_shr<1>(bb, 0.0f);

  // segment totals (lane 15 of every row) and the carry through the segments
  const float ta0 = readlane_f(a, 15), ta1 = readlane_f(a, 31);
  const float ta2 = readlane_f(a, 47), ta3 = readlane_f(a, 63);
  const float tb0 = readlane_f(bb, 15), tb1 = readlane_f(bb, 31);
  const float tb2 = readlane_f(bb, 47), tb3 = readlane_f(bb, 63);
  float tin = carry, cur = carry;
#pragma unroll
  for (int j = 0; j < S; ++j) {
    float ta, tb;
    if (RPW == 1) {
      ta = j == 0 ? ta0 : j == 1 ? ta1 : j == 2 ? ta2 : ta3;
      tb = j == 0 ? tb0 : j == 1 ? tb1 : j == 2 ? tb2 : tb3;
    } else {
      ta = pick4(q * S + j, ta0, ta1, ta2, ta3);
      tb = pick4(q * S + j, tb0, tb1, tb2, tb3);
    }
    tin = (j == s) ? cur : tin;
    cur = fmaxf(ta, cur + tb);
  }
  carry = cur;

  // the lane's customers, in order, from the system time before the first
  float T = fmaxf(ea, tin + eb);
  float sw = 0.0f, st = 0.0f, si = 0.0f;
  const uint64_t n0 = 2 * kb;
#pragma unroll
  for (int j = 0; j < P; ++j) {
    const float W = fmaxf(0.0f, T - A[j]);
    const float I = fmaxf(0.0f, A[j] - T);
    T = W + Sv[j];
    if (TAIL) {
      const bool v = n0 + j < d.n;
      sw += v ? W : 0.0f;
      st += v ? T : 0.0f;
      si += v ? I : 0.0f;
    } else {
      sw += W;
      st += T;
      si += I;
    }
    if (FEAT) {
      const bool f = n0 + j < K;
      ft.sa += f ? A[j] : 0.0f;
      ft.ss += f ? Sv[j] : 0.0f;
      ft.sw += f ? W : 0.0f;
      ft.st += f ? T : 0.0f;
      ft.si += f ? I : 0.0f;
      ft.zeros += (f && W == 0.0f);
      ft.wmax = fmaxf(ft.wmax, f ? W : 0.0f);
      if (n0 + j + 1 == K) ft.tlast = T;
    }
  }
  acc.w.add(sw);
  acc.t.add(st);
  acc.i.add(si);
}

// Runs the replications of one wavefront (RPW of them, one per lane group)
// to completion and writes their outputs.
template <int RPW>
__device__ void wave_group(const Rep &d, uint32_t k0, uint32_t k1, uint64_t K,
                           const Mm1Args &a) {
  constexpr int P = MM1_P;
  constexpr int S = 4 / RPW;
  constexpr int WIDTH = 16 * S;  // lanes per replication
  constexpr uint64_t CHUNK = 16u * P * S;
  const int lane = threadIdx.x & 63;

  // wave-uniform trip counts: chunks of the longest replication, and chunks
  // that are full for every non-empty replication of the wave
  uint32_t hi = (uint32_t)((d.n + CHUNK - 1) / CHUNK);
  uint32_t lo = d.n > 0 ? (uint32_t)(d.n / CHUNK) : 0xFFFFFFFFu;
  for (int off = WIDTH; off < 64; off <<= 1) {
    hi = max(hi, (uint32_t)__shfl_xor((int)hi, off, 64));
    lo = min(lo, (uint32_t)__shfl_xor((int)lo, off, 64));
  }
  const uint32_t chunks = (uint32_t)__builtin_amdgcn_readfirstlane((int)hi);
  const uint32_t full = min(chunks, (uint32_t)__builtin_amdgcn_readfirstlane((int)lo));
  const uint32_t fchunks = min(chunks, (uint32_t)((K + CHUNK - 1) / CHUNK));

  float carry = 0.0f;
  Sums acc;
  Feat ft;
  uint32_t c = 0;
#define MRIP_CHUNK(F, TL)                                                            \
  {                                                                                  \
    const Draw<P> cur = draw_chunk<RPW, P>((uint64_t)c * CHUNK, d, k0, k1);         \
    wave_chunk<RPW, P, F, TL>(c * CHUNK, cur, d, K, carry, acc, ft);                 \
  }
  for (; c < fchunks; ++c) MRIP_CHUNK(true, true)
  for (; c < full; ++c) MRIP_CHUNK(false, false)
  for (; c < chunks; ++c) MRIP_CHUNK(false, true)
#undef MRIP_CHUNK

  const float sw = group_sum_compensated(acc.w.value(), WIDTH);
  const float st = group_sum_compensated(acc.t.value(), WIDTH);
  const float si = group_sum_compensated(acc.i.value(), WIDTH);
  float f[10];
  if (K > 0) {
    const float kf = (float)K;
    f[0] = d.lambda / d.mu;
    f[1] = d.mu;
    f[2] = group_sum_compensated(ft.sa, WIDTH) / kf;
    f[3] = group_sum_compensated(ft.ss, WIDTH) / kf;
    f[4] = group_sum_compensated(ft.sw, WIDTH) / kf;
    f[5] = group_sum_compensated(ft.st, WIDTH) / kf;
    f[6] = (float)group_sum_i(ft.zeros, WIDTH) / kf;
    f[7] = group_max(ft.wmax, WIDTH);
    f[8] = group_sum_compensated(ft.si, WIDTH) / kf;
    f[9] = group_sum_compensated(ft.tlast, WIDTH);
  }
  if ((lane % WIDTH) == 0 && d.n > 0) {
    const float nf = (float)d.n;
    a.mean_w[d.out] = sw / nf;
    a.mean_t[d.out] = st / nf;
    a.mean_i[d.out] = si / nf;
    if (K > 0) {
#pragma unroll
      for (int j = 0; j < 10; ++j) a.features[d.out * 10 + j] = f[j];
    }
  }
}

__device__ __forceinline__ float neg_mean_ln2(float rate) {
  return (float)(-(1.0 / (double)rate) * 0.69314718055994530942);
}

__device__ __forceinline__ Rep uniform_rep(const Mm1Args &a, uint64_t r, float ca, float cs) {
  Rep d;
  d.dp = 0;
  d.rep = (uint32_t)r;
  d.n = r < a.n_reps ? a.customers : 0;
  d.ca = ca;
  d.cs = cs;
  d.lambda = a.lambda;
  d.mu = a.mu;
  d.out = r;
  return d;
}

__device__ __forceinline__ Rep item_rep(const Mm1Args &a, uint64_t slot, uint64_t n_items) {
  Rep d;
  if (slot < n_items) {
    const uint32_t i = a.items.order[slot];
    d.dp = a.items.dp[i];
    d.rep = a.items.rep[i];
    d.n = a.items.customers[i];
    d.lambda = a.items.lambda[i];
    d.mu = a.items.mu[i];
    d.out = i;
  } else {
    d.dp = d.rep = 0;
    d.n = 0;
    d.lambda = d.mu = 1.0f;
    d.out = 0;
  }
  d.ca = neg_mean_ln2(d.lambda);
  d.cs = neg_mean_ln2(d.mu);
  return d;
}

template <int RPW>
__global__ void mm1_wave_kernel(Mm1Args a, float ca, float cs) {
  constexpr int S = 4 / RPW;
  const int lane = threadIdx.x & 63;
  const uint64_t wave = (uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const int q = (lane >> 4) / S;
  const uint64_t r = wave * RPW + q;
  const uint32_t k0 = (uint32_t)a.seed, k1 = (uint32_t)(a.seed >> 32);
  if (wave * RPW >= a.n_reps) return;  // whole wave idle (wave-uniform)
  wave_group<RPW>(uniform_rep(a, r, ca, cs), k0, k1, a.feature_prefix, a);
}

// Persistent plan kernel: every wave pops units of RPW items (longest first)
// until the queue is empty; the exit test is wave-uniform, so the grid always
// drains.
template <int RPW>
__global__ void mm1_plan_kernel(Mm1Args a, uint64_t n_items) {
  constexpr int S = 4 / RPW;
  const int lane = threadIdx.x & 63;
  const int q = (lane >> 4) / S;
  const uint32_t k0 = (uint32_t)a.seed, k1 = (uint32_t)(a.seed >> 32);
  const uint64_t n_units = (n_items + RPW - 1) / RPW;
  for (;;) {
    uint32_t unit = 0;
    if (lane == 0) unit = atomicAdd(a.queue_head, 1u);
    unit = (uint32_t)__builtin_amdgcn_readfirstlane((int)__shfl((int)unit, 0, 64));
    if (unit >= n_units) break;
    wave_group<RPW>(item_rep(a, (uint64_t)unit * RPW + q, n_items), k0, k1, a.feature_prefix,
                    a);
  }
}

__global__ void mm1_simt_kernel(Mm1Args a, float ca, float cs) {
  const uint64_t r = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= a.n_reps) return;
  const uint32_t k0 = (uint32_t)a.seed, k1 = (uint32_t)(a.seed >> 32);
  const uint64_t N = a.customers, K = a.feature_prefix;
  float tprev = 0.0f;
  Kahan sw, st, si;
  Feat ft;
  for (uint64_t k = 0; 2 * k < N; ++k) {
    const Block4 b = philox((uint32_t)k, 0u, (uint32_t)r, TAG_MM1, k0, k1);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const uint64_t n = 2 * k + h;
      if (n >= N) break;
      const float A = exp_variate(h ? b.z : b.x, ca);
      const float Sv = exp_variate(h ? b.w : b.y, cs);
      const float W = fmaxf(0.0f, tprev - A);
      const float I = fmaxf(0.0f, A - tprev);
      const float T = W + Sv;
      sw.add(W);
      st.add(T);
      si.add(I);
      if (n < K) {
        ft.sa += A;
        ft.ss += Sv;
        ft.sw += W;
        ft.st += T;
        ft.si += I;
        ft.zeros += (W == 0.0f);
        ft.wmax = fmaxf(ft.wmax, W);
        if (n + 1 == K) ft.tlast = T;
      }
      tprev = T;
    }
  }
  const float nf = (float)N;
  a.mean_w[r] = sw.value() / nf;
  a.mean_t[r] = st.value() / nf;
  a.mean_i[r] = si.value() / nf;
  if (K > 0) {
    const float kf = (float)K;
    float *f = a.features + r * 10;
    f[0] = a.lambda / a.mu;
    f[1] = a.mu;
    f[2] = ft.sa / kf;
    f[3] = ft.ss / kf;
    f[4] = ft.sw / kf;
    f[5] = ft.st / kf;
    f[6] = (float)ft.zeros / kf;
    f[7] = ft.wmax;
    f[8] = ft.si / kf;
    f[9] = ft.tlast;
  }
}

__global__ void zero_u32_kernel(uint32_t *p, uint32_t n) {
  for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0u;
}

float host_neg_mean_ln2(float rate) {
  return (float)(-(1.0 / (double)rate) * 0.69314718055994530942);
}

}  // namespace

hipError_t launch_mm1_wave(const Mm1Args &a, uint32_t rpw, uint32_t wg, hipStream_t s) {
  const uint64_t waves = (a.n_reps + rpw - 1) / rpw;
  const uint32_t wpb = wg / 64;
  const uint64_t blocks = (waves + wpb - 1) / wpb;
  const float ca = host_neg_mean_ln2(a.lambda), cs = host_neg_mean_ln2(a.mu);
  if (rpw == 1) hipLaunchKernelGGL(mm1_wave_kernel<1>, dim3((uint32_t)blocks), dim3(wg), 0, s, a, ca, cs);
  else if (rpw == 2) hipLaunchKernelGGL(mm1_wave_kernel<2>, dim3((uint32_t)blocks), dim3(wg), 0, s, a, ca, cs);
  else hipLaunchKernelGGL(mm1_wave_kernel<4>, dim3((uint32_t)blocks), dim3(wg), 0, s, a, ca, cs);
  return hipGetLastError();
}

hipError_t launch_mm1_simt(const Mm1Args &a, hipStream_t s) {
  const uint32_t wg = 64;
  const uint64_t blocks = (a.n_reps + wg - 1) / wg;
  const float ca = host_neg_mean_ln2(a.lambda), cs = host_neg_mean_ln2(a.mu);
  hipLaunchKernelGGL(mm1_simt_kernel, dim3((uint32_t)blocks), dim3(wg), 0, s, a, ca, cs);
  return hipGetLastError();
}

hipError_t launch_mm1_plan(const Mm1Args &a, uint64_t n_items, uint32_t rpw, uint32_t wg,
                           hipStream_t s) {
  int dev = 0, cus = 0, per_cu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  const void *fn = rpw == 1 ? (const void *)mm1_plan_kernel<1>
                 : rpw == 2 ? (const void *)mm1_plan_kernel<2>
                            : (const void *)mm1_plan_kernel<4>;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, (int)wg, 0);
  if (e != hipSuccess) return e;
  if (per_cu < 1) per_cu = 1;
  // never more waves than work units
  const uint64_t units = (n_items + rpw - 1) / rpw;
  uint64_t blocks = (uint64_t)cus * (uint64_t)per_cu;
  const uint64_t need = (units + wg / 64 - 1) / (wg / 64);
  if (blocks > need) blocks = need;
  if (blocks < 1) blocks = 1;
  if (rpw == 1) hipLaunchKernelGGL(mm1_plan_kernel<1>, dim3((uint32_t)blocks), dim3(wg), 0, s, a, n_items);
  else if (rpw == 2) hipLaunchKernelGGL(mm1_plan_kernel<2>, dim3((uint32_t)blocks), dim3(wg), 0, s, a, n_items);
  else hipLaunchKernelGGL(mm1_plan_kernel<4>, dim3((uint32_t)blocks), dim3(wg), 0, s, a, n_items);
  return hipGetLastError();
}

hipError_t launch_zero_u32(uint32_t *p, uint32_t n, hipStream_t s) {
  hipLaunchKernelGGL(zero_u32_kernel, dim3(1), dim3(64), 0, s, p, n);
  return hipGetLastError();
}

}  // namespace mrip
