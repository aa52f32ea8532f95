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
// size; only the summation order of the means does. The wavefront engines
// (and the taus88 one) count time in the negative unit -(1/mu) ln 2, in
// which a service time is log2 u itself; there every maximum above is a
// minimum (`later`), and results are scaled back when written.
//
// SIMT mapping (one replication per lane): the sequential recursion, one
// customer after the other, as the paper's thread-per-replication form.
//
// On taus88 streams customer n takes outputs 2n (A) and 2n+1 (S) of the
// replication's stream, a sequential generator: the wavefront engine gives
// every lane a contiguous run of customers instead (mm1_taus_kernel: a
// jump of one table per set bit of the lane's index, two passes over its
// run); a SIMT lane reads the stream in order.
#include <hip/hip_ext.h>

#include <algorithm>
#include <cmath>
#include <type_traits>

#include "device.hpp"
#include "kernels.hpp"
#include "reduce_dev.hpp"
#include "taus.hpp"

namespace mrip {

namespace {

// The later of two times counted in the wavefront engines' negative unit,
// and the value there of a time before all others (the constant part of
// the identity map).
__device__ __forceinline__ float later(float a, float b) { return fminf(a, b); }
constexpr float kBeforeAll = __builtin_huge_valf();

struct Rep {
  uint32_t dp, rep;
  uint64_t n;        // customers (0 = empty slot)
  float ca, cs;      // -(1/lambda) ln 2, -(1/mu) ln 2
  // The wavefront engines count time in units of cs (negative): a service
  // time is then S = log2 u exactly and an interarrival time A = qa log2 u
  // with qa = ca / cs, one multiplication per customer fewer. The unit's
  // sign turns every maximum of times into a minimum of their values
  // (`later`); sums, the largest wait and the T-weighted controls are
  // scaled back by cs when written.
  float qa;
  float lambda, mu;
  float ea, es;      // means of the A and S variates as drawn (control centring)
  uint64_t out;      // output index
};

// Sums of T, S and I, and of the four martingale controls over customers
// n >= K (FT forms only): S_n - E S, A_n - E A, and both weighted by T_{n-1}.
// The waits follow as W_n = T_n - S_n: their sum is that of T less that of S.
struct Sums {
  Kahan t, s, i;
  Kahan c[4];
};

// A lane's sum of waits from its sums of T and S.
__device__ __forceinline__ float wait_sum(const Sums &x) {
  return (x.t.sum - x.s.sum) - (x.t.comp - x.s.comp);
}

// Prefix features, and the four controls over the prefix customers (n < K:
// a lane holds about K / 64 of them, plain fp32 sums suffice).
struct Feat {
  float sa = 0.f, ss = 0.f, sw = 0.f, st = 0.f, si = 0.f, wmax = 0.f, tlast = 0.f;
  int zeros = 0;
  float pc[4] = {0.f, 0.f, 0.f, 0.f};
};

__device__ __forceinline__ float pick4(int q, float v0, float v1, float v2, float v3) {
  return q == 0 ? v0 : q == 1 ? v1 : q == 2 ? v2 : v3;
}

// Customers per lane per chunk (P / 2 Philox blocks). A segment of 16 lanes
// takes 16 P consecutive customers; this fixes the association of the scan,
// so it is the same for every launch shape.
constexpr int MM1_P = 16;

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
    r.A[2 * j] = d.qa * log2_u01(b.x);
    r.S[2 * j] = log2_u01(b.y);
    r.A[2 * j + 1] = d.qa * log2_u01(b.z);
    r.S[2 * j + 1] = log2_u01(b.w);
  }
  return r;
}

// Draw sources for wave_group: chunk c is requested in order c = 0, 1, ...
struct PhiloxSource {
  uint32_t k0, k1;
  template <int RPW, int P>
  __device__ __forceinline__ Draw<P> next(uint64_t base, const Rep &d) {
    return draw_chunk<RPW, P>(base, d, k0, k1);
  }
};

// The scanned maps of one chunk: this lane's exclusive prefix (ea, eb), the
// map of its first P / 2 customers (ha, hb) and the four segment totals.
struct ChunkScan {
  float ea, eb, ha, hb;
  float ta[4], tb[4];
};

// Compose this lane's P customers (its two halves side by side, in order
// within each, then the second half after the first), then scan the
// 16-lane segment.
template <int P>
__device__ __forceinline__ ChunkScan compose_scan(const Draw<P> &dr) {
  constexpr int H = P / 2;
  float a0 = dr.S[0], b0 = dr.S[0] - dr.A[0];
  float a1 = dr.S[H], b1 = dr.S[H] - dr.A[H];
#pragma unroll
  for (int j = 1; j < H; ++j) {
    const float c0 = dr.S[j] - dr.A[j];
    a0 = later(dr.S[j], a0 + c0);
    b0 = b0 + c0;
    const float c1 = dr.S[H + j] - dr.A[H + j];
    a1 = later(dr.S[H + j], a1 + c1);
    b1 = b1 + c1;
  }
  float a = later(a1, a0 + b1);
  float bb = b0 + b1;
#define MRIP_SCAN_STEP(N)                              \
  {                                                    \
    const float as = row_shr<N>(a, kBeforeAll);        \
    const float bs = row_shr<N>(bb, 0.0f);             \
    a = later(a, as + bb);                             \
    bb = bs + bb;                                      \
  }
  MRIP_SCAN_STEP(1)
  MRIP_SCAN_STEP(2)
  MRIP_SCAN_STEP(4)
  MRIP_SCAN_STEP(8)
#undef MRIP_SCAN_STEP
  ChunkScan r;
  r.ha = a0;
  r.hb = b0;
  r.ea = row_shr<1>(a, kBeforeAll);
  r.eb = row_shr<1>(bb, 0.0f);
  r.ta[0] = readlane_f(a, 15);
  r.ta[1] = readlane_f(a, 31);
  r.ta[2] = readlane_f(a, 47);
  r.ta[3] = readlane_f(a, 63);
  r.tb[0] = readlane_f(bb, 15);
  r.tb[1] = readlane_f(bb, 31);
  r.tb[2] = readlane_f(bb, 47);
  r.tb[3] = readlane_f(bb, 63);
  return r;
}

// Pass the carry through the replication's segments in order: returns the
// carry after the chunk and sets `tin`, the carry into this lane's segment.
template <int RPW>
__device__ __forceinline__ float carry_through(const ChunkScan &cs, float carry, float &tin) {
  constexpr int S = 4 / RPW;
  const int row = (threadIdx.x & 63) >> 4;
  const int q = row / S, s = row % S;
  float cur = carry;
  tin = carry;
#pragma unroll
  for (int j = 0; j < S; ++j) {
    float ta, tb;
    if (RPW == 1) {
      ta = cs.ta[j];
      tb = cs.tb[j];
    } else {
      ta = pick4(q * S + j, cs.ta[0], cs.ta[1], cs.ta[2], cs.ta[3]);
      tb = pick4(q * S + j, cs.tb[0], cs.tb[1], cs.tb[2], cs.tb[3]);
    }
    tin = (j == s) ? cur : tin;
    cur = later(ta, cur + tb);
  }
  return cur;
}

// The lane's P customers in order, from the system time T before the first
// (times in the engines' unit, where the later of two is `later`). Each
// customer applies its map: x = T + b with b = S - A, T <- later(x, S)
// (Lindley's W = max(0, T - A), T = W + S with one rounding less), and its
// idle time is I = T - x, exactly 0 whenever the server is busy. The lane
// sums T, S and I (TAIL: only customers < n); the waits follow as T - S.
// With FT: the prefix features and prefix controls (customers < K, FEAT
// chunks only) and the partial sums of the four controls after the prefix
// (customers >= K). A_n and S_n are drawn independently of T_{n-1}, the
// system time the lane holds when it reaches customer n, so every control
// term has mean zero given the past.
template <int P, bool FEAT, bool TAIL, bool FT>
__device__ __forceinline__ void apply_lane(float T0, const ChunkScan &cs, const Draw<P> &dr,
                                           uint64_t n0, uint64_t n, uint64_t K, float unit,
                                           float ea, float es, float &st, float &ss, float &si,
                                           Feat &ft, float (&cl)[4]) {
  constexpr int H = P / 2;
  // the two halves side by side, the second from later(ha, T0 + hb), the
  // system time the first half's map gives; each half sums on its own
  float Th[2] = {T0, later(cs.ha, T0 + cs.hb)};
  const float Ts[2] = {Th[0], Th[1]};  // the halves' starts
  float sth[2] = {0.0f, 0.0f}, ssh[2] = {0.0f, 0.0f}, sih[2] = {0.0f, 0.0f};
  if (FT) cl[0] = cl[1] = cl[2] = cl[3] = 0.0f;
  // FT chunks with every customer counted (no feature prefix, no tail):
  // the controls from raw sums, sum A, sum T_{n-1} S and sum T_{n-1} A,
  // centred once per chunk (three operations per customer instead of six)
  constexpr bool RAW = FT && !FEAT && !TAIL;
  float qa = 0.0f, qts = 0.0f, qta = 0.0f;
#pragma unroll
  for (int j = 0; j < P; ++j) {
    const int h = j >= H;
    float &T = Th[h];
    if (FT) {
      bool v = true;
      if (FEAT) v = n0 + j >= K;
      if (TAIL) v = v && n0 + j < n;
      // the centred variates in time (T-weighted sums stay in the unit)
      const float da = __builtin_fmaf(unit, dr.A[j], -ea), ds = __builtin_fmaf(unit, dr.S[j], -es);
      if (FEAT) {  // customers < K <= n: the prefix four
        const bool p = n0 + j < K;
        ft.pc[0] += p ? ds : 0.0f;
        ft.pc[1] += p ? da : 0.0f;
        ft.pc[2] = p ? __builtin_fmaf(T, ds, ft.pc[2]) : ft.pc[2];
        ft.pc[3] = p ? __builtin_fmaf(T, da, ft.pc[3]) : ft.pc[3];
      }
      if (FEAT || TAIL) {
        cl[0] += v ? ds : 0.0f;
        cl[1] += v ? da : 0.0f;
        cl[2] = v ? __builtin_fmaf(T, ds, cl[2]) : cl[2];
        cl[3] = v ? __builtin_fmaf(T, da, cl[3]) : cl[3];
      } else {
        qa += dr.A[j];
        qts = __builtin_fmaf(T, dr.S[j], qts);
        qta = __builtin_fmaf(T, dr.A[j], qta);
      }
    }
    if (FEAT) {  // the prefix features, from their definitions
      const bool f = n0 + j < K;
      // I = max(0, A - T) = W - (T - A) exactly: A - T = -(T - A) in IEEE
      // arithmetic, and W is either 0 or T - A
      const float dlt = T - dr.A[j];
      const float W = later(0.0f, dlt);
      ft.sa += f ? dr.A[j] : 0.0f;
      ft.ss += f ? dr.S[j] : 0.0f;
      ft.sw += f ? W : 0.0f;
      ft.si += f ? W - dlt : 0.0f;
      ft.zeros += (f && W == 0.0f);
      ft.wmax = later(ft.wmax, f ? W : 0.0f);
    }
    const float x = T + (dr.S[j] - dr.A[j]);
    T = later(x, dr.S[j]);
    const float I = T - x;
    if (TAIL) {
      const bool v = n0 + j < n;
      sth[h] += v ? T : 0.0f;
      ssh[h] += v ? dr.S[j] : 0.0f;
      sih[h] += v ? I : 0.0f;
    } else {
      sth[h] += T;
      ssh[h] += dr.S[j];
      sih[h] += I;
    }
    if (FEAT) {
      const bool f = n0 + j < K;
      ft.st += f ? T : 0.0f;
      if (n0 + j + 1 == K) ft.tlast = T;
    }
  }
  st = sth[0] + sth[1];
  ss = ssh[0] + ssh[1];
  si = sih[0] + sih[1];
  if (RAW) {
    // sum of T_{n-1} over the lane: each half's start, plus its T's but
    // the last
    const float tp = (Ts[0] + (sth[0] - Th[0])) + (Ts[1] + (sth[1] - Th[1]));
    cl[0] = __builtin_fmaf(unit, ss, -(float)P * es);
    cl[1] = __builtin_fmaf(unit, qa, -(float)P * ea);
    cl[2] = __builtin_fmaf(unit, qts, -es * tp);
    cl[3] = __builtin_fmaf(unit, qta, -ea * tp);
  }
}

template <int RPW, int P>
__device__ __forceinline__ uint64_t lane_first_customer(uint64_t base) {
  constexpr int S = 4 / RPW;
  const int lane = threadIdx.x & 63;
  const int s = (lane >> 4) % S, l = lane & 15;
  return base + (uint64_t)(16 * s + l) * P;
}

// One chunk: every segment of the replication takes 16 P customers, whose
// variates are `dr`. FEAT accumulates the prefix features; TAIL masks
// customers >= n (only chunks that reach past some replication's end need
// it); FT adds the controls.
template <int RPW, int P, bool FEAT, bool TAIL, bool FT>
__device__ __forceinline__ void wave_chunk(uint64_t base, const Draw<P> &dr, const Rep &d,
                                           uint64_t K, float &carry, Sums &acc, Feat &ft) {
  const ChunkScan cs = compose_scan<P>(dr);
  float tin;
  carry = carry_through<RPW>(cs, carry, tin);
  float st, ss, si, cl[4];
  apply_lane<P, FEAT, TAIL, FT>(later(cs.ea, tin + cs.eb), cs, dr, lane_first_customer<RPW, P>(base),
                                d.n, K, d.cs, d.ea, d.es, st, ss, si, ft, cl);
  acc.t.add(st);
  acc.s.add(ss);
  acc.i.add(si);
  if (FT) {
#pragma unroll
    for (int k = 0; k < 4; ++k) acc.c[k].add(cl[k]);
  }
}

// Fix-up chunk of a split replication: the same customers from two carries
// (the true one and the speculative one the part started from); adds the
// difference of their sums (S and the two unweighted controls do not depend
// on the carry). Fix-up chunks lie after the feature prefix, so with FT
// every customer counts for the controls.
template <int P, bool TAIL, bool FT>
__device__ __forceinline__ void fixup_chunk(uint64_t base, const Draw<P> &dr, const Rep &d,
                                            float &c_true, float &c_spec, Sums &acc) {
  const ChunkScan cs = compose_scan<P>(dr);
  float tin_t, tin_s;
  c_true = carry_through<1>(cs, c_true, tin_t);
  c_spec = carry_through<1>(cs, c_spec, tin_s);
  const uint64_t n0 = lane_first_customer<1, P>(base);
  Feat none;
  float tt, st_, it, ts, ss_, is, clt[4], cls[4];
  apply_lane<P, false, TAIL, FT>(later(cs.ea, tin_t + cs.eb), cs, dr, n0, d.n, 0, d.cs, d.ea, d.es, tt, st_,
                                 it, none, clt);
  apply_lane<P, false, TAIL, FT>(later(cs.ea, tin_s + cs.eb), cs, dr, n0, d.n, 0, d.cs, d.ea, d.es, ts, ss_,
                                 is, none, cls);
  acc.t.add(tt - ts);
  acc.i.add(it - is);
  if (FT) {
    acc.c[2].add(clt[2] - cls[2]);
    acc.c[3].add(clt[3] - cls[3]);
  }
}

// Runs the replications of one wavefront (RPW of them, one per lane group)
// to completion and writes their outputs. FT: K > 0, with the prefix
// features and the controls; the form without them (K = 0) carries none of
// their registers.
template <int RPW, bool FT, class Src>
__device__ void wave_group(const Rep &d, Src &src, uint64_t K, const Mm1Args &a) {
  constexpr int P = MM1_P;
  constexpr int S = 4 / RPW;
  constexpr int WIDTH = 16 * S;  // lanes per replication
  constexpr uint64_t CHUNK = 16u * P * S;
  const int lane = threadIdx.x & 63;
  if (!FT) K = 0;

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
    const Draw<P> cur = src.template next<RPW, P>((uint64_t)c * CHUNK, d);          \
    wave_chunk<RPW, P, F, TL, FT>(c * CHUNK, cur, d, K, carry, acc, ft);             \
  }
  if (FT)
    for (; c < fchunks; ++c) MRIP_CHUNK(FT, true)
  for (; c < full; ++c) MRIP_CHUNK(false, false)
  for (; c < chunks; ++c) MRIP_CHUNK(false, true)
#undef MRIP_CHUNK

  const float sw = group_sum_compensated(wait_sum(acc), WIDTH);
  const float st = group_sum_compensated(acc.t.value(), WIDTH);
  const float si = group_sum_compensated(acc.i.value(), WIDTH);
  float f[10], cl[8];
  if (FT) {
    const float kf = (float)K;
    f[0] = d.lambda / d.mu;
    f[1] = d.mu;
    f[2] = group_sum_compensated(ft.sa, WIDTH) * d.cs / kf;
    f[3] = group_sum_compensated(ft.ss, WIDTH) * d.cs / kf;
    f[4] = group_sum_compensated(ft.sw, WIDTH) * d.cs / kf;
    f[5] = group_sum_compensated(ft.st, WIDTH) * d.cs / kf;
    f[6] = (float)group_sum_i(ft.zeros, WIDTH) / kf;
    f[7] = group_max(-ft.wmax, WIDTH) * -d.cs;  // the latest of the waits
    f[8] = group_sum_compensated(ft.si, WIDTH) * d.cs / kf;
    f[9] = group_sum_compensated(ft.tlast, WIDTH) * d.cs;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      cl[k] = group_sum_compensated(acc.c[k].value(), WIDTH);
      cl[4 + k] = group_sum_compensated(ft.pc[k], WIDTH);
    }
    // the T-weighted controls, from the unit
    cl[2] *= d.cs;
    cl[3] *= d.cs;
    cl[6] *= d.cs;
    cl[7] *= d.cs;
  }
  if ((lane % WIDTH) == 0 && d.n > 0) {
    const float nf = (float)d.n;
    a.mean_w[d.out] = sw * d.cs / nf;
    a.mean_t[d.out] = st * d.cs / nf;
    a.mean_i[d.out] = si * d.cs / nf;
    if (FT) {
#pragma unroll
      for (int j = 0; j < 10; ++j) a.features[d.out * 10 + j] = f[j];
#pragma unroll
      for (int k = 0; k < 8; ++k) a.controls[d.out * 8 + k] = cl[k];
    }
  }
}

__device__ __forceinline__ float neg_mean_ln2(float rate) {
  return (float)(-(1.0 / (double)rate) * 0.69314718055994530942);
}

// Mean of the exponential variate of `rate` as defined (fp32 scale
// (float)(1 / rate) times the mean of -ln u over the 24-bit grid of u), in
// fp32: the centring constant of the controls.
__device__ __forceinline__ float variate_mean(float rate, double log_grid_mean) {
  return (float)((double)(float)(1.0 / (double)rate) * log_grid_mean);
}

__device__ __forceinline__ Rep uniform_rep(const Mm1Args &a, uint64_t r, float ca, float cs) {
  Rep d;
  d.dp = 0;
  d.rep = (uint32_t)r;
  d.n = r < a.n_reps ? a.customers : 0;
  d.ca = ca;
  d.cs = cs;
  d.qa = ca / cs;
  d.lambda = a.lambda;
  d.mu = a.mu;
  d.ea = a.ea;
  d.es = a.es;
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
  d.qa = d.ca / d.cs;
  d.ea = d.es = 0.0f;
  if (a.feature_prefix > 0) {
    d.ea = variate_mean(d.lambda, a.log_grid_mean);
    d.es = variate_mean(d.mu, a.log_grid_mean);
  }
  return d;
}

// FT kernels (features and controls) launch at most 256 threads per
// workgroup, which leaves them 256 VGPRs instead of 128.
template <bool FT>
constexpr int ft_max_wg() {
  return FT ? 256 : 1024;
}

template <int RPW, bool FT>
__global__ __launch_bounds__(ft_max_wg<FT>()) void mm1_wave_kernel(Mm1Args a, float ca, float cs) {
  constexpr int S = 4 / RPW;
  const int lane = threadIdx.x & 63;
  const uint64_t wave = (uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const int q = (lane >> 4) / S;
  const uint64_t r = wave * RPW + q;
  const uint32_t k0 = (uint32_t)a.seed, k1 = (uint32_t)(a.seed >> 32);
  if (wave * RPW >= a.n_reps) return;  // whole wave idle (wave-uniform)
  const Rep d = uniform_rep(a, r, ca, cs);
  PhiloxSource src{k0, k1};
  wave_group<RPW, FT>(d, src, a.feature_prefix, a);
}

// taus88 streams, WAVE mapping. The LPR lanes of a replication (16 or 32 of
// a wavefront, or 1, 2 or 4 whole wavefronts) each take a contiguous run of
// B = ceil(N / LPR) customers, so a lane reads its run of the stream in
// order after one jump. Pass 1 composes the run's max-plus map; the maps
// are scanned in lane order (shuffles inside a wavefront, the wavefronts'
// totals through LDS), which gives each lane the system time before its
// run; pass 2 re-reads the run from the saved state and applies Lindley's
// recursion. No speculation: the scan is exact max-plus composition.
template <int LPR>
__global__ __launch_bounds__(256) void mm1_taus_kernel(Mm1Args a, float ca, float cs) {
  constexpr int G = LPR < 64 ? LPR : 64;  // lanes of one replication inside a wavefront
  constexpr int RPB = 256 / LPR;          // replications per workgroup
  __shared__ float sh_a[4], sh_b[4];      // wavefront totals of the scan
  __shared__ float sh_f[4][19];           // per-wavefront partial sums
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int j = tid % LPR;                // lane within the replication
  const int g = lane % G;                 // lane within its group of one wavefront
  const uint64_t r = (uint64_t)blockIdx.x * RPB + tid / LPR;
  const uint64_t N = r < a.n_reps ? a.customers : 0, K = a.feature_prefix;
  const uint64_t B = (a.customers + LPR - 1) / LPR;
  const uint64_t n0 = min(N, (uint64_t)j * B), n1 = min(N, n0 + B);
  const uint32_t k0 = (uint32_t)a.seed, k1 = (uint32_t)(a.seed >> 32);
  Taus t0 = taus_seed(TAG_MM1, 0u, (uint32_t)r, k0, k1);
  // to the lane's run, 2 j B outputs in: one table per set bit of j (a lane
  // past the replication's end has no customers, and its place is unused)
  {
    const uint32_t *tb = a.taus_run + (uint64_t)taus_run_base(LPR) * TAUS_COLS;
#pragma unroll
    for (int i = 0; (1 << i) < LPR; ++i)
      if ((j >> i) & 1) taus_jump(t0, tb + (uint64_t)i * TAUS_COLS);
  }

  // Time is counted in the unit cs < 0, as in the wavefront engines: a
  // service time is log2 u, an interarrival time qa log2 u, and maxima of
  // times are minima of their values (`later`).
  const float qa = ca / cs;
  const uint32_t m = (uint32_t)(n1 - n0);  // customers of this lane's run

  // pass 1: the run's composite map T -> later(ma, T + mb)
  float ma = kBeforeAll, mb = 0.0f;
  Taus t = t0;
  {
    auto step = [&]() {
      const float A = qa * log2_u01(taus_next(t));
      const float S = log2_u01(taus_next(t));
      const float bj = S - A;
      ma = later(S, ma + bj);
      mb = mb + bj;
    };
    uint32_t i = 0;
    for (; i + 4 <= m; i += 4) {
      step();
      step();
      step();
      step();
    }
    for (; i < m; ++i) step();
  }
  // inclusive scan in lane order (earlier runs first)
#pragma unroll
  for (int o = 1; o < G; o <<= 1) {
    const float pa = __shfl_up(ma, o, G), pb = __shfl_up(mb, o, G);
    if (g >= o) {
      ma = later(ma, pa + mb);
      mb = pb + mb;
    }
  }
  float ea = __shfl_up(ma, 1, G), eb = __shfl_up(mb, 1, G);
  if (g == 0) {
    ea = kBeforeAll;
    eb = 0.0f;
  }
  // system time entering this wavefront's part of the replication
  float carry = 0.0f;
  if (LPR > 64) {
    if (lane == 63) {
      sh_a[wave] = ma;
      sh_b[wave] = mb;
    }
    __syncthreads();
    for (int w = wave - j / 64; w < wave; ++w) carry = later(sh_a[w], carry + sh_b[w]);
  }
  float T = later(ea, carry + eb);

  // pass 2: Lindley's recursion over the run, from the saved stream state,
  // in the map form of the wavefront engines: x = T + S - A, T <- later(x,
  // S), I = T - x; sums of T, S and I, the waits as their difference
  t = t0;
  Kahan kt, ks, ki;
  Feat ft;
  uint32_t i = 0;
  const uint32_t mf = (uint32_t)(min(n1, max(n0, K)) - n0);  // customers of the feature prefix
  for (; i < mf; ++i) {  // the prefix: features and the prefix controls
    const float A = qa * log2_u01(taus_next(t));
    const float S = log2_u01(taus_next(t));
    const float ds = __builtin_fmaf(cs, S, -a.es), da = __builtin_fmaf(cs, A, -a.ea);
    ft.pc[0] += ds;
    ft.pc[1] += da;
    ft.pc[2] = __builtin_fmaf(T, ds, ft.pc[2]);
    ft.pc[3] = __builtin_fmaf(T, da, ft.pc[3]);
    const float dlt = T - A;
    const float W = later(0.0f, dlt);
    const float x = T + (S - A);
    T = later(x, S);
    kt.add(T);
    ks.add(S);
    ki.add(T - x);
    ft.sa += A;
    ft.ss += S;
    ft.sw += W;
    ft.st += T;
    ft.si += W - dlt;
    ft.zeros += (W == 0.0f);
    ft.wmax = later(ft.wmax, W);
    if (n0 + i + 1 == K) ft.tlast = T;
  }
  // after the prefix (every customer from here on has n >= K): with K > 0,
  // also the four controls, weighted by T_{n-1} where they are; plain fp32
  // sums over 8 customers, then one compensated add each
  Kahan kc[4];
  auto rest = [&](auto ctl_tag) {
    constexpr bool CTL = decltype(ctl_tag)::value;
    while (i < m) {
      const uint32_t e = min(m, i + 8);
      float st = 0.0f, ss = 0.0f, si = 0.0f, c0 = 0.0f, c1 = 0.0f, c2 = 0.0f, c3 = 0.0f;
      auto step = [&]() {
        const float A = qa * log2_u01(taus_next(t));
        const float S = log2_u01(taus_next(t));
        if (CTL) {
          const float ds = __builtin_fmaf(cs, S, -a.es), da = __builtin_fmaf(cs, A, -a.ea);
          c0 += ds;
          c1 += da;
          c2 = __builtin_fmaf(T, ds, c2);
          c3 = __builtin_fmaf(T, da, c3);
        }
        const float x = T + (S - A);
        T = later(x, S);
        st += T;
        ss += S;
        si += T - x;
      };
      if (e - i == 8) {
#pragma unroll
        for (int k = 0; k < 8; ++k) step();
        i = e;
      } else {
        for (; i < e; ++i) step();
      }
      kt.add(st);
      ks.add(ss);
      ki.add(si);
      if (CTL) {
        kc[0].add(c0);
        kc[1].add(c1);
        kc[2].add(c2);
        kc[3].add(c3);
      }
    }
  };
  if (K > 0)
    rest(std::true_type{});
  else
    rest(std::false_type{});

  // the replication's sums (in the unit, except the count of zero waits and
  // the largest wait, kept as -wmax so that the largest wait is a maximum):
  // lanes of the wavefront, then its wavefronts in order. v: W, T, I, then
  // the features' A, S, W, T, zeros, max W, T_{K-1}, I, then the four
  // controls after the prefix and the four over it
  float v[19];
  v[0] = group_sum_compensated((kt.sum - ks.sum) - (kt.comp - ks.comp), G);
  v[1] = group_sum_compensated(kt.value(), G);
  v[2] = group_sum_compensated(ki.value(), G);
  v[3] = group_sum_compensated(ft.sa, G);
  v[4] = group_sum_compensated(ft.ss, G);
  v[5] = group_sum_compensated(ft.sw, G);
  v[6] = group_sum_compensated(ft.st, G);
  v[7] = (float)group_sum_i(ft.zeros, G);
  v[8] = group_max(-ft.wmax, G);
  v[9] = group_sum_compensated(ft.tlast, G);
  v[10] = group_sum_compensated(ft.si, G);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    v[11 + k] = group_sum_compensated(kc[k].value(), G);
    v[15 + k] = group_sum_compensated(ft.pc[k], G);
  }
  if (LPR > 64) {
    if (lane == 0) {
#pragma unroll
      for (int k = 0; k < 19; ++k) sh_f[wave][k] = v[k];
    }
    __syncthreads();
    if (j == 0) {  // lane 0 of the replication's first wavefront
#pragma unroll
      for (int k = 0; k < 19; ++k) {
        float hi = sh_f[wave][k], lo = 0.0f;
        for (int w = wave + 1; w < wave + LPR / 64; ++w) {
          if (k == 8) {
            hi = fmaxf(hi, sh_f[w][k]);
          } else {
            float s2, e;
            two_sum(hi, sh_f[w][k], s2, e);
            hi = s2;
            lo += e;
          }
        }
        v[k] = hi + lo;
      }
    }
  }
  if (j == 0 && N > 0) {
    const float nf_ = (float)N;
    a.mean_w[r] = v[0] * cs / nf_;
    a.mean_t[r] = v[1] * cs / nf_;
    a.mean_i[r] = v[2] * cs / nf_;
    if (K > 0) {
      const float kf = (float)K;
      float *f = a.features + r * 10;
      f[0] = a.lambda / a.mu;
      f[1] = a.mu;
      f[2] = v[3] * cs / kf;
      f[3] = v[4] * cs / kf;
      f[4] = v[5] * cs / kf;
      f[5] = v[6] * cs / kf;
      f[6] = v[7] / kf;
      f[7] = v[8] * -cs;
      f[8] = v[10] * cs / kf;
      f[9] = v[9] * cs;
#pragma unroll
      for (int k = 0; k < 4; ++k) {  // the T-weighted two from the unit
        a.controls[r * 8 + k] = k >= 2 ? v[11 + k] * cs : v[11 + k];
        a.controls[r * 8 + 4 + k] = k >= 2 ? v[15 + k] * cs : v[15 + k];
      }
    }
  }
}

// Persistent plan kernel: every wave pops units of RPW items (longest first)
// until the queue is empty; the exit test is wave-uniform, so the grid always
// drains.
template <int RPW, bool FT>
__global__ __launch_bounds__(ft_max_wg<FT>()) void mm1_plan_kernel(Mm1Args a, uint64_t n_items) {
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
    PhiloxSource src{k0, k1};
    const Rep d = item_rep(a, (uint64_t)unit * RPW + q, n_items);
    wave_group<RPW, FT>(d, src, a.feature_prefix, a);
    // the lane that stored the item's outputs flags it
    if (a.done && (lane % (16 * S)) == 0 && d.n > 0) a.done[d.out] = 1;
  }
}

// Split replication: X wavefronts of one workgroup share each replication,
// part h taking an equal run of its chunks. Every part first runs its chunks
// from carry 0 (speculation; exact for part 0). Then, in order, each part h
// re-runs its leading chunks from the true carry left by part h-1 alongside
// the speculative one and adds the difference of their sums, until the two
// carries are bit-identical: from there on the trajectories coincide (once a
// chunk's composite map takes its constant branch for the larger carry it
// takes it for the smaller one too), so the rest of the speculative pass is
// already exact. Per-customer values equal the unsplit engine's; only the
// summation order of the means differs. Part 0 keeps the feature chunks.
// Workgroup of the split kernels: 256 threads (4 / X replications) for
// X <= 4 wavefronts per replication, one replication of X wavefronts above.
template <int X>
constexpr int split_wg() {
  return X <= 4 ? 256 : 64 * X;
}
template <int X>
constexpr int split_slots() {
  return split_wg<X>() / (64 * X);
}

// Parts h >= 1 only compose and scan their first chunk in phase 1 and
// apply it once, from the true start, in phase 2. STASH: its variates and
// scan per lane ([value][lane]: lane-contiguous) and the segment totals
// wait in LDS; without it (the kernels with the controls, whose registers
// are full) phase 2 draws the chunk again, to the same bits.
template <int X, bool STASH>
struct SplitShared {
  static constexpr int NF = STASH ? X - 1 : 1;
  float spec[split_slots<X>()][X], fin[split_slots<X>()][X];
  float sum[split_slots<X>()][X][7];  // W, T, I, then the four controls
  float first[split_slots<X>()][NF][STASH ? 2 * MM1_P + 4 : 1][64];
  float first_t[split_slots<X>()][NF][8];
};

// Part h of replication d (slot `slot` of the workgroup); every thread of
// the workgroup must call it (it holds X + 2 barriers, whatever the data).
//
// Phase 1: every part runs its chunks from carry 0 (exact for part 0).
// Phase 2: every part h >= 1 at once takes the carry part h-1 ended with in
// phase 1 as its true start and re-runs its leading chunks from both starts,
// adding the difference of the sums, until the two trajectories are
// bit-identical (Lindley's recursion forgets its start once the queue
// empties; carries are ordered, so once they meet they stay equal). The
// assumption holds whenever part h-1 met its own trajectory.
// Phase 3: in order, a part whose assumed start differs from its
// predecessor's true end (the predecessor never coupled) corrects again
// from that end.
//
// FT = false is the form for runs without prefix features (K = 0): the
// feature chunks, the controls and their registers are compiled out (about
// half the registers of the FT form), which the kernels take when K = 0.
// With FT every part adds the controls of its customers (all after the
// prefix except in part 0's feature chunks); the deferred first chunk adds
// all four of its controls, a later correction chunk the difference of the
// two T-weighted ones between its two starts.
template <int X, bool FT>
__device__ __forceinline__ void split_replication(const Rep &d, int slot, int h, uint32_t k0,
                                                  uint32_t k1, uint64_t K, const Mm1Args &a,
                                                  SplitShared<X, !FT> &sh) {
  constexpr bool STASH = !FT;
  if (!FT) K = 0;
  constexpr int P = MM1_P;
  constexpr uint64_t CHUNK = 16u * P * 4;
  const int lane = threadIdx.x & 63;
  const uint32_t chunks = (uint32_t)((d.n + CHUNK - 1) / CHUNK);
  const uint32_t full = (uint32_t)(d.n / CHUNK);
  const uint32_t fchunks = min(chunks, (uint32_t)((K + CHUNK - 1) / CHUNK));
  const bool split = chunks / X >= 2 && chunks / X >= fchunks;
  const uint32_t cb = split ? (uint32_t)((uint64_t)h * chunks / X) : (h == 0 ? 0u : chunks);
  const uint32_t ce = split ? (uint32_t)((uint64_t)(h + 1) * chunks / X) : chunks;

  // phase 1: every part from carry 0
  float carry = 0.0f;
  Sums acc;
  Feat ft;
  uint32_t c = cb;
  // parts h >= 1: their first chunk (full, after any feature prefix: a split
  // part holds at least two chunks and the prefix lies in part 0) is only
  // composed and scanned here, which gives the speculative carry after it;
  // phase 2 applies it from the true start
  const bool deferred_first = split && h >= 1;
  float spec0 = 0.0f;  // the speculative carry after the first chunk
  if (deferred_first) {
    const Draw<P> dr = draw_chunk<1, P>((uint64_t)c * CHUNK, d, k0, k1);
    const ChunkScan cs = compose_scan<P>(dr);
    float tin;
    carry = carry_through<1>(cs, carry, tin);
    spec0 = carry;
    if constexpr (STASH) {
      float(*st)[64] = sh.first[slot][h - 1];
#pragma unroll
      for (int j = 0; j < P; ++j) {
        st[j][lane] = dr.A[j];
        st[P + j][lane] = dr.S[j];
      }
      st[2 * P][lane] = cs.ea;
      st[2 * P + 1][lane] = cs.eb;
      st[2 * P + 2][lane] = cs.ha;
      st[2 * P + 3][lane] = cs.hb;
      if (lane == 0) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          sh.first_t[slot][h - 1][j] = cs.ta[j];
          sh.first_t[slot][h - 1][4 + j] = cs.tb[j];
        }
      }
    }
    ++c;
  }
#define MRIP_CHUNK(F, TL)                                                          \
  {                                                                                \
    const Draw<P> dr = draw_chunk<1, P>((uint64_t)c * CHUNK, d, k0, k1);          \
    wave_chunk<1, P, F, TL, FT>((uint64_t)c * CHUNK, dr, d, K, carry, acc, ft);    \
  }
  if (FT)
    for (; c < min(ce, fchunks); ++c) MRIP_CHUNK(true, true)
  for (; c < min(ce, full); ++c) MRIP_CHUNK(false, false)
  for (; c < ce; ++c) MRIP_CHUNK(false, true)
#undef MRIP_CHUNK
  if (lane == 0) sh.spec[slot][h] = carry;
  __syncthreads();

  // the part's correction from true start `cin`: its first chunk applied
  // from cin, then fix-up chunks until the true and speculative carries
  // meet; returns its true end
  Sums fix;
  auto correct = [&](float cin) -> float {
    fix = Sums();
    Draw<P> dr;
    ChunkScan scan;
    if constexpr (STASH) {
      const float(*st)[64] = sh.first[slot][h - 1];
#pragma unroll
      for (int j = 0; j < P; ++j) {
        dr.A[j] = st[j][lane];
        dr.S[j] = st[P + j][lane];
      }
      scan.ea = st[2 * P][lane];
      scan.eb = st[2 * P + 1][lane];
      scan.ha = st[2 * P + 2][lane];
      scan.hb = st[2 * P + 3][lane];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        scan.ta[j] = sh.first_t[slot][h - 1][j];
        scan.tb[j] = sh.first_t[slot][h - 1][4 + j];
      }
    } else {  // the same chunk drawn and scanned again: the same bits
      dr = draw_chunk<1, P>((uint64_t)cb * CHUNK, d, k0, k1);
      scan = compose_scan<P>(dr);
    }
    float tin;
    float ct = carry_through<1>(scan, cin, tin);
    {
      Feat none;
      float stt, ss, si, cl[4];
      apply_lane<P, false, false, FT>(later(scan.ea, tin + scan.eb), scan, dr,
                                      lane_first_customer<1, P>((uint64_t)cb * CHUNK), d.n, 0,
                                      d.cs, d.ea, d.es, stt, ss, si, none, cl);
      fix.t.add(stt);
      fix.s.add(ss);
      fix.i.add(si);
      if (FT) {
#pragma unroll
        for (int k = 0; k < 4; ++k) fix.c[k].add(cl[k]);
      }
    }
    float cs = spec0;
    bool coupled =
        __builtin_amdgcn_readfirstlane((int)(__float_as_uint(ct) == __float_as_uint(cs))) != 0;
    for (uint32_t cc = cb + 1; cc < ce && !coupled; ++cc) {
      const Draw<P> dr = draw_chunk<1, P>((uint64_t)cc * CHUNK, d, k0, k1);
      if (cc < full) fixup_chunk<P, false, FT>((uint64_t)cc * CHUNK, dr, d, ct, cs, fix);
      else fixup_chunk<P, true, FT>((uint64_t)cc * CHUNK, dr, d, ct, cs, fix);
      coupled = __builtin_amdgcn_readfirstlane((int)(__float_as_uint(ct) == __float_as_uint(cs))) != 0;
    }
    return coupled ? carry : ct;
  };

  // phase 2: all parts at once, each from its predecessor's phase-1 end
  float fin = carry;
  if (split && h >= 1) fin = correct(sh.spec[slot][h - 1]);
  if (lane == 0) sh.fin[slot][h] = fin;
  __syncthreads();

  // phase 3: in order, only where the assumed start was not the true one
  // (kept rolled: one copy of the correction instead of X - 1). It runs at
  // all only if some part of some replication of the workgroup started from
  // a wrong end, a decision the whole workgroup shares (it holds barriers).
  bool wrong = false;
#pragma unroll
  for (int s2 = 0; s2 < split_slots<X>(); ++s2)
#pragma unroll
    for (int j = 1; j < X; ++j)
      wrong |= __float_as_uint(sh.fin[s2][j - 1]) != __float_as_uint(sh.spec[s2][j - 1]);
  if (__builtin_amdgcn_readfirstlane((int)wrong)) {
#pragma unroll 1
    for (int j = 1; j < X; ++j) {
      if (split && h == j &&
          __float_as_uint(sh.fin[slot][j - 1]) != __float_as_uint(sh.spec[slot][j - 1])) {
        const float f = correct(sh.fin[slot][j - 1]);
        if (lane == 0) sh.fin[slot][j] = f;
      }
      __syncthreads();
    }
  }
  acc.t.add(fix.t.value());
  acc.s.add(fix.s.value());
  acc.i.add(fix.i.value());
  if (FT) {
#pragma unroll
    for (int k = 0; k < 4; ++k) acc.c[k].add(fix.c[k].value());
  }

  // phase 3: part sums, then the replication's means in part order
  constexpr int NS = FT ? 7 : 3;
  float part[NS];
  part[0] = group_sum_compensated(wait_sum(acc), 64);
  part[1] = group_sum_compensated(acc.t.value(), 64);
  part[2] = group_sum_compensated(acc.i.value(), 64);
  if (FT) {
#pragma unroll
    for (int k = 0; k < 4; ++k) part[3 + k] = group_sum_compensated(acc.c[k].value(), 64);
  }
  float f[10], pcs[4];
  if (FT && h == 0 && K > 0) {
#pragma unroll
    for (int k = 0; k < 4; ++k) pcs[k] = group_sum_compensated(ft.pc[k], 64);
    const float kf = (float)K;
    f[0] = d.lambda / d.mu;
    f[1] = d.mu;
    f[2] = group_sum_compensated(ft.sa, 64) * d.cs / kf;
    f[3] = group_sum_compensated(ft.ss, 64) * d.cs / kf;
    f[4] = group_sum_compensated(ft.sw, 64) * d.cs / kf;
    f[5] = group_sum_compensated(ft.st, 64) * d.cs / kf;
    f[6] = (float)group_sum_i(ft.zeros, 64) / kf;
    f[7] = group_max(-ft.wmax, 64) * -d.cs;  // the latest of the waits
    f[8] = group_sum_compensated(ft.si, 64) * d.cs / kf;
    f[9] = group_sum_compensated(ft.tlast, 64) * d.cs;
  }
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < NS; ++k) sh.sum[slot][h][k] = part[k];
  }
  __syncthreads();
  if (h == 0 && lane == 0 && d.n > 0) {
    float tot[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      float hi = sh.sum[slot][0][k], lo = 0.0f;
#pragma unroll
      for (int j = 1; j < X; ++j) {
        float s2, e;
        two_sum(hi, sh.sum[slot][j][k], s2, e);
        hi = s2;
        lo += e;
      }
      tot[k] = hi + lo;
    }
    const float nf = (float)d.n;
    a.mean_w[d.out] = tot[0] * d.cs / nf;
    a.mean_t[d.out] = tot[1] * d.cs / nf;
    a.mean_i[d.out] = tot[2] * d.cs / nf;
    if (FT && K > 0) {
#pragma unroll
      for (int j = 0; j < 10; ++j) a.features[d.out * 10 + j] = f[j];
#pragma unroll
      for (int k = 0; k < 4; ++k) {  // the T-weighted two from the unit
        a.controls[d.out * 8 + k] = k >= 2 ? tot[3 + k] * d.cs : tot[3 + k];
        a.controls[d.out * 8 + 4 + k] = k >= 2 ? pcs[k] * d.cs : pcs[k];
      }
    }
  }
}

// The extra workgroup of a split launch: the previous run's statistics,
// the same bits as the reduction kernel's, then the sequence number that
// tells the host they are there.
__device__ void reduce_previous_run(const Mm1Args &a) {
  __shared__ RedShared sh;
  for (int o = 0; o < 3; ++o) reduce_output(a.prev_x[o], 1, a.prev_n, a.prev_out + 3 * o, sh);
  if (threadIdx.x == 0) {
    __threadfence_system();
    __hip_atomic_store(a.prev_seq, a.prev_seq_value, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
  }
}

template <int X, bool FT>
__global__ __launch_bounds__(split_wg<X>(), FT ? 1 : 4) void mm1_split_kernel(Mm1Args a, float ca,
                                                                           float cs) {
  if constexpr (split_wg<X>() == RED_THREADS) {
    if (a.prev_n > 0 && blockIdx.x == gridDim.x - 1) {  // uniform across the workgroup
      reduce_previous_run(a);
      return;
    }
  }
  constexpr int SLOTS = split_slots<X>();  // replications per workgroup
  __shared__ SplitShared<X, !FT> sh;
  const int wave = threadIdx.x >> 6;
  const int slot = wave / X, h = wave % X;
  const uint64_t r = (uint64_t)blockIdx.x * SLOTS + slot;
  split_replication<X, FT>(uniform_rep(a, r, ca, cs), slot, h, (uint32_t)a.seed,
                           (uint32_t)(a.seed >> 32), a.feature_prefix, a, sh);
}

// Persistent plan kernel with the long items split: the first n_long items
// of the longest-first order are served one per X wavefronts of a workgroup
// (X = 2 or 4: 256-thread workgroups of 4 / X items; X = 8: one item per
// 512-thread workgroup)
// (queue_head[0]), at raised wave priority so that the critical path keeps
// its issue slots when it shares a SIMD; then every wavefront serves the
// rest RPW items at a time (queue_head[1]). Both exits are uniform (the
// first per workgroup, the second per wavefront), so the grid drains.
template <int X, int RPW, bool FT>
__global__ __launch_bounds__(split_wg<X>()) void mm1_plan_split_kernel(Mm1Args a, uint64_t n_items,
                                                                       uint64_t n_long) {
  constexpr int SLOTS = split_slots<X>();
  static_assert(X == 2 || X == 4 || X == 8, "plans split over 2, 4 or 8 wavefronts");
  constexpr int S = 4 / RPW;
  __shared__ SplitShared<X, !FT> sh;
  __shared__ uint32_t sh_pop;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int slot = wave / X, h = wave % X;
  const uint32_t k0 = (uint32_t)a.seed, k1 = (uint32_t)(a.seed >> 32);
  __builtin_amdgcn_s_setprio(2);
  for (;;) {
    if (threadIdx.x == 0) sh_pop = atomicAdd(&a.queue_head[0], (uint32_t)SLOTS);
    __syncthreads();
    const uint64_t first = sh_pop;
    __syncthreads();
    if (first >= n_long) break;
    const uint64_t idx = first + slot;
    const Rep d = item_rep(a, idx, idx < n_long ? n_long : 0);
    split_replication<X, FT>(d, slot, h, k0, k1, a.feature_prefix, a, sh);
    if (a.done && h == 0 && lane == 0 && d.n > 0) a.done[d.out] = 1;  // after its outputs
  }
  __builtin_amdgcn_s_setprio(0);
  const int q = (lane >> 4) / S;
  const uint64_t n_short = n_items - n_long;
  const uint64_t n_units = (n_short + RPW - 1) / RPW;
  for (;;) {
    uint32_t unit = 0;
    if (lane == 0) unit = atomicAdd(&a.queue_head[1], 1u);
    unit = (uint32_t)__builtin_amdgcn_readfirstlane((int)__shfl((int)unit, 0, 64));
    if (unit >= n_units) break;
    const uint64_t j = (uint64_t)unit * RPW + q;
    PhiloxSource src{k0, k1};
    const Rep d = item_rep(a, n_long + j, j < n_short ? n_items : 0);
    wave_group<RPW, FT>(d, src, a.feature_prefix, a);
    if (a.done && (lane % (16 * S)) == 0 && d.n > 0) a.done[d.out] = 1;
  }
}

// STRIDE = 1: one replication per lane; 64: one working lane per wavefront
// (the paper's WLP form).
// One replication by Lindley's recursion, customer after customer, in one
// lane (the thread-per-replication form).
template <int RNG>
__device__ void simt_replication(const Rep &d, uint64_t K, uint32_t k0, uint32_t k1,
                                 const Mm1Args &a) {
  const uint64_t N = d.n;
  float tprev = 0.0f;
  Kahan sw, st, si, ctl[8];
  Feat ft;
  Taus ts;
  if (RNG == RNG_TAUS88) ts = taus_seed(TAG_MM1, d.dp, d.rep, k0, k1);
  for (uint64_t k = 0; 2 * k < N; ++k) {
    Block4 b;
    if (RNG == RNG_TAUS88) {
      b.x = taus_next(ts);
      b.y = taus_next(ts);
      b.z = taus_next(ts);
      b.w = taus_next(ts);
    } else {
      b = philox((uint32_t)k, d.dp, d.rep, TAG_MM1, k0, k1);
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const uint64_t n = 2 * k + h;
      if (n >= N) break;
      const float A = exp_variate(h ? b.z : b.x, d.ca);
      const float Sv = exp_variate(h ? b.w : b.y, d.cs);
      if (K > 0) {  // the controls (after the prefix, or over it), weighted by T_{n-1}
        const float ds = Sv - d.es, da = A - d.ea;
        Kahan *c = ctl + (n >= K ? 0 : 4);
        c[0].add(ds);
        c[1].add(da);
        c[2].add(tprev * ds);
        c[3].add(tprev * da);
      }
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
  a.mean_w[d.out] = sw.value() / nf;
  a.mean_t[d.out] = st.value() / nf;
  a.mean_i[d.out] = si.value() / nf;
  if (K > 0) {
    const float kf = (float)K;
    float *f = a.features + d.out * 10;
    f[0] = d.lambda / d.mu;
    f[1] = d.mu;
    f[2] = ft.sa / kf;
    f[3] = ft.ss / kf;
    f[4] = ft.sw / kf;
    f[5] = ft.st / kf;
    f[6] = (float)ft.zeros / kf;
    f[7] = ft.wmax;
    f[8] = ft.si / kf;
    f[9] = ft.tlast;
#pragma unroll
    for (int k = 0; k < 8; ++k) a.controls[d.out * 8 + k] = ctl[k].value();
  }
  if (a.done) a.done[d.out] = 1;
}

// STRIDE = 1: one replication per lane. STRIDE = 64: one per wavefront with
// only its first lane working (the paper's WLP form).
template <int STRIDE, int RNG>
__global__ void mm1_simt_kernel(Mm1Args a, float ca, float cs) {
  if (threadIdx.x % STRIDE) return;
  const uint64_t r = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / STRIDE;
  if (r >= a.n_reps) return;
  simt_replication<RNG>(uniform_rep(a, r, ca, cs), a.feature_prefix, (uint32_t)a.seed,
                        (uint32_t)(a.seed >> 32), a);
}

// A plan in the thread-per-replication form: every working lane pops the
// next item of the longest-first order from the device queue and runs it
// alone, until the queue is empty (each lane's exit is its own; the grid
// drains once every lane has seen the queue exhausted).
template <int STRIDE>
__global__ void mm1_plan_simt_kernel(Mm1Args a, uint64_t n_items) {
  if (threadIdx.x % STRIDE) return;
  const uint32_t k0 = (uint32_t)a.seed, k1 = (uint32_t)(a.seed >> 32);
  for (;;) {
    const uint32_t slot = atomicAdd(a.queue_head, 1u);
    if (slot >= n_items) break;
    simt_replication<RNG_PHILOX>(item_rep(a, slot, n_items), a.feature_prefix, k0, k1, a);
  }
}

__global__ void zero_u32_kernel(uint32_t *p, uint32_t n) {
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = 0u;
}

float host_neg_mean_ln2(float rate) {
  return (float)(-(1.0 / (double)rate) * 0.69314718055994530942);
}

// The launch's copy of the arguments with the controls' centring constants.
Mm1Args centred(const Mm1Args &a) {
  Mm1Args b = a;
  if (b.feature_prefix > 0) {
    b.log_grid_mean = log_grid_mean();
    if (!b.items.dp) {
      b.ea = variate_mean_f32(b.lambda);
      b.es = variate_mean_f32(b.mu);
    }
  }
  return b;
}

}  // namespace

// (1 / 2^24) sum_{k=1}^{2^24} (24 ln 2 - ln k) = 24 ln 2 - ln((2^24)!) / 2^24
double log_grid_mean() {
  return 24.0 * std::log(2.0) - std::lgamma(16777217.0) / 16777216.0;
}

float variate_mean_f32(float rate) {
  return (float)((double)(float)(1.0 / (double)rate) * log_grid_mean());
}

template <int LPR>
hipError_t taus_launch(const Mm1Args &a, hipStream_t s) {
  constexpr uint32_t RPB = 256 / LPR;
  const uint64_t blocks = (a.n_reps + RPB - 1) / RPB;
  const float ca = host_neg_mean_ln2(a.lambda), cs = host_neg_mean_ln2(a.mu);
  hipLaunchKernelGGL(mm1_taus_kernel<LPR>, dim3((uint32_t)blocks), dim3(256), 0, s, a, ca, cs);
  return hipGetLastError();
}

hipError_t launch_mm1_taus(const Mm1Args &a_in, uint32_t lanes_per_rep, hipStream_t s) {
  const Mm1Args a = centred(a_in);
  switch (lanes_per_rep) {
    case 16: return taus_launch<16>(a, s);
    case 32: return taus_launch<32>(a, s);
    case 64: return taus_launch<64>(a, s);
    case 128: return taus_launch<128>(a, s);
    case 256: return taus_launch<256>(a, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_mm1_wave(const Mm1Args &a_in, uint32_t rpw, uint32_t wg, hipStream_t s) {
  const Mm1Args a = centred(a_in);
  if (a.feature_prefix > 0) wg = std::min<uint32_t>(wg, ft_max_wg<true>());
  const uint64_t waves = (a.n_reps + rpw - 1) / rpw;
  const uint32_t wpb = wg / 64;
  const uint64_t blocks = (waves + wpb - 1) / wpb;
  const float ca = host_neg_mean_ln2(a.lambda), cs = host_neg_mean_ln2(a.mu);
  const dim3 g((uint32_t)blocks), b(wg);
  if (a.rng == RNG_TAUS88) return launch_mm1_taus(a, 64 / rpw, s);
  const bool ft = a.feature_prefix > 0;
  if (rpw == 1 && ft) hipLaunchKernelGGL((mm1_wave_kernel<1, true>), g, b, 0, s, a, ca, cs);
  else if (rpw == 1) hipLaunchKernelGGL((mm1_wave_kernel<1, false>), g, b, 0, s, a, ca, cs);
  else if (rpw == 2 && ft) hipLaunchKernelGGL((mm1_wave_kernel<2, true>), g, b, 0, s, a, ca, cs);
  else if (rpw == 2) hipLaunchKernelGGL((mm1_wave_kernel<2, false>), g, b, 0, s, a, ca, cs);
  else if (ft) hipLaunchKernelGGL((mm1_wave_kernel<4, true>), g, b, 0, s, a, ca, cs);
  else hipLaunchKernelGGL((mm1_wave_kernel<4, false>), g, b, 0, s, a, ca, cs);
  return hipGetLastError();
}

template <int X, bool FT>
hipError_t split_launch_as(const Mm1Args &a, float ca, float cs, hipStream_t s,
                           const KernelEvents *ev) {
  if (a.prev_n > 0 && split_wg<X>() != RED_THREADS) return hipErrorInvalidValue;
  // one more workgroup when it reduces the previous run
  const uint64_t blocks =
      (a.n_reps + split_slots<X>() - 1) / split_slots<X>() + (a.prev_n > 0 ? 1 : 0);
  const dim3 g((uint32_t)blocks), b(split_wg<X>());
  if (ev)
    hipExtLaunchKernelGGL((mm1_split_kernel<X, FT>), g, b, 0, s, ev->start, ev->stop, 0, a, ca,
                          cs);
  else
    hipLaunchKernelGGL((mm1_split_kernel<X, FT>), g, b, 0, s, a, ca, cs);
  return hipGetLastError();
}

template <int X>
hipError_t split_launch(const Mm1Args &a, float ca, float cs, hipStream_t s,
                        const KernelEvents *ev) {
  return a.feature_prefix > 0 ? split_launch_as<X, true>(a, ca, cs, s, ev)
                              : split_launch_as<X, false>(a, ca, cs, s, ev);
}

hipError_t launch_mm1_split(const Mm1Args &a_in, uint32_t waves_per_rep, hipStream_t s,
                            const KernelEvents *ev) {
  const Mm1Args a = centred(a_in);
  if (a.rng == RNG_TAUS88) {
    if (ev) return hipErrorInvalidValue;  // the taus88 form is not self-timed
    return launch_mm1_taus(a, 64 * waves_per_rep, s);
  }
  const float ca = host_neg_mean_ln2(a.lambda), cs = host_neg_mean_ln2(a.mu);
  if (waves_per_rep == 2) return split_launch<2>(a, ca, cs, s, ev);
  if (waves_per_rep == 4) return split_launch<4>(a, ca, cs, s, ev);
  if (waves_per_rep == 8) return split_launch<8>(a, ca, cs, s, ev);
  return hipErrorInvalidValue;
}

hipError_t launch_mm1_simt(const Mm1Args &a_in, bool one_lane, hipStream_t s) {
  const Mm1Args a = centred(a_in);
  const uint32_t wg = 64;
  const uint64_t threads = a.n_reps * (one_lane ? 64 : 1);
  const uint64_t blocks = (threads + wg - 1) / wg;
  const float ca = host_neg_mean_ln2(a.lambda), cs = host_neg_mean_ln2(a.mu);
  const dim3 g((uint32_t)blocks), b(wg);
  if (a.rng == RNG_TAUS88) {
    if (one_lane) hipLaunchKernelGGL((mm1_simt_kernel<64, RNG_TAUS88>), g, b, 0, s, a, ca, cs);
    else hipLaunchKernelGGL((mm1_simt_kernel<1, RNG_TAUS88>), g, b, 0, s, a, ca, cs);
  } else {
    if (one_lane) hipLaunchKernelGGL((mm1_simt_kernel<64, RNG_PHILOX>), g, b, 0, s, a, ca, cs);
    else hipLaunchKernelGGL((mm1_simt_kernel<1, RNG_PHILOX>), g, b, 0, s, a, ca, cs);
  }
  return hipGetLastError();
}

hipError_t launch_mm1_plan_simt(const Mm1Args &a_in, uint64_t n_items, bool one_lane,
                                hipStream_t s) {
  const Mm1Args a = centred(a_in);
  int dev = 0, cus = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  // working lanes: at most one per item, at most a wavefront per SIMD's worth
  const uint64_t lanes = std::min<uint64_t>(n_items, (uint64_t)cus * 4 * 64);
  const uint64_t threads = lanes * (one_lane ? 64 : 1);
  const dim3 g((uint32_t)((threads + 63) / 64)), b(64);
  if (one_lane) hipLaunchKernelGGL(mm1_plan_simt_kernel<64>, g, b, 0, s, a, n_items);
  else hipLaunchKernelGGL(mm1_plan_simt_kernel<1>, g, b, 0, s, a, n_items);
  return hipGetLastError();
}

hipError_t launch_mm1_plan(const Mm1Args &a_in, uint64_t n_items, uint32_t rpw, uint32_t wg,
                           hipStream_t s) {
  const Mm1Args a = centred(a_in);
  if (a.feature_prefix > 0) wg = std::min<uint32_t>(wg, ft_max_wg<true>());
  int dev = 0, cus = 0, per_cu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  const bool ft = a.feature_prefix > 0;
  const void *fn = rpw == 1 ? (ft ? (const void *)mm1_plan_kernel<1, true>
                                  : (const void *)mm1_plan_kernel<1, false>)
                 : rpw == 2 ? (ft ? (const void *)mm1_plan_kernel<2, true>
                                  : (const void *)mm1_plan_kernel<2, false>)
                            : (ft ? (const void *)mm1_plan_kernel<4, true>
                                  : (const void *)mm1_plan_kernel<4, false>);
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, (int)wg, 0);
  if (e != hipSuccess) return e;
  if (per_cu < 1) per_cu = 1;
  // never more waves than work units
  const uint64_t units = (n_items + rpw - 1) / rpw;
  uint64_t blocks = (uint64_t)cus * (uint64_t)per_cu;
  const uint64_t need = (units + wg / 64 - 1) / (wg / 64);
  if (blocks > need) blocks = need;
  if (blocks < 1) blocks = 1;
  void *args[] = {(void *)&a, (void *)&n_items};
  e = hipLaunchKernel(fn, dim3((uint32_t)blocks), dim3(wg), args, 0, s);
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

hipError_t launch_mm1_plan_split(const Mm1Args &a_in, uint64_t n_items, uint64_t n_long,
                                 uint32_t waves_per_rep, uint32_t rpw, hipStream_t s) {
  const Mm1Args a = centred(a_in);
  int dev = 0, cus = 0, per_cu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  const bool ft = a.feature_prefix > 0;
#define MRIP_PICK(X, R) (ft ? (const void *)mm1_plan_split_kernel<X, R, true> \
                            : (const void *)mm1_plan_split_kernel<X, R, false>)
#define MRIP_PICK_X(X) (rpw == 1 ? MRIP_PICK(X, 1) : rpw == 2 ? MRIP_PICK(X, 2) : MRIP_PICK(X, 4))
  const void *fn = waves_per_rep == 2   ? MRIP_PICK_X(2)
                   : waves_per_rep == 4 ? MRIP_PICK_X(4)
                                        : MRIP_PICK_X(8);
#undef MRIP_PICK_X
#undef MRIP_PICK
  const int wg = waves_per_rep == 8 ? split_wg<8>() : 256;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, wg, 0);
  if (e != hipSuccess) return e;
  if (per_cu < 1) per_cu = 1;
  const uint64_t blocks = (uint64_t)cus * (uint64_t)per_cu;
  void *args[] = {(void *)&a, (void *)&n_items, (void *)&n_long};
  e = hipLaunchKernel(fn, dim3((uint32_t)blocks), dim3(wg), args, 0, s);
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

hipError_t launch_zero_u32(uint32_t *p, uint32_t n, hipStream_t s) {
  const uint32_t blocks = n <= 64 ? 1u : std::min<uint32_t>(1024u, (n + 255u) / 256u);
  hipLaunchKernelGGL(zero_u32_kernel, dim3(blocks), dim3(n <= 64 ? 64 : 256), 0, s, p, n);
  return hipGetLastError();
}

}  // namespace mrip
