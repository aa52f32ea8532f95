/*
 * MRIP reference oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, sequential CPU implementation of what the MRIP hot path
 * computes (Passerat-Palmbach et al., "Warp-Level Parallelism: Enabling
 * Multiple Replications In Parallel on GPU", ESM 2011). One replication at a
 * time, one event at a time, in the order the model definitions state.
 *
 * Only the test-suite, the smoke check and the benchmark's CPU-baseline leg
 * may load this library. The GPU library never links, includes or calls it,
 * and this file includes nothing from the GPU library.
 *
 * Build: gcc -O2 -fno-fast-math -ffp-contract=off -shared -fPIC (see build.py).
 *
 * Pins (tests/test_oracle_*.py):
 *   philox   -- two independent Philox4x32-10 implementations (PyTorch's and
 *               rocRAND's engines) on >=1e4 random (key, counter) pairs.
 *   rw       -- E[ssd] = W*T (unbiased lattice walk, MSD = t), parity of ssd,
 *               exact distinct-site distribution by 4^T enumeration; the
 *               per-walker site counts hand-traced and equal to the sum of
 *               one-walker runs.
 *   mm1      -- M/M/1 closed form Wq = rho/(mu-lambda), a hand-traced case,
 *               an independent absolute-clock event simulation, degenerate
 *               inputs (S == 0, A == 0). Controls: hand-traced values, the
 *               degenerate inputs against brute force, flow balance, the
 *               grid mean's closed form, mean zero times functions of the
 *               prefix over replications, and the perturbation-analysis
 *               coefficients of the weighted pair.
 *   ff       -- injected-uniform cases with closed-form burnt counts and an
 *               independent array-rolling implementation on tiny grids.
 *   pi       -- hand-checked inside/outside points on and near the circle,
 *               E[hits/N] = pi/4 and the binomial variance N p (1 - p).
 *   taus88   -- each component against the bit-serial linear recurrence of
 *               its trinomial, primitivity of the three trinomials, Random
 *               Spacing seeds against an independent Philox, and the three
 *               models on streams built from the bit-serial definition.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define EXPORT __attribute__((visibility("default")))

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11, section 3.2):          */
/* each round multiplies counter words 0 and 2 by two fixed constants into  */
/* 64-bit products; the new words are (hi(M1*c2) ^ c1 ^ k0, lo(M1*c2),      */
/* hi(M0*c0) ^ c3 ^ k1, lo(M0*c0)); the key is bumped by two Weyl constants */
/* between rounds; 10 rounds.                                               */
/* ------------------------------------------------------------------------ */
#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

EXPORT void oracle_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2],
                                 uint32_t out[4]) {
  uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
  uint32_t k0 = key_in[0], k1 = key_in[1];
  for (int round = 0; round < 10; ++round) {
    uint64_t p0 = (uint64_t)PHILOX_M0 * (uint64_t)c0;
    uint64_t p1 = (uint64_t)PHILOX_M1 * (uint64_t)c2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    c0 = hi1 ^ c1 ^ k0;
    c1 = lo1;
    c2 = hi0 ^ c3 ^ k1;
    c3 = lo0;
    if (round < 9) {
      k0 += PHILOX_W0;
      k1 += PHILOX_W1;
    }
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* n blocks; ctr is n x 4, key is n x 2, out is n x 4 (row-major). */
EXPORT void oracle_philox_batch(uint64_t n, const uint32_t *ctr, const uint32_t *key,
                                uint32_t *out) {
  for (uint64_t i = 0; i < n; ++i) oracle_philox4x32_10(ctr + 4 * i, key + 2 * i, out + 4 * i);
}

static void philox_block(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                         uint32_t out[4]) {
  uint32_t ctr[4] = {c0, c1, c2, c3};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  oracle_philox4x32_10(ctr, key, out);
}

/* Model tags: the fourth counter word separates the streams of each model;
 * TAG_TAUS_SEED marks the blocks that seed the second generator's streams. */
enum { TAG_RW = 1, TAG_MM1 = 2, TAG_FF = 3, TAG_PI = 4, TAG_TAUS_SEED = 5 };

/* ------------------------------------------------------------------------ */
/* Variates.                                                                */
/* ------------------------------------------------------------------------ */
/* Uniform on (0, 1]: the top 24 bits plus one, times 2^-24 (exact in fp32). */
EXPORT float oracle_u01(uint32_t x) { return (float)((x >> 8) + 1u) * 0x1p-24f; }

/* Exponential with the given rate by inversion: mean * (-log u). */
EXPORT float oracle_exp_variate(uint32_t x, float rate) {
  float mean = (float)(1.0 / (double)rate);
  float u = oracle_u01(x);
  return mean * (-logf(u));
}

/* ------------------------------------------------------------------------ */
/* Lattice random walk (paper section 5.1, third model; sizes and outputs   */
/* as the configuration fixes them): W walkers on an L x L periodic         */
/* lattice, T unit moves each. Walker w starts at                           */
/* ((w mod 8) * L/8 + L/16, (w div 8) * L/8 + L/16) mod L. Move t of walker  */
/* w in replication r takes 2 bits of Philox block (t>>6, w, r, TAG_RW):     */
/* word (t>>4)&3, bits 2*(t&15)..+1. 0:+x 1:-x 2:+y 3:-y.                    */
/* Outputs: ssd = sum over walkers of the squared unwrapped displacement;   */
/* distinct = number of lattice sites visited by any walker (starts incl.); */
/* walker_sites = sum over walkers of the number of sites each one visited  */
/* (its start included).                                                    */
/* ------------------------------------------------------------------------ */
EXPORT int oracle_rw_direction(uint64_t seed, uint32_t rep, uint32_t walker, uint32_t t) {
  uint32_t blk[4];
  philox_block(seed, t >> 6, walker, rep, TAG_RW, blk);
  return (int)((blk[(t >> 4) & 3u] >> (2u * (t & 15u))) & 3u);
}

/* Core walk over an explicit direction source: dirs == NULL draws from
 * Philox, else dirs[w * T + t] gives the move. walker_sites_out may be
 * NULL. Returns 0 on success. */
static int rw_core(uint64_t seed, uint32_t rep, uint32_t W, uint32_t L, uint32_t T,
                   const uint8_t *dirs, int64_t *ssd_out, int64_t *distinct_out,
                   int64_t *walker_sites_out) {
  uint8_t *visited = (uint8_t *)calloc((size_t)L * L, 1);
  uint8_t *mine = (uint8_t *)calloc((size_t)L * L, 1);  /* this walker's sites */
  if (!visited || !mine) {
    free(visited);
    free(mine);
    return -1;
  }
  int64_t ssd = 0, walker_sites = 0;
  for (uint32_t w = 0; w < W; ++w) {
    int64_t x = ((w % 8u) * (L / 8u) + L / 16u) % L;
    int64_t y = ((w / 8u) * (L / 8u) + L / 16u) % L;
    int64_t ux = 0, uy = 0;
    memset(mine, 0, (size_t)L * L);
    visited[y * L + x] = 1;
    mine[y * L + x] = 1;
    for (uint32_t t = 0; t < T; ++t) {
      int d = dirs ? (int)dirs[(size_t)w * T + t] : oracle_rw_direction(seed, rep, w, t);
      int64_t dx = 0, dy = 0;
      if (d == 0) dx = 1;
      else if (d == 1) dx = -1;
      else if (d == 2) dy = 1;
      else dy = -1;
      ux += dx;
      uy += dy;
      x = (x + dx + L) % L;
      y = (y + dy + L) % L;
      visited[y * L + x] = 1;
      mine[y * L + x] = 1;
    }
    ssd += ux * ux + uy * uy;
    for (size_t i = 0; i < (size_t)L * L; ++i) walker_sites += mine[i];
  }
  int64_t distinct = 0;
  for (size_t i = 0; i < (size_t)L * L; ++i) distinct += visited[i];
  free(visited);
  free(mine);
  *ssd_out = ssd;
  *distinct_out = distinct;
  if (walker_sites_out) *walker_sites_out = walker_sites;
  return 0;
}

EXPORT int oracle_rw(uint64_t seed, uint32_t rep, uint32_t walkers, uint32_t grid,
                     uint32_t steps, int64_t *ssd, int64_t *distinct, int64_t *walker_sites) {
  return rw_core(seed, rep, walkers, grid, steps, NULL, ssd, distinct, walker_sites);
}

EXPORT int oracle_rw_injected(const uint8_t *dirs, uint32_t walkers, uint32_t grid,
                              uint32_t steps, int64_t *ssd, int64_t *distinct,
                              int64_t *walker_sites) {
  return rw_core(0, 0, walkers, grid, steps, dirs, ssd, distinct, walker_sites);
}

/* ------------------------------------------------------------------------ */
/* M/M/1 queue (paper section 5.1, second model). Customer n arrives A_n    */
/* after customer n-1 (A_0 after time 0, the system starting empty) and     */
/* needs service S_n. With T_{-1} = 0 the system time of the previous       */
/* customer:                                                                */
/*   W_n = max(0, T_{n-1} - A_n)   waiting time in queue                    */
/*   I_n = max(0, A_n - T_{n-1})   server idle time before customer n       */
/*   T_n = W_n + S_n               time in system                           */
/* (Lindley's recursion, each step in fp32 with one subtraction.) A_n and   */
/* S_n come from Philox block (n>>1, dp, rep, TAG_MM1): words 2(n&1) and    */
/* 2(n&1)+1, exponential with rates lambda and mu. Sums are taken in fp64   */
/* over the fp32 values and the means rounded to fp32 at the end.           */
/* Features over the first K customers (K = 0: none):                       */
/*   [rho, mu, mean A, mean S, mean W, mean T, frac(W == 0), max W,         */
/*    mean I, T_{K-1}]                                                      */
/* and four controls over the customers after them, n >= K, in fp64:       */
/*   c0 = sum (S_n - E S)          c1 = sum (A_n - E A)                     */
/*   c2 = sum T_{n-1} (S_n - E S)  c3 = sum T_{n-1} (A_n - E A)              */
/* then c4..c7, the same four sums over the prefix, n < K.                 */
/* E S, E A are the variates' exact means. A_n and S_n are independent of  */
/* everything before customer n, T_{n-1} included, so every term has mean  */
/* zero given the past: each of c0..c3 times any function of the first K   */
/* customers has mean zero, and so has each of c4..c7 (sums of martingale */
/* differences).                                                           */
/* ------------------------------------------------------------------------ */
typedef struct {
  double sum_w, sum_t, sum_i;
  double f_sum_a, f_sum_s, f_sum_w, f_sum_t, f_sum_i, f_zero, f_max_w, f_last_t;
  double es, ea;  /* exact means of S and A */
  double ctl[8];  /* after the prefix (0..3), over it (4..7) */
} mm1_acc;

/* E[-ln u] for u = (k + 1) 2^-24, k uniform on [0, 2^24): the average of   */
/* -ln(j 2^-24) over j = 1..2^24, i.e. 24 ln 2 - ln((2^24)!) / 2^24.        */
static double log_grid_mean(void) {
  return 24.0 * log(2.0) - lgamma(16777217.0) / 16777216.0;
}

/* Exact mean of the exponential variate of the given rate as drawn: its   */
/* fp32 scale (float)(1 / rate) times the grid mean of -ln u.               */
EXPORT double oracle_variate_mean(float rate) {
  return (double)(float)(1.0 / (double)rate) * log_grid_mean();
}

static void mm1_customer(float a, float s, float *t_prev, uint64_t n, uint64_t K,
                         mm1_acc *acc, float *w_out, float *i_out, float *t_out) {
  {
    double ds = (double)s - acc->es, da = (double)a - acc->ea, tp = (double)*t_prev;
    double *c = acc->ctl + (n >= K ? 0 : 4);
    c[0] += ds;
    c[1] += da;
    c[2] += tp * ds;
    c[3] += tp * da;
  }
  float w = fmaxf(0.0f, *t_prev - a);
  float idle = fmaxf(0.0f, a - *t_prev);
  float t = w + s;
  acc->sum_w += (double)w;
  acc->sum_t += (double)t;
  acc->sum_i += (double)idle;
  if (n < K) {
    acc->f_sum_a += (double)a;
    acc->f_sum_s += (double)s;
    acc->f_sum_w += (double)w;
    acc->f_sum_t += (double)t;
    acc->f_sum_i += (double)idle;
    acc->f_zero += (w == 0.0f) ? 1.0 : 0.0;
    if ((double)w > acc->f_max_w) acc->f_max_w = (double)w;
    if (n == K - 1) acc->f_last_t = (double)t;
  }
  if (w_out) *w_out = w;
  if (i_out) *i_out = idle;
  if (t_out) *t_out = t;
  *t_prev = t;
}

static void mm1_finish(const mm1_acc *acc, uint64_t N, uint64_t K, float lambda, float mu,
                       float out[3], float *feat) {
  out[0] = (float)(acc->sum_w / (double)N);
  out[1] = (float)(acc->sum_t / (double)N);
  out[2] = (float)(acc->sum_i / (double)N);
  if (feat && K > 0) {
    double k = (double)K;
    feat[0] = (float)((double)lambda / (double)mu);
    feat[1] = mu;
    feat[2] = (float)(acc->f_sum_a / k);
    feat[3] = (float)(acc->f_sum_s / k);
    feat[4] = (float)(acc->f_sum_w / k);
    feat[5] = (float)(acc->f_sum_t / k);
    feat[6] = (float)(acc->f_zero / k);
    feat[7] = (float)acc->f_max_w;
    feat[8] = (float)(acc->f_sum_i / k);
    feat[9] = (float)acc->f_last_t;
  }
}

static void mm1_start(mm1_acc *acc, float lambda, float mu) {
  memset(acc, 0, sizeof(*acc));
  acc->es = oracle_variate_mean(mu);
  acc->ea = oracle_variate_mean(lambda);
}

/* out[3] = {mean W, mean T, mean I}; feat[10] written when K > 0, and
 * ctl[8] (nullable) the four controls over n >= K, then over n < K. */
EXPORT int oracle_mm1(uint64_t seed, uint32_t dp, uint32_t rep, uint64_t N, float lambda,
                      float mu, uint64_t K, float out[3], float *feat, double *ctl) {
  if (N == 0 || K > N) return -1;
  mm1_acc acc;
  mm1_start(&acc, lambda, mu);
  float t_prev = 0.0f;
  uint32_t blk[4];
  for (uint64_t n = 0; n < N; ++n) {
    if ((n & 1u) == 0) philox_block(seed, (uint32_t)(n >> 1), dp, rep, TAG_MM1, blk);
    uint32_t j = 2u * (uint32_t)(n & 1u);
    float a = oracle_exp_variate(blk[j], lambda);
    float s = oracle_exp_variate(blk[j + 1], mu);
    mm1_customer(a, s, &t_prev, n, K, &acc, NULL, NULL, NULL);
  }
  mm1_finish(&acc, N, K, lambda, mu, out, feat);
  if (ctl) memcpy(ctl, acc.ctl, sizeof(acc.ctl));
  return 0;
}

/* Test seam: explicit interarrival/service arrays; per-customer W, I, T
 * (any of them may be NULL), the three means and, for a prefix of K
 * customers, the eight controls with the given means es, ea (nullable). */
EXPORT int oracle_mm1_injected(const float *A, const float *S, uint64_t N, uint64_t K, double es,
                               double ea, float *W, float *I, float *T, float out[3],
                               double *ctl) {
  if (N == 0 || K > N) return -1;
  mm1_acc acc;
  memset(&acc, 0, sizeof(acc));
  acc.es = es;
  acc.ea = ea;
  float t_prev = 0.0f;
  for (uint64_t n = 0; n < N; ++n)
    mm1_customer(A[n], S[n], &t_prev, n, K, &acc, W ? W + n : NULL, I ? I + n : NULL,
                 T ? T + n : NULL);
  mm1_finish(&acc, N, 0, 1.0f, 1.0f, out, NULL);
  if (ctl) memcpy(ctl, acc.ctl, sizeof(acc.ctl));
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Drossel-Schwabl forest fire, synchronous, on an L x L torus with the     */
/* 4-neighbourhood. States: 0 empty, 1 tree, 2 burning. Per step every      */
/* cell c = y*L + x reads u = word c&3 of Philox block (t, c>>2, rep,       */
/* TAG_FF); burning -> empty; tree -> burning if a neighbour burns, else if */
/* u < TF; empty -> tree if u < TP. TP = floor(p * 2^32), TF = floor(f *    */
/* 2^32) in fp64. burnt counts tree -> burning transitions.                 */
/* ------------------------------------------------------------------------ */
EXPORT uint32_t oracle_ff_threshold(double prob) {
  double v = floor(prob * 4294967296.0);
  if (v < 0.0) v = 0.0;
  if (v > 4294967295.0) v = 4294967295.0;
  return (uint32_t)v;
}

static int ff_core(uint64_t seed, uint32_t rep, uint32_t L, uint32_t T, uint32_t tp,
                   uint32_t tf, const uint32_t *u_inj, const uint8_t *init, uint8_t *final,
                   int64_t *burnt_out) {
  size_t cells = (size_t)L * L;
  uint8_t *cur = (uint8_t *)malloc(cells), *nxt = (uint8_t *)malloc(cells);
  if (!cur || !nxt) {
    free(cur);
    free(nxt);
    return -1;
  }
  if (init) memcpy(cur, init, cells);
  else memset(cur, 0, cells);
  int64_t burnt = 0;
  uint32_t blk[4];
  for (uint32_t t = 0; t < T; ++t) {
    for (uint32_t y = 0; y < L; ++y) {
      for (uint32_t x = 0; x < L; ++x) {
        uint32_t c = y * L + x;
        uint32_t u;
        if (u_inj) {
          u = u_inj[(size_t)t * cells + c];
        } else {
          philox_block(seed, t, c >> 2, rep, TAG_FF, blk);
          u = blk[c & 3u];
        }
        uint8_t s = cur[c], ns;
        if (s == 2) {
          ns = 0;
        } else if (s == 1) {
          uint32_t xl = (x + L - 1) % L, xr = (x + 1) % L;
          uint32_t yu = (y + L - 1) % L, yd = (y + 1) % L;
          int nb = cur[y * L + xl] == 2 || cur[y * L + xr] == 2 || cur[yu * L + x] == 2 ||
                   cur[yd * L + x] == 2;
          if (nb || u < tf) {
            ns = 2;
            ++burnt;
          } else {
            ns = 1;
          }
        } else {
          ns = (u < tp) ? 1 : 0;
        }
        nxt[c] = ns;
      }
    }
    uint8_t *tmp = cur;
    cur = nxt;
    nxt = tmp;
  }
  if (final) memcpy(final, cur, cells);
  free(cur);
  free(nxt);
  *burnt_out = burnt;
  return 0;
}

EXPORT int oracle_ff(uint64_t seed, uint32_t rep, uint32_t L, uint32_t T, double p, double f,
                     int64_t *burnt) {
  if (L == 0 || (L % 4u) != 0) return -1;
  return ff_core(seed, rep, L, T, oracle_ff_threshold(p), oracle_ff_threshold(f), NULL, NULL,
                 NULL, burnt);
}

/* Test seam: u[t * L*L + c] supplies the uniform of cell c at step t;
 * init (nullable = all empty) and final are L*L state arrays. */
EXPORT int oracle_ff_injected(uint32_t L, uint32_t T, double p, double f, const uint32_t *u,
                              const uint8_t *init, uint8_t *final, int64_t *burnt) {
  if (L == 0) return -1;
  return ff_core(0, 0, L, T, oracle_ff_threshold(p), oracle_ff_threshold(f), u, init, final,
                 burnt);
}

/* Final grid of a Philox-driven run (for debugging parity on small cases). */
EXPORT int oracle_ff_state(uint64_t seed, uint32_t rep, uint32_t L, uint32_t T, double p,
                           double f, uint8_t *final, int64_t *burnt) {
  if (L == 0 || (L % 4u) != 0) return -1;
  return ff_core(seed, rep, L, T, oracle_ff_threshold(p), oracle_ff_threshold(f), NULL, NULL,
                 final, burnt);
}

/* ------------------------------------------------------------------------ */
/* Monte Carlo pi (paper section 5.1, first model): draw points uniformly in */
/* the unit square and count those inside the quarter disc. Point i of      */
/* replication r takes words 2(i&1), 2(i&1)+1 of block (i>>1, 0, r, TAG_PI); */
/* each word's top 24 bits X give the coordinate u = (X + 1/2) 2^-24, so    */
/* the point is inside iff u^2 + v^2 <= 1, i.e. (2X+1)^2 + (2Y+1)^2 <= 2^50, */
/* decided exactly in 64-bit integers. The estimate is 4 hits / N.          */
/* ------------------------------------------------------------------------ */
EXPORT int oracle_pi_inside(uint32_t wx, uint32_t wy) {
  uint64_t a = 2ull * (uint64_t)(wx >> 8) + 1ull;
  uint64_t b = 2ull * (uint64_t)(wy >> 8) + 1ull;
  return a * a + b * b <= (1ull << 50);
}

EXPORT int64_t oracle_pi(uint64_t seed, uint32_t rep, uint64_t points) {
  int64_t hits = 0;
  uint32_t blk[4];
  for (uint64_t i = 0; i < points; ++i) {
    if ((i & 1u) == 0) philox_block(seed, (uint32_t)(i >> 1), 0, rep, TAG_PI, blk);
    uint32_t j = 2u * (uint32_t)(i & 1u);
    hits += oracle_pi_inside(blk[j], blk[j + 1]);
  }
  return hits;
}


/* ------------------------------------------------------------------------ */
/* Second generator (paper section 5: the models draw from L'Ecuyer's       */
/* three-component Tausworthe generator, streams split by Random Spacing).  */
/* taus88 (L'Ecuyer, Math. Comp. 65, 1996): component j keeps a k_j-bit     */
/* state in the top bits of a 32-bit word and advances it s_j steps of the  */
/* recurrence of the trinomial z^k + z^q + 1 at a time; the output is the   */
/* xor of the three words after the step. (k, q, s) = (31, 13, 12),         */
/* (29, 2, 4), (28, 3, 17).                                                  */
/* Random Spacing: the stream of (model, dp, replication) starts from a     */
/* random state, here the words x, y, z of Philox block (model, dp, rep,    */
/* TAG_TAUS_SEED) under the run's seed, each raised by 2, 8 or 16 when its  */
/* k-bit part would be zero. Draw d of a replication is output d of its     */
/* stream. Models: point i of pi uses outputs 2i, 2i+1; customer n of the   */
/* M/M/1 queue uses 2n (interarrival) and 2n+1 (service); move t of walker  */
/* w uses bits 2(t&15) of output w*ceil(T/16) + (t>>4).                      */
/* ------------------------------------------------------------------------ */
static uint32_t taus_component(uint32_t z, int k, int q, int s) {
  uint32_t keep = 0xFFFFFFFFu << (32 - k);
  uint32_t feedback = ((z << q) ^ z) >> (k - s);
  return ((z & keep) << s) ^ feedback;
}

EXPORT uint32_t oracle_taus88_next(uint32_t st[3]) {
  st[0] = taus_component(st[0], 31, 13, 12);
  st[1] = taus_component(st[1], 29, 2, 4);
  st[2] = taus_component(st[2], 28, 3, 17);
  return st[0] ^ st[1] ^ st[2];
}

EXPORT void oracle_taus88_seed(uint64_t seed, uint32_t model, uint32_t dp, uint32_t rep,
                               uint32_t st[3]) {
  uint32_t blk[4];
  philox_block(seed, model, dp, rep, TAG_TAUS_SEED, blk);
  st[0] = blk[0] < 2u ? blk[0] + 2u : blk[0];
  st[1] = blk[1] < 8u ? blk[1] + 8u : blk[1];
  st[2] = blk[2] < 16u ? blk[2] + 16u : blk[2];
}

/* n consecutive outputs from state st (st is advanced). */
EXPORT void oracle_taus88_outputs(uint32_t st[3], uint64_t n, uint32_t *out) {
  for (uint64_t i = 0; i < n; ++i) out[i] = oracle_taus88_next(st);
}

EXPORT int64_t oracle_pi_taus(uint64_t seed, uint32_t rep, uint64_t points) {
  uint32_t st[3];
  oracle_taus88_seed(seed, TAG_PI, 0, rep, st);
  int64_t hits = 0;
  for (uint64_t i = 0; i < points; ++i) {
    uint32_t wx = oracle_taus88_next(st);
    uint32_t wy = oracle_taus88_next(st);
    hits += oracle_pi_inside(wx, wy);
  }
  return hits;
}

EXPORT int oracle_rw_taus(uint64_t seed, uint32_t rep, uint32_t walkers, uint32_t grid,
                          uint32_t steps, int64_t *ssd, int64_t *distinct,
                          int64_t *walker_sites) {
  uint8_t *dirs = (uint8_t *)malloc((size_t)walkers * steps + 1);
  if (!dirs) return -1;
  uint32_t st[3];
  oracle_taus88_seed(seed, TAG_RW, 0, rep, st);
  uint32_t per_walker = (steps + 15u) / 16u;
  for (uint32_t w = 0; w < walkers; ++w) {
    for (uint32_t j = 0; j < per_walker; ++j) {
      uint32_t word = oracle_taus88_next(st);
      for (uint32_t t = 16u * j; t < steps && t < 16u * j + 16u; ++t)
        dirs[(size_t)w * steps + t] = (uint8_t)((word >> (2u * (t & 15u))) & 3u);
    }
  }
  int rc = rw_core(0, 0, walkers, grid, steps, dirs, ssd, distinct, walker_sites);
  free(dirs);
  return rc;
}

EXPORT int oracle_mm1_taus(uint64_t seed, uint32_t dp, uint32_t rep, uint64_t N, float lambda,
                           float mu, uint64_t K, float out[3], float *feat, double *ctl) {
  if (N == 0 || K > N) return -1;
  mm1_acc acc;
  mm1_start(&acc, lambda, mu);
  float t_prev = 0.0f;
  uint32_t st[3];
  oracle_taus88_seed(seed, TAG_MM1, dp, rep, st);
  for (uint64_t n = 0; n < N; ++n) {
    float a = oracle_exp_variate(oracle_taus88_next(st), lambda);
    float s = oracle_exp_variate(oracle_taus88_next(st), mu);
    mm1_customer(a, s, &t_prev, n, K, &acc, NULL, NULL, NULL);
  }
  mm1_finish(&acc, N, K, lambda, mu, out, feat);
  if (ctl) memcpy(ctl, acc.ctl, sizeof(acc.ctl));
  return 0;
}
