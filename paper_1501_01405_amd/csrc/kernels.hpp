// Host-side launchers of the MRIP kernels (one .hip file per model). Every
// launcher only enqueues on `stream`; shapes are validated by the caller
// (api.cpp) before any launch.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mrip {

// Stream source of a run: counter-based Philox (default) or taus88 with
// Random Spacing (taus.hpp); `taus` points to the device jump tables.
enum Rng : int { RNG_PHILOX = 0, RNG_TAUS88 = 1 };

// Outputs to reduce: x[o] holds n values of dtype[o] (0 = int32, 1 = fp32).
struct ReduceSet {
  const void *x[4];
  int dtype[4];
};

// ------------------------------------------------------------ random walk
struct RwArgs {
  uint64_t seed;
  uint32_t walkers, grid, steps;
  uint64_t n_reps;
  int32_t *ssd, *distinct;
  uint32_t *scratch_bitmaps;  // SIMT only: n_reps * grid*grid/32 words
  int rng;
  const uint32_t *taus;
  const uint32_t *taus_walk;  // taus88: the walk's jump tables (taus_build_walk_tables)
  // per-walker site counts (nullptr = off): output and the walkers' own
  // bitmaps (WAVE: n_reps * walkers * grid*grid/32 words, SIMT: n_reps *
  // grid*grid/32)
  int32_t *walker_sites;
  uint32_t *walker_bitmaps;
  // replication id of output 0: outputs and bitmaps are indexed from 0,
  // random streams by rep0 + index
  uint64_t rep0;
};
// device bytes of per-walker bitmaps one WAVE launch may use
constexpr uint64_t WALKER_SCRATCH_MAX = 1ull << 30;
hipError_t launch_rw_wave(const RwArgs &a, uint32_t workgroup, hipStream_t s);
// one_lane: one working lane per wavefront (the paper's WLP form)
hipError_t launch_rw_simt(const RwArgs &a, bool one_lane, hipStream_t s);

// ------------------------------------------------------------ M/M/1
// Per-item parameters in structure-of-arrays form on the device.
struct Mm1Items {
  const uint32_t *dp, *rep;
  const uint64_t *customers;
  const float *lambda, *mu;
  const uint32_t *order;  // queue order (longest first); index into the arrays
};
struct Mm1Args {
  uint64_t seed;
  uint64_t n_reps;              // uniform mode: replications 0..n_reps-1
  float lambda, mu;             // uniform mode
  uint64_t customers;           // uniform mode
  uint64_t feature_prefix;      // K (0 = no features)
  Mm1Items items;               // plan mode (items.dp != nullptr)
  uint32_t *queue_head;         // plan mode: device counter, zero at launch
  float *mean_w, *mean_t, *mean_i;
  float *features;              // n x 10 when feature_prefix > 0
  // n x 8 when feature_prefix > 0: the martingale controls over customers
  // n >= K, sum (S_n - es), sum (A_n - ea), sum T_{n-1} (S_n - es),
  // sum T_{n-1} (A_n - ea), then the same four over n < K, with es, ea the
  // variates' means in fp32. The launchers fill in ea, es (uniform mode)
  // and log_grid_mean (plans derive each item's means from it).
  float *controls;
  float ea, es;
  double log_grid_mean;
  int rng;                      // uniform mode only; plans use Philox
  const uint32_t *taus;
  // Split kernels of 256-thread workgroups (uniform mode): with prev_n > 0
  // one extra workgroup reduces the previous run's three fp32 outputs
  // (prev_n replications each) into prev_out, 3 x (n, mean, variance) as
  // the reduction kernel writes them, then stores prev_seq_value to
  // *prev_seq (host-visible) once they are visible.
  const float *prev_x[3];
  uint64_t prev_n;
  double *prev_out;
  uint64_t *prev_seq;
  uint64_t prev_seq_value;
  uint8_t *done;                // plan mode (nullable): done[i] = 1 once item i's outputs are written
  const uint32_t *taus_run;     // taus88: the runs' jump tables (taus_build_run_tables)
};
// Mean of -ln u over the 24-bit grid of u, {k 2^-24 : k = 1..2^24}, and
// the fp32 mean of the exponential variate of `rate` as drawn, (float)(1 /
// rate) times it: the controls' centring constants.
double log_grid_mean();
float variate_mean_f32(float rate);
hipError_t launch_mm1_wave(const Mm1Args &a, uint32_t reps_per_wave, uint32_t workgroup,
                           hipStream_t s);
hipError_t launch_mm1_simt(const Mm1Args &a, bool one_lane, hipStream_t s);
// taus88 streams, WAVE mapping: lanes_per_rep (16, 32, 64, 128 or 256)
// lanes per replication, each on a contiguous run of its customers.
hipError_t launch_mm1_taus(const Mm1Args &a, uint32_t lanes_per_rep, hipStream_t s);
// WAVE mapping with each replication split over 2 or 4 wavefronts of a
// 256-thread workgroup (speculate from carry 0, then correct in order).
// Events a kernel launch records around the kernel itself (start, stop).
struct KernelEvents {
  hipEvent_t start, stop;
};
// ev (nullable, Philox only): the kernel records ev->start and ev->stop
hipError_t launch_mm1_split(const Mm1Args &a, uint32_t waves_per_rep, hipStream_t s,
                            const KernelEvents *ev = nullptr);
// Persistent plan kernel: grid sized to full residency, waves pop work.
// plan in the SIMT (one_lane = false) or one-working-lane form
hipError_t launch_mm1_plan_simt(const Mm1Args &a, uint64_t n_items, bool one_lane, hipStream_t s);
hipError_t launch_mm1_plan(const Mm1Args &a, uint64_t n_items, uint32_t reps_per_wave,
                           uint32_t workgroup, hipStream_t s);
// Plan kernel whose first n_long items (longest first) are each split over
// waves_per_rep (2 or 4) wavefronts of a 256-thread workgroup; the rest go
// rpw per wavefront. queue_head[0..1] must be zero at launch.
hipError_t launch_mm1_plan_split(const Mm1Args &a, uint64_t n_items, uint64_t n_long,
                                 uint32_t waves_per_rep, uint32_t rpw, hipStream_t s);
// Zero the queue head with a one-thread kernel (no memset node in graphs).
hipError_t launch_zero_u32(uint32_t *p, uint32_t n, hipStream_t s);

// ------------------------------------------------------------ forest fire
struct FfArgs {
  uint64_t seed;
  uint32_t grid, steps;
  uint32_t tp, tf;  // integer thresholds for growth and lightning
  uint64_t n_reps;
  int32_t *burnt;
  uint32_t *state;  // SIMT only: 2 planes * grid rows * grid/32 words * n_reps
};
hipError_t launch_ff_wave(const FfArgs &a, uint32_t workgroup, hipStream_t s);
hipError_t launch_ff_simt(const FfArgs &a, bool one_lane, hipStream_t s);

// ------------------------------------------------------------ Monte Carlo pi
struct PiArgs {
  uint64_t seed;
  uint64_t points;  // per replication, < 2^31
  uint64_t n_reps;
  int32_t *hits;
  float *estimate;  // 4 hits / points
  int rng;
  const uint32_t *taus;
};
hipError_t launch_pi_wave(const PiArgs &a, uint32_t workgroup, hipStream_t s);
hipError_t launch_pi_simt(const PiArgs &a, bool one_lane, hipStream_t s);

// ------------------------------------------------------------ reductions
// out[3*g + {0,1,2}] = (n, mean, unbiased var) in fp64 over segment g of x;
// segment g is x[offsets[g] .. offsets[g+1]) (offsets nullptr: one segment
// of n values). dtype 0 = int32, 1 = fp32.
hipError_t launch_reduce_f64(const void *x, int dtype, uint64_t n, const uint64_t *offsets,
                             uint32_t n_segments, double *out, hipStream_t s);
// Several outputs of n values each in one launch (one workgroup each):
// out[3*o + {0,1,2}] for output o (ReduceSet is declared above).
hipError_t launch_reduce_f64_multi(const ReduceSet &set, uint32_t n_outputs, uint64_t n,
                                   double *out, hipStream_t s);
// Gathered variant: segment g reads x[index[offsets[g] .. offsets[g+1])].
// The pair form reduces two fp32 arrays over the same segments in one launch.
hipError_t launch_reduce_f64_gather(const void *x, int dtype, const uint32_t *index,
                                    const uint64_t *offsets, uint32_t n_segments, double *out,
                                    hipStream_t s);
hipError_t launch_reduce_f64_gather2(const float *x0, const float *x1, const uint32_t *index,
                                     const uint64_t *offsets, uint32_t n_segments, double *out0,
                                     double *out1, hipStream_t s);

// ------------------------------------------------------------ utilities
// out[i] = output skip + i of the taus88 stream of (model, dp, rep), each
// reached by its own jump from the stream's start (tests the jump tables).
hipError_t launch_taus_dump(uint64_t seed, uint32_t model, uint32_t dp, uint32_t rep, uint64_t skip,
                            uint64_t n, const uint32_t *tables, uint32_t *out, hipStream_t s);
hipError_t launch_philox_dump(uint64_t seed, const uint32_t *ctr, uint64_t n, uint32_t *out,
                              hipStream_t s);

}  // namespace mrip
