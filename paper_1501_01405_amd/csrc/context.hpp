// The library context behind the opaque mrip_ctx handle: parameters, launch
// shape and every device buffer the context owns.
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>
#include <string>
#include <vector>

#include "../../include/mrip.h"

namespace mrip {

// A device allocation owned by the context; grows on demand, freed with it.
struct DevBuf {
  void *p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf &) = delete;
  DevBuf &operator=(const DevBuf &) = delete;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
  hipError_t ensure(size_t n) {
    if (n <= bytes && p) return hipSuccess;
    if (p) {
      // work queued earlier may still use the old buffer
      const hipError_t e = hipDeviceSynchronize();
      if (e != hipSuccess) return e;
      (void)hipFree(p);
      p = nullptr;
      bytes = 0;
    }
    hipError_t e = hipMalloc(&p, n ? n : 1);
    if (e == hipSuccess) bytes = n;
    return e;
  }
  template <class T>
  T *as() const {
    return (T *)p;
  }
};

// RUN_PLAN_PARTIAL: a plan run stopped by the item limit; its outputs and
// done flags are readable, its statistics were not computed.
enum RunKind { RUN_NONE = 0, RUN_UNIFORM = 1, RUN_PLAN = 2, RUN_PLAN_PARTIAL = 3 };

// An item table on the device (structure of arrays) with its queue order
// (longest first) and its grouping by design point (index + offsets).
struct ItemBufs {
  DevBuf dp, rep, n, lambda, mu, order, index, offsets;
  uint64_t count = 0, max_customers = 0, n_long = 0, total_customers = 0;
  std::vector<uint32_t> dp_ids;          // distinct design points, ascending
  std::vector<uint64_t> group_offsets;   // host copy of offsets
  std::vector<uint32_t> index_host;      // host copy of index
};

// State of the learned control variate.
struct CvState {
  bool trained = false, applied = false;
  DevBuf theta, adam_m, adam_v, partial, loss_hist;
  DevBuf image;  // the weights' bf16 image the gradient kernel stages (Adam keeps it current)
  DevBuf queue, norm, colstats, unit4;
  std::vector<float> mean, std_;  // feature mean / std of the training set
  // MRIP_CV_BETA_BINS rows of MRIP_CV_COEFS coefficients over [rho_lo, rho_hi]
  // (the network's control h, then the four prefix controls), and on the device
  std::vector<float> coef;
  DevBuf coef_d;
  float rho_lo = 0.f, rho_hi = 1.f;
  float final_loss = 0.f, train_ms = 0.f;
  int bin_of(float rho) const {
    const float u = (rho - rho_lo) / (rho_hi - rho_lo) * (float)MRIP_CV_BETA_BINS;
    const int k = (int)std::floor(u);
    return k < 0 ? 0 : k >= MRIP_CV_BETA_BINS ? MRIP_CV_BETA_BINS - 1 : k;
  }
  // training: Y, features, controls and multipliers per item (item order),
  // the standardised target, and the rows in training order (fit rows,
  // then the held-out ones, grouped by design point): perm[j] is the item
  // of row j; network outputs g_train in item order after training
  ItemBufs train_items;
  DevBuf y_train, x_train, c_train, z_train, t_train, zt_train, g_rows, g_train, group;
  DevBuf xn, yn, zn, scratch_t, scratch_i;
  std::vector<uint32_t> perm;
  uint64_t n_fit = 0;
  // application: per item Y, features, controls, network outputs, the
  // network's control h, residual d = Y - coef . (h, z_pre) and the item's
  // bin of rho
  ItemBufs items;
  DevBuf y, x, c, g, h, d, bin_item, red_y, red_d;
  // per design point of the last apply: cv = (n, mean, var of the
  // estimator, dof, coefficient of h used), plain = (n, mean, var of Y)
  std::vector<uint32_t> dp_ids;
  std::vector<double> cv, plain;
  float run_ms = 0.f, infer_ms = 0.f;
};

// Wavefronts per long item for a plan run whose longest item has `longest`
// customers out of `total`: as fixed by mrip_set_plan_split or the
// autotuner, else the fewest (up to plan_split) that bring the longest
// item's share down to the run's average work per wavefront the chip holds
// at once. Splitting shortens a plan only while its longest item sets the
// makespan; beyond that its corrections and barriers cost time.
uint32_t plan_split_for(mrip_ctx ctx, uint64_t longest, uint64_t total);

}  // namespace mrip

struct mrip_ctx_s {
  mrip_model model;
  mrip_mapping mapping;
  mrip_rw_params rw;
  mrip_mm1_params mm1;
  mrip_ff_params ff;
  mrip_pi_params pi;
  uint32_t rpw = 1, wg = 256;
  uint32_t split = 1;  // wavefronts per M/M/1 replication in mrip_run
  // the plans' shape: mrip_set_shape sets it with the runs' one, the
  // autotuner alone (it never touches the runs' shape)
  uint32_t plan_rpw = 1, plan_wg = 256;
  // plans: wavefronts per long item (1 = none) and what counts as long;
  // until mrip_set_plan_split or the autotuner fixes it, plan_split is the
  // most a run uses (plan_split_for)
  uint32_t plan_split = 8;
  uint64_t long_min = 65536;
  bool plan_split_set = false;
  uint32_t cus = 0;  // compute units of the device (queried on first use)
  // stream source of mrip_run (MRIP_RNG_*) and, for taus88, its jump tables
  int rng = MRIP_RNG_PHILOX;
  mrip::DevBuf taus_tables;

  // Outputs per run: up to three scalar outputs (idx 0..2) and, for M/M/1
  // runs with a feature prefix, the features (idx 3, 10 per replication)
  // and the controls (idx 4, 8 per replication).
  static constexpr uint32_t MAX_OUT = 5;
  // Two sets of output buffers: a uniform run writes one while the
  // reduction of the run before it, on red_stream, still reads the other.
  mrip::DevBuf out[2][MAX_OUT];
  uint32_t next_set = 0;                 // output set of the next uniform run
  bool set_pending[2] = {};              // a reduction may still read set i
  hipEvent_t ev_set_free[2] = {};        // recorded after that reduction
  hipStream_t red_stream = nullptr;      // the library's stream for reductions
  // caller-owned output buffers (mrip_bind_output) and the buffers the last
  // run wrote (bound or owned)
  struct Bound {
    void *p = nullptr;
    uint64_t bytes = 0;
  } bound[MAX_OUT];
  void *cur[MAX_OUT] = {};
  mrip::DevBuf scratch;
  mrip::DevBuf walker_scratch;  // the walk's per-walker bitmaps
  mrip::DevBuf taus_walk;       // the walk's taus88 jump tables (its steps are fixed)
  mrip::DevBuf taus_run;        // the M/M/1 runs' taus88 jump tables (customers are fixed)
  // (n, mean, var) per scalar output: pinned host memory written by the
  // reduction kernel through its device view
  // A ring of STATS_RING slots, one per run, so a caller may read run k's
  // statistics after enqueuing run k + 1.
  static constexpr uint32_t STATS_RING = 4, STATS_SLOT = 12;  // doubles per slot
  double *stats_host = nullptr, *stats_view = nullptr;
  hipEvent_t ev_stats[STATS_RING] = {};  // recorded after each slot's reduction
  uint64_t stats_runs = 0;               // reductions enqueued so far
  mrip::RunKind last = mrip::RUN_NONE;
  uint64_t last_n = 0;
  // the stream of the last launching call, and the last event that call
  // recorded on it, after everything it enqueued there (a call on another
  // stream waits for it first)
  hipStream_t last_stream = nullptr;
  hipEvent_t done_ev = nullptr;
  // set when that call recorded no event after its work (a run whose
  // statistics are deferred): a call on another stream then records one on
  // last_stream first (switch_ev)
  bool last_unmarked = false;
  hipEvent_t switch_ev = nullptr;
  // Deferred statistics: a uniform run in the split headline form leaves
  // its reduction to the next such run on the same stream, whose kernel
  // reduces it in one extra workgroup, so no event or reduction launch sits
  // between consecutive simulation kernels; any other call launches the
  // reduction first (flush_pending).
  struct Pending {
    bool active = false;
    hipStream_t stream = nullptr;
    uint32_t set = 0;          // the output set it wrote
    uint64_t n = 0;            // its replications
    uint64_t stats_index = 0;  // its place in the statistics ring
  } pend;
  // per ring slot: the statistics are signalled by a sequence number the
  // reducing kernel stores (seq_host[slot] >= stats index + 1) on
  // seq_stream[slot], instead of by ev_stats[slot]
  bool slot_by_seq[STATS_RING] = {};
  hipStream_t seq_stream[STATS_RING] = {};
  uint64_t *seq_host = nullptr, *seq_view = nullptr;
  // time one simulation launch in timing_every with HIP events (0 = none)
  uint32_t timing_every = 1;
  uint64_t timing_count = 0;
  // event pairs of the last RING simulation-kernel launches (run history)
  static constexpr uint32_t RING = 256;
  hipEvent_t ring0[RING] = {}, ring1[RING] = {};
  uint64_t launches = 0;
  std::string err;

  // plan
  uint64_t n_items = 0, n_long = 0;
  std::vector<uint64_t> lpt_customers;  // customers in longest-first order
  std::vector<uint32_t> lpt_order;      // item indices in longest-first order
  mrip::DevBuf resume_order;            // the queue of a resumed plan
  mrip::DevBuf item_done;               // per item: 1 once the last plan run wrote its outputs
  uint64_t plan_limit = 0;              // plan runs stop after this many items (0 = none)
  mrip::DevBuf it_dp, it_rep, it_n, it_lambda, it_mu, it_order, queue, dp_index, dp_offsets,
      dp_stats;
  std::vector<uint32_t> dp_ids;

  // learned control variate
  mrip::CvState cv;

  ~mrip_ctx_s() {
    if (stats_host) (void)hipHostFree(stats_host);
    if (seq_host) (void)hipHostFree(seq_host);
    if (switch_ev) (void)hipEventDestroy(switch_ev);
    for (uint32_t i = 0; i < STATS_RING; ++i)
      if (ev_stats[i]) (void)hipEventDestroy(ev_stats[i]);
    for (uint32_t i = 0; i < 2; ++i)
      if (ev_set_free[i]) (void)hipEventDestroy(ev_set_free[i]);
    if (red_stream) (void)hipStreamDestroy(red_stream);
    for (uint32_t i = 0; i < RING; ++i) {
      if (ring0[i]) (void)hipEventDestroy(ring0[i]);
      if (ring1[i]) (void)hipEventDestroy(ring1[i]);
    }
  }
};
