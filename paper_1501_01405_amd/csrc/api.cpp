// C ABI of the MRIP library (include/mrip.h): argument checks, device
// buffers owned by the context, kernel launches and the host-side end of
// the statistics. No C++ exception crosses the boundary.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "../../include/mrip.h"
#include "context.hpp"
#include "kernels.hpp"
#include "taus.hpp"

namespace mrip {
double t_quantile(double p, double nu);
}

using namespace mrip;

namespace {

mrip_status hip_fail(mrip_ctx c, hipError_t e, const char *what) {
  if (c) {
    c->err = std::string(what) + ": " + hipGetErrorString(e);
  }
  return MRIP_E_HIP;
}

mrip_status inval(mrip_ctx c, const char *why) {
  if (c) c->err = why;
  return MRIP_E_INVAL;
}

#define HIP_TRY(ctx, expr)                                   \
  do {                                                       \
    hipError_t _e = (expr);                                  \
    if (_e != hipSuccess) return hip_fail((ctx), _e, #expr); \
  } while (0)

// Let single-kernel runs record their timing events from the kernel's own
// dispatch (hipExtLaunchKernelGGL) instead of separate stream markers.
constexpr bool kSelfTimedLaunch = true;

uint32_t scalar_outputs(mrip_ctx c) {
  const mrip_model m = c->model;
  return m == MRIP_RW ? (c->rw.walker_sites ? 3 : 2) : m == MRIP_MM1 ? 3 : m == MRIP_PI ? 2 : 1;
}

// Values per replication of vector output o (M/M/1 with a feature prefix:
// 3 = the 10 features, 4 = the 8 controls); 0 when o is no vector output.
uint32_t vector_width(mrip_ctx c, uint32_t o) {
  if (c->model != MRIP_MM1) return 0;
  return o == 3 ? 10u : o == 4 ? 8u : 0u;
}

// dtype of scalar output o for the reduction kernel: 0 = int32, 1 = fp32
int output_dtype(mrip_model m, uint32_t o) {
  return m == MRIP_MM1 ? 1 : (m == MRIP_PI && o == 1) ? 1 : 0;
}

bool is_pow2_grid(uint32_t g) { return g == 16 || g == 32 || g == 64 || g == 128; }

mrip_mapping effective(mrip_mapping m) {
  return (m == MRIP_MAP_SIMT || m == MRIP_MAP_LANE0) ? m : MRIP_MAP_WAVE;
}

uint32_t ff_threshold(double prob) {
  double v = std::floor(prob * 4294967296.0);
  if (v < 0.0) v = 0.0;
  if (v > 4294967295.0) v = 4294967295.0;
  return (uint32_t)v;
}

// The run's statistics land in pinned host memory that the reduction
// kernel writes directly (no copy launch), one ring slot per run; reading
// them waits for that slot's event.
mrip_status ensure_events(mrip_ctx c) {
  for (uint32_t i = 0; i < mrip_ctx_s::STATS_RING; ++i)
    if (!c->ev_stats[i])
      HIP_TRY(c, hipEventCreateWithFlags(&c->ev_stats[i], hipEventDisableTiming));
  for (uint32_t i = 0; i < 2; ++i)
    if (!c->ev_set_free[i])
      HIP_TRY(c, hipEventCreateWithFlags(&c->ev_set_free[i], hipEventDisableTiming));
  if (!c->red_stream) HIP_TRY(c, hipStreamCreateWithFlags(&c->red_stream, hipStreamNonBlocking));
  if (!c->stats_host) {
    const size_t bytes = sizeof(double) * mrip_ctx_s::STATS_RING * mrip_ctx_s::STATS_SLOT;
    HIP_TRY(c, hipHostMalloc((void **)&c->stats_host, bytes, hipHostMallocMapped));
    HIP_TRY(c, hipHostGetDevicePointer((void **)&c->stats_view, c->stats_host, 0));
  }
  if (!c->seq_host) {
    HIP_TRY(c, hipHostMalloc((void **)&c->seq_host, sizeof(uint64_t) * mrip_ctx_s::STATS_RING,
                             hipHostMallocMapped));
    for (uint32_t i = 0; i < mrip_ctx_s::STATS_RING; ++i) c->seq_host[i] = 0;
    HIP_TRY(c, hipHostGetDevicePointer((void **)&c->seq_view, c->seq_host, 0));
  }
  if (!c->switch_ev) HIP_TRY(c, hipEventCreateWithFlags(&c->switch_ev, hipEventDisableTiming));
  return MRIP_OK;
}

// Device view of the next run's statistics slot.
double *next_stats_slot(mrip_ctx c) {
  const uint32_t slot = (uint32_t)(c->stats_runs % mrip_ctx_s::STATS_RING);
  return c->stats_view + (size_t)slot * mrip_ctx_s::STATS_SLOT;
}

// Before a run on stream s writes output set `set`: wait for the reduction
// that may still be reading it.
mrip_status claim_set(mrip_ctx c, uint32_t set, hipStream_t s) {
  if (!c->set_pending[set]) return MRIP_OK;
  // a reduction already finished needs no wait packet on the run's stream
  const hipError_t q = hipEventQuery(c->ev_set_free[set]);
  if (q == hipSuccess) {
    c->set_pending[set] = false;
    return MRIP_OK;
  }
  if (q != hipErrorNotReady) return hip_fail(c, q, "hipEventQuery(ev_set_free)");
  (void)hipGetLastError();  // "not ready" is an answer, not a failure to keep
  HIP_TRY(c, hipStreamWaitEvent(s, c->ev_set_free[set], 0));
  return MRIP_OK;
}

// Mark the slot written by the reduction just enqueued on s.
mrip_status commit_stats_slot(mrip_ctx c, hipStream_t s) {
  const uint32_t slot = (uint32_t)(c->stats_runs % mrip_ctx_s::STATS_RING);
  HIP_TRY(c, hipEventRecord(c->ev_stats[slot], s));
  c->slot_by_seq[slot] = false;
  ++c->stats_runs;
  return MRIP_OK;
}

// Work enqueued on another stream than the last call's first waits, on the
// device, for everything that call enqueued on its stream: the context's
// buffers (device queue, scratch, outputs) serve one call at a time. Every
// launching call makes this its first enqueue and ends with mark_done,
// naming the last event it recorded on its stream (no extra packet between
// consecutive runs on one stream).
mrip_status order_after_last(mrip_ctx c, hipStream_t s) {
  if (s == c->last_stream) return MRIP_OK;
  if (c->last_unmarked) {
    // everything enqueued on last_stream so far
    HIP_TRY(c, hipEventRecord(c->switch_ev, c->last_stream));
    HIP_TRY(c, hipStreamWaitEvent(s, c->switch_ev, 0));
  } else if (c->done_ev) {
    HIP_TRY(c, hipStreamWaitEvent(s, c->done_ev, 0));
  }
  return MRIP_OK;
}

void mark_done(mrip_ctx c, hipStream_t s, hipEvent_t last_on_s) {
  c->done_ev = last_on_s;
  c->last_stream = s;
  c->last_unmarked = false;
}

// The call enqueued work on s after its last event (or recorded none).
void mark_unmarked(mrip_ctx c, hipStream_t s) {
  c->done_ev = nullptr;
  c->last_stream = s;
  c->last_unmarked = true;
}

// Launch the deferred reduction of the last uniform run on its stream (no
// later run of the same form on that stream will carry it) and signal its
// statistics slot by event, as a run that reduces at once does.
mrip_status flush_pending(mrip_ctx c) {
  if (!c->pend.active) return MRIP_OK;
  const mrip_ctx_s::Pending p = c->pend;
  c->pend.active = false;
  ReduceSet rs{};
  for (uint32_t o = 0; o < 3; ++o) {
    rs.x[o] = c->out[p.set][o].p;
    rs.dtype[o] = 1;
  }
  const uint32_t slot = (uint32_t)(p.stats_index % mrip_ctx_s::STATS_RING);
  HIP_TRY(c, launch_reduce_f64_multi(rs, 3, p.n,
                                     c->stats_view + (size_t)slot * mrip_ctx_s::STATS_SLOT, p.stream));
  HIP_TRY(c, hipEventRecord(c->ev_stats[slot], p.stream));
  c->slot_by_seq[slot] = false;
  // the pending run was the last call's (any call flushes before its own work)
  mark_done(c, p.stream, c->ev_stats[slot]);
  return MRIP_OK;
}

// Wait for the statistics a kernel publishes by sequence number: poll the
// slot's number in pinned memory; a stream that has drained without
// publishing it, or reports an error, ends the wait with an error.
mrip_status wait_seq(mrip_ctx c, uint32_t slot, uint64_t value) {
  for (uint32_t spin = 1;; ++spin) {
    if (__atomic_load_n(c->seq_host + slot, __ATOMIC_ACQUIRE) >= value) return MRIP_OK;
    if ((spin & 255) == 0) {
      const hipError_t q = hipStreamQuery(c->seq_stream[slot]);
      if (q == hipSuccess) {
        if (__atomic_load_n(c->seq_host + slot, __ATOMIC_ACQUIRE) >= value) return MRIP_OK;
        c->err = "a run's statistics were not published";
        return MRIP_E_HIP;
      }
      if (q != hipErrorNotReady) return hip_fail(c, q, "hipStreamQuery");
      (void)hipGetLastError();  // "not ready" is an answer, not a failure to keep
      std::this_thread::yield();
    }
  }
}

// The last run-history and statistics events recorded.
hipEvent_t last_ring_event(mrip_ctx c) {
  return c->ring1[(c->launches - 1) % mrip_ctx_s::RING];
}
hipEvent_t last_stats_event(mrip_ctx c) {
  return c->ev_stats[(c->stats_runs - 1) % mrip_ctx_s::STATS_RING];
}

// Events bracketing one simulation-kernel launch: the next slot of the
// run-history ring (the last run's pair is the slot before `launches`).
// `markers`: record the pair as separate stream markers; otherwise the one
// kernel of the launch records them itself (KernelEvents), which saves two
// packets between consecutive runs.
mrip_status record_begin(mrip_ctx c, hipStream_t s, bool markers = true) {
  const uint32_t slot = (uint32_t)(c->launches % mrip_ctx_s::RING);
  if (!c->ring0[slot]) HIP_TRY(c, hipEventCreate(&c->ring0[slot]));
  if (!c->ring1[slot]) HIP_TRY(c, hipEventCreate(&c->ring1[slot]));
  if (markers) HIP_TRY(c, hipEventRecord(c->ring0[slot], s));
  return MRIP_OK;
}

// The events the next launch's kernel records around itself.
KernelEvents kernel_events(mrip_ctx c) {
  const uint32_t slot = (uint32_t)(c->launches % mrip_ctx_s::RING);
  return KernelEvents{c->ring0[slot], c->ring1[slot]};
}

mrip_status record_end(mrip_ctx c, hipStream_t s, bool markers = true) {
  const uint32_t slot = (uint32_t)(c->launches % mrip_ctx_s::RING);
  if (markers) HIP_TRY(c, hipEventRecord(c->ring1[slot], s));
  ++c->launches;
  return MRIP_OK;
}

// Kernel milliseconds of the context's last simulation launch.
mrip_status last_launch_ms(mrip_ctx c, float *ms) {
  if (c->launches == 0) return (c->err = "no timed launch yet"), MRIP_E_STATE;
  const uint32_t slot = (uint32_t)((c->launches - 1) % mrip_ctx_s::RING);
  HIP_TRY(c, hipEventSynchronize(c->ring1[slot]));
  HIP_TRY(c, hipEventElapsedTime(ms, c->ring0[slot], c->ring1[slot]));
  return MRIP_OK;
}

// Device buffer for output o of a run over n items: the caller's bound
// buffer when there is one (it must hold `need` bytes), else the context's
// buffer of output set `set`.
mrip_status output_buffer(mrip_ctx c, uint32_t set, uint32_t o, uint64_t need, void **p) {
  if (c->bound[o].p) {
    if (c->bound[o].bytes < need) {
      c->err = "bound output " + std::to_string(o) + " is smaller than the run's output";
      return MRIP_E_INVAL;
    }
    *p = c->bound[o].p;
  } else {
    HIP_TRY(c, c->out[set][o].ensure(need));
    *p = c->out[set][o].p;
  }
  c->cur[o] = *p;
  return MRIP_OK;
}

mrip_status finish_stats(const double *nmv, double confidence, mrip_stats_t *out) {
  const uint64_t n = (uint64_t)nmv[0];
  if (n < 2) return MRIP_E_TOO_FEW;
  out->n = n;
  out->mean = nmv[1];
  out->var = nmv[2];
  out->confidence = confidence;
  out->t_quantile = mrip::t_quantile(0.5 + 0.5 * confidence, (double)(n - 1));
  out->half_width = out->t_quantile * std::sqrt(nmv[2] / (double)n);
  return MRIP_OK;
}

// Plans and the control variate draw from Philox only.
mrip_status philox_only(mrip_ctx c) {
  if (c->rng != MRIP_RNG_PHILOX)
    return (c->err = "plans and the control variate use Philox streams"), MRIP_E_UNSUPPORTED;
  return MRIP_OK;
}

mrip_status upload_taus_tables(mrip_ctx c) {
  if (!c->taus_tables.p) {
    std::vector<uint32_t> host((size_t)TAUS_TABLES * TAUS_COLS);
    taus_build_tables(host.data());
    HIP_TRY(c, c->taus_tables.ensure(host.size() * sizeof(uint32_t)));
    HIP_TRY(c, hipMemcpy(c->taus_tables.p, host.data(), host.size() * sizeof(uint32_t),
                         hipMemcpyHostToDevice));
  }
  if (c->model == MRIP_MM1 && !c->taus_run.p) {
    // each lane of an M/M/1 replication reaches its run with one table per
    // set bit of its index
    std::vector<uint32_t> host((size_t)TAUS_RUN_TABLES * TAUS_COLS);
    taus_build_run_tables(c->mm1.customers, host.data());
    HIP_TRY(c, c->taus_run.ensure(host.size() * sizeof(uint32_t)));
    HIP_TRY(c, hipMemcpy(c->taus_run.p, host.data(), host.size() * sizeof(uint32_t),
                         hipMemcpyHostToDevice));
  }
  if (c->model == MRIP_RW && !c->taus_walk.p) {
    // the walk's lanes reach their place with one table per level
    std::vector<uint32_t> host((size_t)TAUS_WALK_TABLES * TAUS_COLS);
    taus_build_walk_tables(c->rw.steps, host.data());
    HIP_TRY(c, c->taus_walk.ensure(host.size() * sizeof(uint32_t)));
    HIP_TRY(c, hipMemcpy(c->taus_walk.p, host.data(), host.size() * sizeof(uint32_t),
                         hipMemcpyHostToDevice));
  }
  return MRIP_OK;
}

mrip_status validate(mrip_model model, const void *params, mrip_mapping map, std::string &why) {
  if (!params) return why = "params is NULL", MRIP_E_INVAL;
  if (map != MRIP_MAP_AUTO && map != MRIP_MAP_SIMT && map != MRIP_MAP_WAVE &&
      map != MRIP_MAP_LANE0)
    return why = "unknown mapping", MRIP_E_INVAL;
  if (model == MRIP_RW) {
    const mrip_rw_params *p = (const mrip_rw_params *)params;
    if (p->size != sizeof(mrip_rw_params)) return why = "mrip_rw_params.size mismatch", MRIP_E_INVAL;
    if (p->walkers < 1 || p->walkers > 64) return why = "walkers must be in 1..64", MRIP_E_INVAL;
    if (!is_pow2_grid(p->grid)) return why = "grid must be 16, 32, 64 or 128", MRIP_E_INVAL;
    if ((double)p->walkers * (double)p->steps * (double)p->steps >= 2147483648.0)
      return why = "walkers * steps^2 must be < 2^31", MRIP_E_INVAL;
    if (p->walker_sites > 1) return why = "walker_sites must be 0 or 1", MRIP_E_INVAL;
    return MRIP_OK;
  }
  if (model == MRIP_MM1) {
    const mrip_mm1_params *p = (const mrip_mm1_params *)params;
    if (p->size != sizeof(mrip_mm1_params)) return why = "mrip_mm1_params.size mismatch", MRIP_E_INVAL;
    if (!(p->lambda > 0.0f) || !(p->mu > 0.0f) || !std::isfinite(p->lambda) || !std::isfinite(p->mu))
      return why = "lambda and mu must be finite and > 0", MRIP_E_INVAL;
    if (p->customers < 1 || p->customers >= (1ull << 33))
      return why = "customers must be in [1, 2^33)", MRIP_E_INVAL;
    if (p->feature_prefix > p->customers) return why = "feature_prefix > customers", MRIP_E_INVAL;
    return MRIP_OK;
  }
  if (model == MRIP_FF) {
    const mrip_ff_params *p = (const mrip_ff_params *)params;
    if (p->size != sizeof(mrip_ff_params)) return why = "mrip_ff_params.size mismatch", MRIP_E_INVAL;
    if (p->grid < 32 || p->grid > 256 || p->grid % 32 != 0)
      return why = "grid must be a multiple of 32 in 32..256", MRIP_E_INVAL;
    if (effective(map) == MRIP_MAP_WAVE && p->grid != 64 && p->grid != 128)
      return why = "the WAVE mapping supports grid 64 or 128", MRIP_E_INVAL;
    if (!(p->p_grow >= 0.0 && p->p_grow <= 1.0) || !(p->f_light >= 0.0 && p->f_light <= 1.0))
      return why = "probabilities must be in [0, 1]", MRIP_E_INVAL;
    if ((double)p->grid * p->grid * (double)p->steps >= 2147483648.0)
      return why = "grid^2 * steps must be < 2^31", MRIP_E_INVAL;
    return MRIP_OK;
  }
  if (model == MRIP_PI) {
    const mrip_pi_params *p = (const mrip_pi_params *)params;
    if (p->size != sizeof(mrip_pi_params)) return why = "mrip_pi_params.size mismatch", MRIP_E_INVAL;
    if (p->points < 1 || p->points >= (1ull << 31)) return why = "points must be in [1, 2^31)", MRIP_E_INVAL;
    return MRIP_OK;
  }
  return why = "unknown model", MRIP_E_INVAL;
}

}  // namespace

uint32_t mrip::plan_split_for(mrip_ctx ctx, uint64_t longest, uint64_t total) {
  if (ctx->plan_split_set) return ctx->plan_split;
  if (ctx->cus == 0) {
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && n > 0)
      ctx->cus = (uint32_t)n;
    else
      ctx->cus = 256;
  }
  // wavefronts the chip holds at once in the feature-free kernels: four
  // per SIMD, four SIMDs per compute unit
  const uint64_t slots = 16ull * ctx->cus;
  uint32_t x = 1;
  while (x < ctx->plan_split && (double)longest * (double)slots > (double)total * x) x *= 2;
  return x;
}

extern "C" {

const char *mrip_version(void) { return "mrip 0.1 (gfx950)"; }

const char *mrip_status_string(mrip_status s) {
  switch (s) {
    case MRIP_OK: return "ok";
    case MRIP_E_INVAL: return "invalid argument";
    case MRIP_E_NOMEM: return "out of memory";
    case MRIP_E_HIP: return "HIP error";
    case MRIP_E_STATE: return "call out of order";
    case MRIP_E_TOO_FEW: return "fewer than two replications";
    case MRIP_E_UNSUPPORTED: return "unsupported";
  }
  return "unknown status";
}

const char *mrip_last_error(mrip_ctx ctx) { return ctx ? ctx->err.c_str() : ""; }

double mrip_t_quantile(double p, double dof) { return mrip::t_quantile(p, dof); }

mrip_status mrip_create(mrip_ctx *out, mrip_model model, const void *params,
                        mrip_mapping mapping) {
  if (!out) return MRIP_E_INVAL;
  *out = nullptr;
  std::string why;
  mrip_status st = validate(model, params, mapping, why);
  if (st != MRIP_OK) return st;
  mrip_ctx c = new (std::nothrow) mrip_ctx_s();
  if (!c) return MRIP_E_NOMEM;
  c->model = model;
  c->mapping = effective(mapping);
  if (model == MRIP_RW) c->rw = *(const mrip_rw_params *)params;
  if (model == MRIP_MM1) c->mm1 = *(const mrip_mm1_params *)params;
  if (model == MRIP_FF) c->ff = *(const mrip_ff_params *)params;
  if (model == MRIP_PI) c->pi = *(const mrip_pi_params *)params;
  *out = c;
  return MRIP_OK;
}

void mrip_destroy(mrip_ctx ctx) {
  if (!ctx) return;
  if (ctx->last_stream) (void)hipStreamSynchronize(ctx->last_stream);
  if (ctx->red_stream) (void)hipStreamSynchronize(ctx->red_stream);
  delete ctx;
}

mrip_status mrip_set_shape(mrip_ctx ctx, uint32_t rpw, uint32_t wg) {
  if (!ctx) return MRIP_E_INVAL;
  if (rpw != 1 && rpw != 2 && rpw != 4) return inval(ctx, "reps_per_wave must be 1, 2 or 4");
  if (wg != 64 && wg != 256 && wg != 1024) return inval(ctx, "workgroup must be 64, 256 or 1024");
  if (rpw != 1 && ctx->model != MRIP_MM1)
    return inval(ctx, "reps_per_wave > 1 is only defined for the M/M/1 engine");
  if (rpw != 1 && ctx->split != 1) return inval(ctx, "a split replication needs reps_per_wave = 1");
  ctx->rpw = ctx->plan_rpw = rpw;
  ctx->wg = ctx->plan_wg = wg;
  return MRIP_OK;
}

mrip_status mrip_set_split(mrip_ctx ctx, uint32_t waves_per_rep) {
  if (!ctx) return MRIP_E_INVAL;
  if (waves_per_rep != 1 && waves_per_rep != 2 && waves_per_rep != 4 && waves_per_rep != 8)
    return inval(ctx, "waves_per_rep must be 1, 2, 4 or 8");
  if (waves_per_rep > 1 && (ctx->model != MRIP_MM1 || ctx->mapping != MRIP_MAP_WAVE))
    return inval(ctx, "splitting a replication is defined for the M/M/1 WAVE engine");
  if (waves_per_rep > 1 && ctx->rpw != 1) return inval(ctx, "splitting needs reps_per_wave = 1");
  if (waves_per_rep > 4 && ctx->rng != MRIP_RNG_PHILOX)
    return (ctx->err = "taus88 replications split over at most 4 wavefronts"), MRIP_E_UNSUPPORTED;
  ctx->split = waves_per_rep;
  return MRIP_OK;
}

mrip_status mrip_set_rng(mrip_ctx ctx, mrip_rng rng) {
  if (!ctx) return MRIP_E_INVAL;
  if (rng != MRIP_RNG_PHILOX && rng != MRIP_RNG_TAUS88) return inval(ctx, "unknown generator");
  if (rng == MRIP_RNG_TAUS88) {
    if (ctx->model == MRIP_FF)
      return (ctx->err = "the forest fire draws from Philox streams"), MRIP_E_UNSUPPORTED;
    if (ctx->split > 4)
      return (ctx->err = "taus88 replications split over at most 4 wavefronts"), MRIP_E_UNSUPPORTED;
    mrip_status st = upload_taus_tables(ctx);
    if (st != MRIP_OK) return st;
  }
  ctx->rng = rng;
  return MRIP_OK;
}

mrip_status mrip_set_plan_split(mrip_ctx ctx, uint32_t waves_per_item, uint64_t long_min) {
  if (!ctx) return MRIP_E_INVAL;
  if (waves_per_item != 1 && waves_per_item != 2 && waves_per_item != 4 && waves_per_item != 8)
    return inval(ctx, "waves_per_item must be 1, 2, 4 or 8");
  if (ctx->model != MRIP_MM1) return inval(ctx, "plans are defined for the M/M/1 engine");
  ctx->plan_split = waves_per_item;
  ctx->plan_split_set = true;
  ctx->long_min = long_min > 0 ? long_min : 65536;
  return MRIP_OK;
}

mrip_status mrip_get_shape(mrip_ctx ctx, uint32_t *rpw, uint32_t *wg, uint32_t *split,
                           uint32_t *plan_split) {
  if (!ctx) return MRIP_E_INVAL;
  if (rpw) *rpw = ctx->rpw;
  if (wg) *wg = ctx->wg;
  if (split) *split = ctx->split;
  if (plan_split) *plan_split = ctx->plan_split;
  return MRIP_OK;
}

// Lanes one replication occupies in its launch (a launch holds < 2^32).
uint64_t lanes_per_rep(mrip_ctx c) {
  if (c->mapping == MRIP_MAP_SIMT) return 1;
  if (c->mapping == MRIP_MAP_LANE0) return 64;
  if (c->model == MRIP_MM1 && c->split > 1) return 64ull * c->split;
  if (c->model == MRIP_MM1 && c->rpw > 1) return 64ull / c->rpw;
  return 64;
}

mrip_status mrip_run(mrip_ctx ctx, uint64_t n_reps, uint64_t seed, void *hip_stream) {
  if (!ctx) return MRIP_E_INVAL;
  if (n_reps == 0) return inval(ctx, "n_reps must be >= 1");
  if (n_reps > 0xFFFFFFFFull) return inval(ctx, "n_reps must be < 2^32");
  if (n_reps * lanes_per_rep(ctx) > 0xFFFFFFFFull - 1024)
    return inval(ctx, "too many replications for one launch of this mapping "
                      "(replications x lanes per replication must stay below 2^32 - 1024)");
  hipStream_t s = (hipStream_t)hip_stream;
  mrip_status st = ensure_events(ctx);
  if (st != MRIP_OK) return st;
  const uint32_t nout = scalar_outputs(ctx);
  // With the outputs in the context's buffers, the reduction runs on the
  // library's own stream, so the next run's simulation need not wait for
  // it: runs alternate between two output sets.
  bool overlap = true;
  for (uint32_t o = 0; o < mrip_ctx_s::MAX_OUT; ++o) overlap = overlap && !ctx->bound[o].p;
  const bool wave = ctx->mapping == MRIP_MAP_WAVE;
  // the headline form, one kernel per run, times itself
  const bool self_timed = kSelfTimedLaunch && ctx->model == MRIP_MM1 && wave && ctx->split > 1 &&
                          ctx->rng == MRIP_RNG_PHILOX;
  // ... and leaves its statistics to the next run of the same form on the
  // same stream, whose kernel reduces them in one extra workgroup: no event
  // or reduction launch between consecutive simulation kernels
  const bool deferred = self_timed && overlap && ctx->mm1.feature_prefix == 0 &&
                        (ctx->split == 2 || ctx->split == 4);
  if (ctx->pend.active && !(deferred && ctx->pend.stream == s)) {
    st = flush_pending(ctx);
    if (st != MRIP_OK) return st;
  }
  st = order_after_last(ctx, s);
  if (st != MRIP_OK) return st;
  const uint32_t set = overlap ? ctx->next_set : 0u;
  st = claim_set(ctx, set, s);
  if (st != MRIP_OK) return st;
  void *outp[mrip_ctx_s::MAX_OUT] = {};
  for (uint32_t o = 0; o < nout; ++o) {
    st = output_buffer(ctx, set, o, n_reps * 4, &outp[o]);
    if (st != MRIP_OK) return st;
  }
  if (deferred) {
    // one launch in timing_every records the kernel's own events
    const bool timed = ctx->timing_every > 0 && ctx->timing_count % ctx->timing_every == 0;
    ++ctx->timing_count;
    KernelEvents ev{};
    if (timed) {
      st = record_begin(ctx, s, false);
      if (st != MRIP_OK) return st;
      ev = kernel_events(ctx);
    }
    Mm1Args a{};
    a.seed = seed;
    a.n_reps = n_reps;
    a.lambda = ctx->mm1.lambda;
    a.mu = ctx->mm1.mu;
    a.customers = ctx->mm1.customers;
    a.mean_w = (float *)outp[0];
    a.mean_t = (float *)outp[1];
    a.mean_i = (float *)outp[2];
    a.rng = ctx->rng;
    if (ctx->pend.active) {  // the previous run's statistics, in this launch
      const mrip_ctx_s::Pending &p = ctx->pend;
      const uint32_t slot = (uint32_t)(p.stats_index % mrip_ctx_s::STATS_RING);
      for (uint32_t o = 0; o < 3; ++o) a.prev_x[o] = ctx->out[p.set][o].as<float>();
      a.prev_n = p.n;
      a.prev_out = ctx->stats_view + (size_t)slot * mrip_ctx_s::STATS_SLOT;
      a.prev_seq = ctx->seq_view + slot;
      a.prev_seq_value = p.stats_index + 1;
      ctx->slot_by_seq[slot] = true;
      ctx->seq_stream[slot] = s;
      ctx->pend.active = false;
    }
    HIP_TRY(ctx, launch_mm1_split(a, ctx->split, s, timed ? &ev : nullptr));
    if (timed) {
      st = record_end(ctx, s, false);
      if (st != MRIP_OK) return st;
    }
    ctx->pend.active = true;
    ctx->pend.stream = s;
    ctx->pend.set = set;
    ctx->pend.n = n_reps;
    ctx->pend.stats_index = ctx->stats_runs++;
    // the set's next writer follows on s, after the kernel that reduces it
    ctx->set_pending[set] = false;
    ctx->next_set = set ^ 1u;
    if (timed) mark_done(ctx, s, last_ring_event(ctx));
    else mark_unmarked(ctx, s);
    ctx->last = RUN_UNIFORM;
    ctx->last_n = n_reps;
    return MRIP_OK;
  }

  st = record_begin(ctx, s, !self_timed);
  if (st != MRIP_OK) return st;
  if (ctx->model == MRIP_RW) {
    RwArgs a{};
    a.seed = seed;
    a.walkers = ctx->rw.walkers;
    a.grid = ctx->rw.grid;
    a.steps = ctx->rw.steps;
    a.n_reps = n_reps;
    a.ssd = (int32_t *)outp[0];
    a.distinct = (int32_t *)outp[1];
    a.rng = ctx->rng;
    a.taus = ctx->taus_tables.as<uint32_t>();
    a.taus_walk = ctx->taus_walk.as<uint32_t>();
    uint64_t chunk = n_reps;  // replications per launch
    if (ctx->rw.walker_sites) {
      const uint64_t bytes = (uint64_t)a.grid * a.grid / 8;  // one bitmap
      const uint64_t per_rep = wave ? a.walkers * bytes : bytes;
      // WAVE keeps a bitmap per walker: launch at most WALKER_SCRATCH_MAX
      // bytes' worth of replications at a time (each launch reuses them)
      if (wave) chunk = std::max<uint64_t>(1, std::min(n_reps, WALKER_SCRATCH_MAX / per_rep));
      HIP_TRY(ctx, ctx->walker_scratch.ensure(chunk * per_rep));
      a.walker_bitmaps = ctx->walker_scratch.as<uint32_t>();
      a.walker_sites = (int32_t *)outp[2];
    }
    if (wave) {
      for (uint64_t r0 = 0; r0 < n_reps; r0 += chunk) {
        RwArgs b = a;
        b.rep0 = r0;
        b.n_reps = std::min(chunk, n_reps - r0);
        b.ssd += r0;
        b.distinct += r0;
        if (b.walker_sites) b.walker_sites += r0;
        HIP_TRY(ctx, launch_rw_wave(b, ctx->wg, s));
      }
    } else {
      HIP_TRY(ctx, ctx->scratch.ensure(n_reps * (uint64_t)a.grid * a.grid / 8));
      a.scratch_bitmaps = ctx->scratch.as<uint32_t>();
      HIP_TRY(ctx, launch_rw_simt(a, ctx->mapping == MRIP_MAP_LANE0, s));
    }
  } else if (ctx->model == MRIP_MM1) {
    Mm1Args a{};
    a.seed = seed;
    a.n_reps = n_reps;
    a.lambda = ctx->mm1.lambda;
    a.mu = ctx->mm1.mu;
    a.customers = ctx->mm1.customers;
    a.feature_prefix = ctx->mm1.feature_prefix;
    a.mean_w = (float *)outp[0];
    a.mean_t = (float *)outp[1];
    a.mean_i = (float *)outp[2];
    a.rng = ctx->rng;
    a.taus = ctx->taus_tables.as<uint32_t>();
    a.taus_run = ctx->taus_run.as<uint32_t>();
    if (a.feature_prefix > 0) {
      st = output_buffer(ctx, set, 3, n_reps * 40, &outp[3]);
      if (st != MRIP_OK) return st;
      st = output_buffer(ctx, set, 4, n_reps * 32, &outp[4]);
      if (st != MRIP_OK) return st;
      a.features = (float *)outp[3];
      a.controls = (float *)outp[4];
    }
    if (self_timed) {
      const KernelEvents ev = kernel_events(ctx);
      HIP_TRY(ctx, launch_mm1_split(a, ctx->split, s, &ev));
    } else if (wave && ctx->split > 1) HIP_TRY(ctx, launch_mm1_split(a, ctx->split, s));
    else if (wave) HIP_TRY(ctx, launch_mm1_wave(a, ctx->rpw, ctx->wg, s));
    else HIP_TRY(ctx, launch_mm1_simt(a, ctx->mapping == MRIP_MAP_LANE0, s));
  } else if (ctx->model == MRIP_PI) {
    PiArgs a{};
    a.seed = seed;
    a.points = ctx->pi.points;
    a.n_reps = n_reps;
    a.hits = (int32_t *)outp[0];
    a.estimate = (float *)outp[1];
    a.rng = ctx->rng;
    a.taus = ctx->taus_tables.as<uint32_t>();
    if (wave) HIP_TRY(ctx, launch_pi_wave(a, ctx->wg, s));
    else HIP_TRY(ctx, launch_pi_simt(a, ctx->mapping == MRIP_MAP_LANE0, s));
  } else {
    FfArgs a{};
    a.seed = seed;
    a.grid = ctx->ff.grid;
    a.steps = ctx->ff.steps;
    a.tp = ff_threshold(ctx->ff.p_grow);
    a.tf = ff_threshold(ctx->ff.f_light);
    a.n_reps = n_reps;
    a.burnt = (int32_t *)outp[0];
    if (wave) {
      HIP_TRY(ctx, launch_ff_wave(a, ctx->wg, s));
    } else {
      HIP_TRY(ctx, ctx->scratch.ensure(n_reps * 2ull * a.grid * (a.grid / 32) * 4));
      a.state = ctx->scratch.as<uint32_t>();
      HIP_TRY(ctx, launch_ff_simt(a, ctx->mapping == MRIP_MAP_LANE0, s));
    }
  }
  st = record_end(ctx, s, !self_timed);
  if (st != MRIP_OK) return st;
  // all scalar outputs in one reduction launch, written straight into
  // pinned host memory, so mrip_stats only waits for an event
  ReduceSet rs{};
  for (uint32_t o = 0; o < nout; ++o) {
    rs.x[o] = outp[o];
    rs.dtype[o] = output_dtype(ctx->model, o);
  }
  hipStream_t rstream = s;
  if (overlap) {
    // the reduction waits for this run's simulation (the event just
    // recorded after it) on the library's stream
    const uint32_t slot = (uint32_t)((ctx->launches - 1) % mrip_ctx_s::RING);
    rstream = ctx->red_stream;
    HIP_TRY(ctx, hipStreamWaitEvent(rstream, ctx->ring1[slot], 0));
  }
  HIP_TRY(ctx, launch_reduce_f64_multi(rs, nout, n_reps, next_stats_slot(ctx), rstream));
  st = commit_stats_slot(ctx, rstream);
  if (st != MRIP_OK) return st;
  if (overlap) {
    HIP_TRY(ctx, hipEventRecord(ctx->ev_set_free[set], rstream));
    ctx->set_pending[set] = true;
    ctx->next_set = set ^ 1u;
  }
  // on s: the kernel's end, and after it the reduction unless that ran on
  // the library's stream
  mark_done(ctx, s, overlap ? last_ring_event(ctx) : last_stats_event(ctx));
  ctx->last = RUN_UNIFORM;
  ctx->last_n = n_reps;
  return MRIP_OK;
}

mrip_status mrip_stats_back(mrip_ctx ctx, uint32_t back, uint32_t output, double confidence,
                            mrip_stats_t *out) {
  if (!ctx || !out) return MRIP_E_INVAL;
  if (!(confidence > 0.0 && confidence < 1.0)) return inval(ctx, "confidence must be in (0, 1)");
  if (ctx->last == RUN_NONE || ctx->stats_runs == 0) return (ctx->err = "no run yet"), MRIP_E_STATE;
  if (ctx->last == RUN_PLAN_PARTIAL)
    return (ctx->err = "the last plan run stopped at its item limit: no statistics"), MRIP_E_STATE;
  if (output >= scalar_outputs(ctx)) return inval(ctx, "no such scalar output");
  if (back >= mrip_ctx_s::STATS_RING || back >= ctx->stats_runs)
    return (ctx->err = "no statistics kept for that run"), MRIP_E_STATE;
  const uint64_t idx = ctx->stats_runs - 1 - back;
  const uint32_t slot = (uint32_t)(idx % mrip_ctx_s::STATS_RING);
  if (ctx->pend.active && ctx->pend.stats_index == idx) {
    mrip_status st = flush_pending(ctx);  // no later run has reduced it yet
    if (st != MRIP_OK) return st;
  }
  if (ctx->slot_by_seq[slot]) {
    mrip_status st = wait_seq(ctx, slot, idx + 1);
    if (st != MRIP_OK) return st;
  } else {
    HIP_TRY(ctx, hipEventSynchronize(ctx->ev_stats[slot]));
  }
  double nmv[3];
  std::memcpy(nmv, ctx->stats_host + (size_t)slot * mrip_ctx_s::STATS_SLOT + 3 * output,
              sizeof(nmv));
  mrip_status st = finish_stats(nmv, confidence, out);
  if (st == MRIP_E_TOO_FEW) ctx->err = "fewer than two replications";
  return st;
}

mrip_status mrip_stats(mrip_ctx ctx, uint32_t output, double confidence, mrip_stats_t *out) {
  return mrip_stats_back(ctx, 0, output, confidence, out);
}

mrip_status mrip_output_ptr(mrip_ctx ctx, uint32_t output, const void **ptr) {
  if (!ctx || !ptr) return MRIP_E_INVAL;
  if (ctx->last == RUN_NONE) return (ctx->err = "no run yet"), MRIP_E_STATE;
  const bool vec = vector_width(ctx, output) > 0 && ctx->mm1.feature_prefix > 0;
  if (output >= scalar_outputs(ctx) && !vec) return inval(ctx, "no such output");
  *ptr = ctx->cur[output];
  return MRIP_OK;
}

mrip_status mrip_outputs(mrip_ctx ctx, uint32_t output, void *dst, uint64_t bytes,
                         int dst_is_device) {
  if (!ctx || !dst) return MRIP_E_INVAL;
  if (ctx->last == RUN_NONE) return (ctx->err = "no run yet"), MRIP_E_STATE;
  const bool vec = vector_width(ctx, output) > 0 && ctx->mm1.feature_prefix > 0;
  if (output >= scalar_outputs(ctx) && !vec) return inval(ctx, "no such output");
  const uint64_t need = ctx->last_n * 4 * (vec ? vector_width(ctx, output) : 1);
  if (bytes < need) return inval(ctx, "destination too small");
  HIP_TRY(ctx, hipStreamSynchronize(ctx->last_stream));
  HIP_TRY(ctx, hipMemcpy(dst, ctx->cur[output], need,
                         dst_is_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost));
  return MRIP_OK;
}

mrip_status mrip_run_history_ms(mrip_ctx ctx, float *ms, uint32_t max_n, uint32_t *n_out) {
  if (!ctx || !n_out || (max_n > 0 && !ms)) return MRIP_E_INVAL;
  uint64_t avail = std::min<uint64_t>(ctx->launches, mrip_ctx_s::RING);
  uint32_t n = (uint32_t)std::min<uint64_t>(avail, max_n);
  for (uint32_t i = 0; i < n; ++i) {
    const uint64_t launch = ctx->launches - n + i;
    const uint32_t slot = (uint32_t)(launch % mrip_ctx_s::RING);
    HIP_TRY(ctx, hipEventSynchronize(ctx->ring1[slot]));
    HIP_TRY(ctx, hipEventElapsedTime(&ms[i], ctx->ring0[slot], ctx->ring1[slot]));
  }
  *n_out = n;
  return MRIP_OK;
}

mrip_status mrip_set_timing(mrip_ctx ctx, uint32_t every) {
  if (!ctx) return MRIP_E_INVAL;
  ctx->timing_every = every;
  ctx->timing_count = 0;
  return MRIP_OK;
}

mrip_status mrip_last_run_ms(mrip_ctx ctx, float *ms) {
  if (!ctx || !ms) return MRIP_E_INVAL;
  if (ctx->last == RUN_NONE) return (ctx->err = "no run yet"), MRIP_E_STATE;
  return last_launch_ms(ctx, ms);
}

// ------------------------------------------------------------------ plan

mrip_status mrip_plan_set(mrip_ctx ctx, const mrip_plan_item *items, uint64_t n) {
  if (!ctx) return MRIP_E_INVAL;
  if (philox_only(ctx) != MRIP_OK) return MRIP_E_UNSUPPORTED;
  if (ctx->model != MRIP_MM1) return (ctx->err = "plans need an M/M/1 context"), MRIP_E_UNSUPPORTED;
  if (!items || n == 0) return inval(ctx, "empty plan");
  if (n > 0xFFFFFFFFull) return inval(ctx, "plan too large");
  std::vector<uint32_t> dp(n), rep(n), order(n), index(n);
  std::vector<uint64_t> cust(n);
  std::vector<float> lam(n), mu(n);
  for (uint64_t i = 0; i < n; ++i) {
    const mrip_plan_item &it = items[i];
    if (it.customers < 1 || it.customers >= (1ull << 33)) return inval(ctx, "item customers out of range");
    if (!(it.lambda > 0.0f) || !(it.mu > 0.0f) || !std::isfinite(it.lambda) || !std::isfinite(it.mu))
      return inval(ctx, "item rates must be finite and > 0");
    if (ctx->mm1.feature_prefix > it.customers) return inval(ctx, "item shorter than the feature prefix");
    dp[i] = it.dp;
    rep[i] = it.rep;
    cust[i] = it.customers;
    lam[i] = it.lambda;
    mu[i] = it.mu;
    order[i] = (uint32_t)i;
    index[i] = (uint32_t)i;
  }
  // longest-processing-time-first queue order
  std::stable_sort(order.begin(), order.end(),
                   [&](uint32_t a, uint32_t b) { return cust[a] > cust[b]; });
  // items grouped by design point for the per-dp reductions
  std::stable_sort(index.begin(), index.end(), [&](uint32_t a, uint32_t b) { return dp[a] < dp[b]; });
  std::vector<uint64_t> offsets;
  std::vector<uint32_t> ids;
  for (uint64_t j = 0; j < n; ++j) {
    if (j == 0 || dp[index[j]] != dp[index[j - 1]]) {
      offsets.push_back(j);
      ids.push_back(dp[index[j]]);
    }
  }
  offsets.push_back(n);
  // an earlier plan run may still read the item buffers
  if (ctx->last_stream) HIP_TRY(ctx, hipStreamSynchronize(ctx->last_stream));
  HIP_TRY(ctx, ctx->it_dp.ensure(4 * n));
  HIP_TRY(ctx, ctx->it_rep.ensure(4 * n));
  HIP_TRY(ctx, ctx->it_n.ensure(8 * n));
  HIP_TRY(ctx, ctx->it_lambda.ensure(4 * n));
  HIP_TRY(ctx, ctx->it_mu.ensure(4 * n));
  HIP_TRY(ctx, ctx->it_order.ensure(4 * n));
  HIP_TRY(ctx, ctx->dp_index.ensure(4 * n));
  HIP_TRY(ctx, ctx->dp_offsets.ensure(8 * offsets.size()));
  HIP_TRY(ctx, ctx->dp_stats.ensure(sizeof(double) * 3 * ids.size()));
  HIP_TRY(ctx, ctx->queue.ensure(256));
  HIP_TRY(ctx, hipMemcpy(ctx->it_dp.p, dp.data(), 4 * n, hipMemcpyHostToDevice));
  HIP_TRY(ctx, hipMemcpy(ctx->it_rep.p, rep.data(), 4 * n, hipMemcpyHostToDevice));
  HIP_TRY(ctx, hipMemcpy(ctx->it_n.p, cust.data(), 8 * n, hipMemcpyHostToDevice));
  HIP_TRY(ctx, hipMemcpy(ctx->it_lambda.p, lam.data(), 4 * n, hipMemcpyHostToDevice));
  HIP_TRY(ctx, hipMemcpy(ctx->it_mu.p, mu.data(), 4 * n, hipMemcpyHostToDevice));
  HIP_TRY(ctx, hipMemcpy(ctx->it_order.p, order.data(), 4 * n, hipMemcpyHostToDevice));
  HIP_TRY(ctx, hipMemcpy(ctx->dp_index.p, index.data(), 4 * n, hipMemcpyHostToDevice));
  HIP_TRY(ctx, hipMemcpy(ctx->dp_offsets.p, offsets.data(), 8 * offsets.size(), hipMemcpyHostToDevice));
  ctx->n_items = n;
  ctx->dp_ids = ids;
  ctx->lpt_customers.resize(n);
  for (uint64_t j = 0; j < n; ++j) ctx->lpt_customers[j] = cust[order[j]];
  ctx->lpt_order = order;
  return MRIP_OK;
}

// Items of a longest-first order that count as long (a prefix of it).
// The split of the uploaded plan's long items: decided on the whole plan
// (its longest item and all its customers), so a run stopped at an item
// limit or resumed from saved outputs splits every item as the
// uninterrupted run does and gives the same bits.
static uint32_t plan_split_of(mrip_ctx ctx) {
  uint64_t total = 0;
  for (uint64_t n : ctx->lpt_customers) total += n;
  return plan_split_for(ctx, ctx->lpt_customers.empty() ? 0 : ctx->lpt_customers[0], total);
}

static uint64_t count_long(const std::vector<uint64_t> &lpt, uint64_t n, uint64_t long_min) {
  uint64_t k = 0;
  while (k < n && lpt[k] >= long_min) ++k;
  return k;
}

// done (nullable): the per-item done flags the kernels set, cleared first
// on the stream when clear_done is set.
static mrip_status run_plan_impl(mrip_ctx ctx, uint64_t seed, hipStream_t s, const uint32_t *order,
                                 uint64_t n, uint64_t n_long, uint32_t rpw, uint32_t wg,
                                 uint32_t split, bool reduce, uint8_t *done = nullptr,
                                 bool clear_done = false) {
  mrip_status st = ensure_events(ctx);
  if (st != MRIP_OK) return st;
  st = flush_pending(ctx);  // a deferred reduction may read output set 0
  if (st != MRIP_OK) return st;
  st = order_after_last(ctx, s);  // before the queue reset below
  if (st != MRIP_OK) return st;
  if (done && clear_done)
    HIP_TRY(ctx, launch_zero_u32((uint32_t *)done, (uint32_t)((ctx->n_items + 3) / 4), s));
  st = claim_set(ctx, 0, s);
  if (st != MRIP_OK) return st;
  void *outp[mrip_ctx_s::MAX_OUT] = {};
  for (uint32_t o = 0; o < 3; ++o) {
    st = output_buffer(ctx, 0, o, ctx->n_items * 4, &outp[o]);
    if (st != MRIP_OK) return st;
  }
  Mm1Args a{};
  a.seed = seed;
  a.feature_prefix = ctx->mm1.feature_prefix;
  if (a.feature_prefix > 0) {
    st = output_buffer(ctx, 0, 3, ctx->n_items * 40, &outp[3]);
    if (st != MRIP_OK) return st;
    st = output_buffer(ctx, 0, 4, ctx->n_items * 32, &outp[4]);
    if (st != MRIP_OK) return st;
    a.features = (float *)outp[3];
    a.controls = (float *)outp[4];
  }
  a.items.dp = ctx->it_dp.as<uint32_t>();
  a.items.rep = ctx->it_rep.as<uint32_t>();
  a.items.customers = ctx->it_n.as<uint64_t>();
  a.items.lambda = ctx->it_lambda.as<float>();
  a.items.mu = ctx->it_mu.as<float>();
  a.items.order = order;
  a.queue_head = ctx->queue.as<uint32_t>();
  a.done = done;
  a.mean_w = (float *)outp[0];
  a.mean_t = (float *)outp[1];
  a.mean_i = (float *)outp[2];
  HIP_TRY(ctx, launch_zero_u32(a.queue_head, 2, s));
  st = record_begin(ctx, s);
  if (st != MRIP_OK) return st;
  if (n == 0) {
    // nothing left to simulate (a resumed plan): only the reductions run
  } else if (ctx->mapping != MRIP_MAP_WAVE) {
    HIP_TRY(ctx, launch_mm1_plan_simt(a, n, ctx->mapping == MRIP_MAP_LANE0, s));
  } else if (split > 1 && n_long > 0) {
    HIP_TRY(ctx, launch_mm1_plan_split(a, n, n_long, split, rpw, s));
  } else {
    HIP_TRY(ctx, launch_mm1_plan(a, n, rpw, wg, s));
  }
  st = record_end(ctx, s);
  if (st != MRIP_OK) return st;
  if (reduce) {
    HIP_TRY(ctx, launch_reduce_f64_gather(outp[0], 1, ctx->dp_index.as<uint32_t>(),
                                          ctx->dp_offsets.as<uint64_t>(), (uint32_t)ctx->dp_ids.size(),
                                          ctx->dp_stats.as<double>(), s));
    ReduceSet set{};
    for (uint32_t o = 0; o < 3; ++o) {
      set.x[o] = outp[o];
      set.dtype[o] = 1;
    }
    HIP_TRY(ctx, launch_reduce_f64_multi(set, 3, ctx->n_items, next_stats_slot(ctx), s));
    st = commit_stats_slot(ctx, s);
    if (st != MRIP_OK) return st;
  }
  mark_done(ctx, s, reduce ? last_stats_event(ctx) : last_ring_event(ctx));
  return MRIP_OK;
}

// The done flags, one byte per item (rounded up to whole words for the
// clearing kernel).
static mrip_status done_flags(mrip_ctx ctx, uint8_t **out) {
  HIP_TRY(ctx, ctx->item_done.ensure((ctx->n_items + 3) / 4 * 4));
  *out = ctx->item_done.as<uint8_t>();
  return MRIP_OK;
}

mrip_status mrip_run_plan(mrip_ctx ctx, uint64_t seed, void *hip_stream) {
  if (!ctx) return MRIP_E_INVAL;
  if (philox_only(ctx) != MRIP_OK) return MRIP_E_UNSUPPORTED;
  if (ctx->n_items == 0) return (ctx->err = "no plan uploaded"), MRIP_E_STATE;
  // the item limit stops the run after a prefix of the longest-first order
  const uint64_t n_run =
      ctx->plan_limit ? std::min<uint64_t>(ctx->n_items, ctx->plan_limit) : ctx->n_items;
  const uint64_t n_long =
      std::min<uint64_t>(count_long(ctx->lpt_customers, ctx->n_items, ctx->long_min), n_run);
  const bool whole = n_run == ctx->n_items;
  const uint32_t split = plan_split_of(ctx);
  uint8_t *done = nullptr;
  mrip_status st = done_flags(ctx, &done);
  if (st != MRIP_OK) return st;
  st = run_plan_impl(ctx, seed, (hipStream_t)hip_stream, ctx->it_order.as<uint32_t>(), n_run,
                     n_long, ctx->plan_rpw, ctx->plan_wg, split, whole, done, true);
  if (st != MRIP_OK) return st;
  ctx->last = whole ? RUN_PLAN : RUN_PLAN_PARTIAL;
  ctx->last_n = ctx->n_items;
  return MRIP_OK;
}

mrip_status mrip_run_plan_resume(mrip_ctx ctx, uint64_t seed, const uint8_t *skip_done,
                                 void *hip_stream) {
  if (!ctx) return MRIP_E_INVAL;
  if (philox_only(ctx) != MRIP_OK) return MRIP_E_UNSUPPORTED;
  if (ctx->n_items == 0) return (ctx->err = "no plan uploaded"), MRIP_E_STATE;
  if (!skip_done) return mrip_run_plan(ctx, seed, hip_stream);
  hipStream_t s = (hipStream_t)hip_stream;
  // the remaining items, still longest first
  std::vector<uint32_t> todo;
  std::vector<uint64_t> todo_n;
  todo.reserve(ctx->n_items);
  for (uint64_t j = 0; j < ctx->n_items; ++j) {
    const uint32_t i = ctx->lpt_order[j];
    if (!skip_done[i]) {
      todo.push_back(i);
      todo_n.push_back(ctx->lpt_customers[j]);
    }
  }
  // the item limit stops the run after a prefix of the remaining items
  const bool whole = !ctx->plan_limit || todo.size() <= ctx->plan_limit;
  if (!whole) {
    todo.resize(ctx->plan_limit);
    todo_n.resize(ctx->plan_limit);
  }
  // an earlier plan run (on this stream or the last one) may still read the
  // resume queue and the done flags
  HIP_TRY(ctx, hipStreamSynchronize(s));
  if (ctx->last_stream && ctx->last_stream != s) HIP_TRY(ctx, hipStreamSynchronize(ctx->last_stream));
  if (!todo.empty()) {
    HIP_TRY(ctx, ctx->resume_order.ensure(4 * todo.size()));
    HIP_TRY(ctx, hipMemcpy(ctx->resume_order.p, todo.data(), 4 * todo.size(),
                           hipMemcpyHostToDevice));
  }
  // the items the caller reports done start flagged; the run flags the rest
  uint8_t *done = nullptr;
  mrip_status st = done_flags(ctx, &done);
  if (st != MRIP_OK) return st;
  std::vector<uint8_t> flags(ctx->n_items);
  for (uint64_t i = 0; i < ctx->n_items; ++i) flags[i] = skip_done[i] ? 1 : 0;
  HIP_TRY(ctx, hipMemcpy(done, flags.data(), ctx->n_items, hipMemcpyHostToDevice));
  const uint64_t n_long = count_long(todo_n, todo.size(), ctx->long_min);
  const uint32_t split = plan_split_of(ctx);
  st = run_plan_impl(ctx, seed, s, ctx->resume_order.as<uint32_t>(), todo.size(), n_long,
                     ctx->plan_rpw, ctx->plan_wg, split, whole, done, false);
  if (st != MRIP_OK) return st;
  ctx->last = whole ? RUN_PLAN : RUN_PLAN_PARTIAL;
  ctx->last_n = ctx->n_items;
  return MRIP_OK;
}

mrip_status mrip_set_plan_limit(mrip_ctx ctx, uint64_t max_items) {
  if (!ctx) return MRIP_E_INVAL;
  ctx->plan_limit = max_items;
  return MRIP_OK;
}

mrip_status mrip_plan_done(mrip_ctx ctx, uint8_t *done, uint64_t n) {
  if (!ctx || !done) return MRIP_E_INVAL;
  if (ctx->last != RUN_PLAN && ctx->last != RUN_PLAN_PARTIAL)
    return (ctx->err = "no plan run yet"), MRIP_E_STATE;
  if (n != ctx->n_items) return inval(ctx, "n must be the plan's item count");
  HIP_TRY(ctx, hipStreamSynchronize(ctx->last_stream));
  HIP_TRY(ctx, hipMemcpy(done, ctx->item_done.p, n, hipMemcpyDeviceToHost));
  return MRIP_OK;
}

mrip_status mrip_bind_output(mrip_ctx ctx, uint32_t output, void *ptr_dev, uint64_t bytes) {
  if (!ctx) return MRIP_E_INVAL;
  const bool vec = vector_width(ctx, output) > 0;
  if (output >= scalar_outputs(ctx) && !vec) return inval(ctx, "no such output");
  if (ptr_dev && (bytes == 0 || ((uintptr_t)ptr_dev & 3u)))
    return inval(ctx, "a bound output needs a non-empty, 4-byte aligned buffer");
  ctx->bound[output].p = ptr_dev;
  ctx->bound[output].bytes = ptr_dev ? bytes : 0;
  return MRIP_OK;
}

mrip_status mrip_plan_stats(mrip_ctx ctx, uint32_t dp, double confidence, mrip_stats_t *out) {
  if (!ctx || !out) return MRIP_E_INVAL;
  if (!(confidence > 0.0 && confidence < 1.0)) return inval(ctx, "confidence must be in (0, 1)");
  if (ctx->last == RUN_PLAN_PARTIAL)
    return (ctx->err = "the last plan run stopped at its item limit: no statistics"), MRIP_E_STATE;
  if (ctx->last != RUN_PLAN) return (ctx->err = "no plan run yet"), MRIP_E_STATE;
  auto it = std::lower_bound(ctx->dp_ids.begin(), ctx->dp_ids.end(), dp);
  if (it == ctx->dp_ids.end() || *it != dp) return inval(ctx, "no such design point");
  const size_t g = (size_t)(it - ctx->dp_ids.begin());
  HIP_TRY(ctx, hipStreamSynchronize(ctx->last_stream));
  double nmv[3];
  HIP_TRY(ctx, hipMemcpy(nmv, ctx->dp_stats.as<double>() + 3 * g, sizeof(nmv), hipMemcpyDeviceToHost));
  mrip_status st = finish_stats(nmv, confidence, out);
  if (st == MRIP_E_TOO_FEW) ctx->err = "fewer than two replications";
  return st;
}

mrip_status mrip_autotune(mrip_ctx ctx, uint64_t seed, uint64_t calib_items, void *hip_stream,
                          uint32_t *best_rpw, uint32_t *best_wg, float *best_ms) {
  if (!ctx) return MRIP_E_INVAL;
  if (philox_only(ctx) != MRIP_OK) return MRIP_E_UNSUPPORTED;
  if (ctx->n_items == 0) return (ctx->err = "no plan uploaded"), MRIP_E_STATE;
  if (ctx->mapping != MRIP_MAP_WAVE)
    return (ctx->err = "the autotuner times the WAVE plan shapes"), MRIP_E_UNSUPPORTED;
  hipStream_t s = (hipStream_t)hip_stream;
  const uint32_t *order = ctx->it_order.as<uint32_t>();
  uint64_t n = ctx->n_items;
  DevBuf sub;
  if (calib_items > 0 && calib_items < ctx->n_items) {
    // an evenly strided slice of the longest-first order keeps its length mix
    std::vector<uint32_t> full(ctx->n_items), pick;
    HIP_TRY(ctx, hipMemcpy(full.data(), order, 4 * ctx->n_items, hipMemcpyDeviceToHost));
    const double stride = (double)ctx->n_items / (double)calib_items;
    for (uint64_t j = 0; j < calib_items; ++j) pick.push_back(full[(uint64_t)(j * stride)]);
    HIP_TRY(ctx, sub.ensure(4 * pick.size()));
    HIP_TRY(ctx, hipMemcpy(sub.p, pick.data(), 4 * pick.size(), hipMemcpyHostToDevice));
    order = sub.as<uint32_t>();
    n = pick.size();
  }
  // the slice's lengths in longest-first order decide which items are long
  std::vector<uint64_t> lpt(n);
  if (n == ctx->n_items) {
    lpt = ctx->lpt_customers;
  } else {
    const double stride = (double)ctx->n_items / (double)n;
    for (uint64_t j = 0; j < n; ++j) lpt[j] = ctx->lpt_customers[(uint64_t)(j * stride)];
  }
  const uint64_t n_long = count_long(lpt, n, ctx->long_min);
  // the cache named by MRIP_TUNE_CACHE: a stored shape for this kind of
  // plan on this kind of GPU is installed without timing
  const char *cache = std::getenv("MRIP_TUNE_CACHE");
  char key[256] = {0};
  bool use_cache = false;
  if (cache && *cache) {
    int dev = 0, cus = 0;
    hipDeviceProp_t prop;
    HIP_TRY(ctx, hipGetDevice(&dev));
    HIP_TRY(ctx, hipGetDeviceProperties(&prop, dev));
    HIP_TRY(ctx, hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    use_cache = mrip_tune_key(ctx->model, ctx->mapping, n, n_long, lpt.empty() ? 0 : lpt[0],
                              prop.gcnArchName, (uint32_t)cus, key, sizeof key) == MRIP_OK;
    mrip_tune_entry e{};
    if (use_cache && mrip_tune_cache_get(cache, key, &e) == MRIP_OK &&
        (e.reps_per_wave == 1 || e.reps_per_wave == 2 || e.reps_per_wave == 4) &&
        (e.workgroup == 64 || e.workgroup == 256 || e.workgroup == 1024) &&
        (e.plan_split == 1 || e.plan_split == 2 || e.plan_split == 4 || e.plan_split == 8)) {
      ctx->plan_rpw = e.reps_per_wave;
      ctx->plan_wg = e.workgroup;
      ctx->plan_split = e.plan_split;
      ctx->plan_split_set = true;
      if (best_rpw) *best_rpw = e.reps_per_wave;
      if (best_wg)
        *best_wg = (e.plan_split > 1 && n_long > 0) ? (e.plan_split == 8 ? 512u : 256u) : e.workgroup;
      if (best_ms) *best_ms = e.ms;
      return MRIP_OK;
    }
  }
  struct Shape { uint32_t rpw, wg, split; };
  std::vector<Shape> shapes;
  for (uint32_t r : {1u, 2u, 4u})
    for (uint32_t w : {64u, 256u, 1024u}) shapes.push_back({r, w, 1});
  if (n_long > 0)
    for (uint32_t r : {1u, 2u, 4u})
      for (uint32_t x : {2u, 4u, 8u}) shapes.push_back({r, 256u, x});
  float best = 1e30f;
  uint32_t br = ctx->plan_rpw, bw = ctx->plan_wg, bx = ctx->plan_split;
  for (const Shape &sh : shapes) {
    float t_min = 1e30f;
    // the first launch warms up; the best of four more, since shapes a few
    // per cent apart swap places in single timings
    for (int rep = 0; rep < 5; ++rep) {
      mrip_status st = run_plan_impl(ctx, seed, s, order, n, n_long, sh.rpw, sh.wg, sh.split, false);
      if (st != MRIP_OK) return st;
      float ms = 0.f;
      st = last_launch_ms(ctx, &ms);
      if (st != MRIP_OK) return st;
      if (rep > 0) t_min = std::min(t_min, ms);
    }
    if (t_min < best) {
      best = t_min;
      br = sh.rpw;
      bw = sh.wg;
      bx = sh.split;
    }
  }
  ctx->plan_split = bx;
  ctx->plan_split_set = true;
  ctx->plan_rpw = br;
  ctx->plan_wg = bw;
  ctx->last = RUN_NONE;  // outputs of the timing runs are partial
  if (use_cache) {
    const mrip_tune_entry e{br, bw, bx, best};
    (void)mrip_tune_cache_put(cache, key, &e);  // a cache that cannot be written is only slower
  }
  if (best_rpw) *best_rpw = br;
  // the workgroup size actually launched: a split plan launches 256
  // threads per workgroup for 2 or 4 wavefronts per item, 512 for 8
  if (best_wg) *best_wg = (bx > 1 && n_long > 0) ? (bx == 8 ? 512u : 256u) : bw;
  if (best_ms) *best_ms = best;
  return MRIP_OK;
}

// ------------------------------------------------------------- utilities

// one lane per value: a dump launch holds fewer than 2^32 lanes
constexpr uint64_t kDumpMax = 0xFFFFFF00ull;

mrip_status mrip_taus88(uint64_t seed, uint32_t model, uint32_t dp, uint32_t rep, uint64_t skip,
                        uint64_t n, uint32_t *out_dev, void *hip_stream) {
  if (n == 0) return MRIP_OK;
  if (!out_dev || n > kDumpMax) return MRIP_E_INVAL;
  std::vector<uint32_t> host((size_t)TAUS_TABLES * TAUS_COLS);
  taus_build_tables(host.data());
  DevBuf tables;
  hipStream_t s = (hipStream_t)hip_stream;
  if (tables.ensure(host.size() * sizeof(uint32_t)) != hipSuccess) return MRIP_E_NOMEM;
  if (hipMemcpy(tables.p, host.data(), host.size() * sizeof(uint32_t), hipMemcpyHostToDevice) !=
      hipSuccess)
    return MRIP_E_HIP;
  if (launch_taus_dump(seed, model, dp, rep, skip, n, tables.as<uint32_t>(), out_dev, s) !=
      hipSuccess)
    return MRIP_E_HIP;
  // the tables are freed on return: wait for the kernel that reads them
  return hipStreamSynchronize(s) == hipSuccess ? MRIP_OK : MRIP_E_HIP;
}

mrip_status mrip_philox(uint64_t seed, const uint32_t *ctr_dev, uint64_t n, uint32_t *out_dev,
                        void *hip_stream) {
  if (n > 0 && (!ctr_dev || !out_dev)) return MRIP_E_INVAL;
  if (n > kDumpMax) return MRIP_E_INVAL;
  hipError_t e = launch_philox_dump(seed, ctr_dev, n, out_dev, (hipStream_t)hip_stream);
  return e == hipSuccess ? MRIP_OK : MRIP_E_HIP;
}

}  // extern "C"

