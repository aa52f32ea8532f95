/*
 * mrip.h -- Multiple Replications In Parallel on one MI355X (gfx950).
 *
 * The method (Passerat-Palmbach et al., "Warp-Level Parallelism: Enabling
 * Multiple Replications In Parallel on GPU", ESM 2011, section 1): run the
 * same stochastic simulation many times with independent random sources,
 * in parallel, and reduce the per-replication outputs to a mean, a variance
 * and a confidence interval (at least 30 replications, central limit
 * theorem). Section 3 compares one replication per thread (SIMT) with one
 * replication per warp; here the second form is one replication per 64-lane
 * wavefront with every lane working on it (MRIP_MAP_WAVE).
 *
 * Random streams: Philox4x32-10 (Salmon et al., SC'11), key = the 64-bit
 * seed, counter = (draw index, entity, replication, model tag). Outputs are
 * pure functions of (seed, replication id, parameters): they do not depend
 * on the mapping's launch shape, on the number of replications run, or on
 * the order in which the device schedules them.
 *
 * Conventions for every call:
 *  - Every call returns mrip_status; nothing throws across this boundary.
 *    HIP failures return MRIP_E_HIP with the HIP error text in
 *    mrip_last_error(ctx).
 *  - `hip_stream` is a caller-owned hipStream_t (NULL = the null stream).
 *    Run calls only enqueue work and return; calls that hand results back
 *    to the host synchronise that stream first. A run enqueued on another
 *    stream than the context's previous run waits on the device for that
 *    run's simulation (the context's scratch buffers serve one at a time).
 *  - Pointers named *_dev are device pointers the caller owns (for example
 *    torch tensors); pointers without the suffix are host pointers, read
 *    during the call only. The context owns every buffer it allocates and
 *    frees them in mrip_destroy.
 *  - A context is not thread-safe: use one per host thread.
 */
#ifndef MRIP_H
#define MRIP_H

#include <stdint.h>

#if defined(__GNUC__)
#define MRIP_API __attribute__((visibility("default")))
#else
#define MRIP_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mrip_ctx_s *mrip_ctx;

/* The enumerated types are plain 32-bit integers at the boundary, so that
 * any value a caller passes is one the library can receive and refuse
 * (MRIP_E_INVAL) rather than an out-of-range enumeration. */
typedef int32_t mrip_status;
enum {
  MRIP_OK = 0,
  MRIP_E_INVAL = -1,       /* bad argument or parameter                       */
  MRIP_E_NOMEM = -2,       /* device or host allocation failed                */
  MRIP_E_HIP = -3,         /* a HIP runtime call failed                       */
  MRIP_E_STATE = -4,       /* call out of order (e.g. stats before any run)   */
  MRIP_E_TOO_FEW = -5,     /* fewer than two replications for an interval     */
  MRIP_E_UNSUPPORTED = -6  /* valid request the library does not implement    */
};

typedef int32_t mrip_model;
enum { MRIP_RW = 1, MRIP_MM1 = 2, MRIP_FF = 3, MRIP_PI = 4 };

/* SIMT: one replication per lane (the paper's thread-level form, section
 * 3). WAVE: one replication per 64-lane wavefront with every lane working on
 * it (or 2 / 4 replications per wavefront on 32 / 16 lanes each, see
 * mrip_set_shape). LANE0: one replication per wavefront with only its first
 * lane working, the paper's own warp-level form (sections 3 and 4: every
 * thread but the first of its warp disabled). AUTO picks WAVE. */
/* Stream source. PHILOX (default): counter-based Philox4x32-10, as stated
 * per model below. TAUS88: the generator the paper's models draw from
 * (section 5), L'Ecuyer's three-component Tausworthe generator taus88
 * ((k, q, s) = (31, 13, 12), (29, 2, 4), (28, 3, 17); the output is the xor
 * of the three component words after each step), with streams split by
 * Random Spacing (section 5): the stream of (model, dp, replication r)
 * starts from words x, y, z of Philox block (model tag, dp, r, 5) under the
 * seed, raised by 2, 8 and 16 when below them; draw d of a replication is
 * output d of its stream. Running a second set of replications on another
 * generator checks that the streams do not bias the results (section 5.3).
 * On TAUS88 streams: pi point i takes outputs 2i, 2i+1; M/M/1 customer n
 * takes 2n (A) and 2n+1 (S); walk move t of walker w takes bits 2(t&15) of
 * output w*ceil(steps/16) + (t>>4). */
typedef int32_t mrip_rng;
enum { MRIP_RNG_PHILOX = 0, MRIP_RNG_TAUS88 = 1 };

typedef int32_t mrip_mapping;
enum { MRIP_MAP_AUTO = 0, MRIP_MAP_SIMT = 1, MRIP_MAP_WAVE = 2, MRIP_MAP_LANE0 = 3 };

/* Parameter structs: `size` must equal sizeof(the struct); they are copied
 * by mrip_create. */

/* Lattice random walk (paper section 5.1, third model): `walkers` walkers
 * (1..64) on a grid x grid torus (grid in {16, 32, 64, 128}), `steps` unit
 * moves each; walker w starts at ((w%8)*grid/8 + grid/16, (w/8)*grid/8 +
 * grid/16). Move t of walker w in replication r is 2 bits of block
 * (t>>6, w, r, 1): word (t>>4)&3, bits 2(t&15); 0:+x 1:-x 2:+y 3:-y.
 * Outputs: 0 = int32 sum of squared unwrapped displacements,
 *          1 = int32 number of distinct sites visited (starts included),
 *          2 = when walker_sites != 0, int32 sum over walkers of the
 *              number of sites each one visited (its start included): the
 *              union count nearly fills the torus, this one does not.
 *              Costs a bitmap per walker in device memory and its
 *              updates: WAVE keeps walkers * grid^2 / 8 bytes per
 *              replication and runs at most 1 GiB of them per launch (a
 *              larger run is launched in slices, same outputs); SIMT and
 *              LANE0 keep grid^2 / 8 bytes per replication.
 * Requires walkers * steps^2 < 2^31. */
typedef struct {
  uint32_t size;
  uint32_t walkers, grid, steps;
  uint32_t walker_sites; /* 0 or 1 */
} mrip_rw_params;

/* M/M/1 queue (paper section 5.1, second model), starting empty. Customer n
 * draws interarrival A_n ~ Exp(lambda) and service S_n ~ Exp(mu) from words
 * 2(n&1), 2(n&1)+1 of block (n>>1, dp, r, 2) as mean * -log(u),
 * u = ((x>>8)+1) 2^-24; then W_n = max(0, T_{n-1} - A_n),
 * I_n = max(0, A_n - T_{n-1}), T_n = W_n + S_n, T_{-1} = 0, all in fp32.
 * Outputs: 0 = mean W (waiting time in queue), 1 = mean T (time in system),
 *          2 = mean I (server idle time per arrival), all fp32;
 *          3 = when feature_prefix K > 0, 10 fp32 features per replication
 *              over customers 0..K-1: rho, mu, mean A, mean S, mean W,
 *              mean T, fraction with W = 0, max W, mean I, T_{K-1};
 *          4 = when K > 0, 8 fp32 controls per replication: over
 *              customers n = K..N-1 sum (S_n - E S), sum (A_n - E A),
 *              sum T_{n-1} (S_n - E S), sum T_{n-1} (A_n - E A), then the
 *              same four over n = 0..K-1. E S and E A are the variates'
 *              means as drawn, (float)(1/rate) times the mean of -ln u over
 *              the 24-bit grid of u, in fp32. A_n and S_n are independent
 *              of everything before customer n, so each term has mean zero
 *              given the past (martingale differences): so has each of the
 *              first four times any function of customers 0..K-1, and each
 *              of the last four (up to the rounding of E S, E A and of the
 *              variates).
 * mrip_run uses dp = 0. Requires 1 <= customers < 2^33, K <= customers. */
typedef struct {
  uint32_t size;
  float lambda, mu;
  uint64_t customers;
  uint64_t feature_prefix;
} mrip_mm1_params;

/* Drossel-Schwabl forest fire, synchronous, grid x grid torus, von Neumann
 * neighbourhood, starting empty. Per step, cell c = y*grid + x reads
 * u = word c&3 of block (t, c>>2, r, 3): burning -> empty; tree -> burning
 * if a neighbour burns or u < floor(f_light 2^32); empty -> tree if
 * u < floor(p_grow 2^32). Output 0 = int32 count of tree -> burning
 * transitions. grid in {64, 128} for WAVE, a multiple of 32 up to 256 for
 * SIMT; grid^2 * steps < 2^31. */
typedef struct {
  uint32_t size;
  uint32_t grid, steps;
  double p_grow, f_light;
} mrip_ff_params;

/* Monte Carlo pi (paper section 5.1, first model): `points` points per
 * replication (1 <= points < 2^31); point i takes words 2(i&1), 2(i&1)+1 of
 * block (i>>1, 0, r, 4), a word's top 24 bits X give u = (X + 1/2) 2^-24, and
 * the point counts when u^2 + v^2 <= 1 (decided exactly in integers).
 * Outputs: 0 = int32 hits, 1 = fp32 estimate 4 hits / points. */
typedef struct {
  uint32_t size;
  uint64_t points;
} mrip_pi_params;

typedef struct {
  uint64_t n;
  double mean, var;        /* var: unbiased, over replications          */
  double half_width;       /* t_quantile * sqrt(var / n)                */
  double t_quantile;       /* Student-t quantile, n - 1 degrees of freedom */
  double confidence;
} mrip_stats_t;

/* One replication of an experimental plan (M/M/1 design point dp). */
typedef struct {
  uint32_t dp, rep;
  uint64_t customers;
  float lambda, mu;
} mrip_plan_item;

/* ---------------------------------------------------------------- context */

/* Validate `params` (a struct matching `model`: mrip_rw_params,
 * mrip_mm1_params, mrip_ff_params or mrip_pi_params) and create a context;
 * no kernel runs. */
MRIP_API mrip_status mrip_create(mrip_ctx *out, mrip_model model, const void *params,
                        mrip_mapping mapping);
MRIP_API void mrip_destroy(mrip_ctx ctx);

/* WAVE launch shape: replications per wavefront (1, 2 or 4; M/M/1 only)
 * and workgroup size (64, 256 or 1024) of the one-wavefront-per-replication
 * kernels, for runs and for plans (mrip_autotune later sets the plans'
 * alone). Outputs do not depend on it. Defaults 1 and 256. Runs of few
 * replications use workgroup-per-replication forms instead, whose size the
 * model fixes: the walk up to 2048 replications (16 lanes per walker), pi
 * below 4096 replications of at least 65536 points (2 to 16 wavefronts). */
MRIP_API mrip_status mrip_set_shape(mrip_ctx ctx, uint32_t reps_per_wave, uint32_t workgroup);

/* Wavefronts per replication for mrip_run on an M/M/1 WAVE context: 1, 2,
 * 4 or 8 (default 1; needs reps_per_wave = 1). With more than one, the
 * wavefronts of a workgroup (256 threads, or 512 for 8) each take an equal
 * run of the replication's customers from an empty system; then every part
 * at once re-runs its leading chunks from the carry its predecessor ended
 * with until the two trajectories meet (Lindley's recursion forgets its
 * start once the queue empties), and, in order, a part whose predecessor
 * never met corrects again from that part's true end. On Philox streams the
 * per-customer values are those of the unsplit run and the means differ
 * only by fp32 summation order; on taus88 streams (at most 4) each lane
 * takes a run of N / (64 split) customers, so values agree to fp32
 * rounding. */
MRIP_API mrip_status mrip_set_split(mrip_ctx ctx, uint32_t waves_per_rep);

/* Stream source of mrip_run (see mrip_rng). TAUS88 is defined for the
 * random walk, M/M/1 and pi models in every mapping; its M/M/1 WAVE engine
 * gives each of the replication's lanes (16, 32 or 64 of a wavefront, or 2
 * or 4 wavefronts with mrip_set_split) a contiguous run of customers.
 * MRIP_E_UNSUPPORTED for the forest fire, for splits over 8 wavefronts, and
 * for later plan or control-variate calls on the context (those use
 * Philox). Builds and uploads the generator's jump tables (22.5 KB; for a
 * walk context also 28 KB of per-walker and per-segment tables) once,
 * synchronously. Default PHILOX. */
MRIP_API mrip_status mrip_set_rng(mrip_ctx ctx, mrip_rng rng);

/* --------------------------------------------------------------- the path */

/* Run replications 0..n_reps-1 with key `seed` (paper section 1: MRIP),
 * then reduce every scalar output over replications in fp64 on the device.
 * Asynchronous on hip_stream. One launch holds fewer than 2^32 lanes:
 * n_reps times the lanes of a replication (1 in SIMT; 64 in LANE0 and
 * WAVE, 64 / reps_per_wave with mrip_set_shape, 64 x waves_per_rep with
 * mrip_set_split) must stay below 2^32 - 1024, else MRIP_E_INVAL (about
 * 67 million replications per call in WAVE). In the split M/M/1 form
 * (WAVE, 2 or 4 wavefronts per replication, Philox, no feature prefix,
 * outputs not bound) the reduction is deferred: the next such run on the
 * same stream computes it in one extra workgroup of its own kernel, so
 * consecutive runs have no event or extra launch between their kernels;
 * asking for the statistics (mrip_stats, mrip_stats_back) or any other
 * launching call computes a reduction still pending. The statistics are
 * the same either way. */
MRIP_API mrip_status mrip_run(mrip_ctx ctx, uint64_t n_reps, uint64_t seed, void *hip_stream);

/* Mean, unbiased variance and Student-t interval of output `output` of the
 * last run (paper section 1). Waits for that run's reduction (an event on
 * its stream). MRIP_E_TOO_FEW if fewer than two replications. */
MRIP_API mrip_status mrip_stats(mrip_ctx ctx, uint32_t output, double confidence, mrip_stats_t *out);

/* The same for the run `back` runs before the last one (0 = the last, at
 * most 3), so a loop may enqueue run k + 1 before it reads run k's interval
 * and keep the device busy meanwhile. Each run (mrip_run, mrip_run_plan)
 * keeps its statistics in its own slot of a 4-run ring in pinned host
 * memory; MRIP_E_STATE for runs no longer kept. Waits for that run only. */
MRIP_API mrip_status mrip_stats_back(mrip_ctx ctx, uint32_t back, uint32_t output,
                                     double confidence, mrip_stats_t *out);

/* Copy output `output` of the last run (n_reps values; 10 per replication
 * for M/M/1 features, 8 for the controls) to dst, a device pointer if
 * dst_is_device, else host.
 * `bytes` must be at least the output's size. Synchronises. */
MRIP_API mrip_status mrip_outputs(mrip_ctx ctx, uint32_t output, void *dst, uint64_t bytes,
                         int dst_is_device);

/* Bind a caller-owned device buffer (for example a torch tensor) as output
 * `output` (a scalar output, 3 = the M/M/1 features or 4 = the controls):
 * later runs and plan runs write there instead of into a buffer of the
 * context, and the statistics reduce it. It must hold at least the run's
 * output (n values, 4 bytes each, 40 per replication for features and 32
 * for the controls; MRIP_E_INVAL at the run
 * otherwise), be 4-byte aligned, and stay alive until the run's results
 * have been read. ptr_dev NULL unbinds (back to the context's buffer). */
MRIP_API mrip_status mrip_bind_output(mrip_ctx ctx, uint32_t output, void *ptr_dev, uint64_t bytes);

/* Device pointer to output `output` of the last run (valid until the next
 * run or mrip_destroy); for zero-copy readers on the same stream. */
MRIP_API mrip_status mrip_output_ptr(mrip_ctx ctx, uint32_t output, const void **ptr_dev);

/* Time one simulation launch of the deferred split M/M/1 form in `every`
 * (1 = every launch, the default; 0 = none) with the HIP events its
 * dispatch records; the other forms time every launch. Each timed launch
 * costs a dispatch gap before the next kernel (about 9 us on MI355X), so a
 * pipelined loop of short runs times a sample. Restarts the count. */
MRIP_API mrip_status mrip_set_timing(mrip_ctx ctx, uint32_t every);

/* Milliseconds of the last timed simulation kernel (hipEvents around the
 * launch on its stream; MRIP_E_STATE if none). Synchronises. */
MRIP_API mrip_status mrip_last_run_ms(mrip_ctx ctx, float *ms);

/* Kernel milliseconds of the last min(max_n, launches, 256) timed simulation
 * launches of this context (mrip_run, mrip_run_plan, autotune), oldest
 * first, into ms[0..*n_out). Synchronises on those launches. */
MRIP_API mrip_status mrip_run_history_ms(mrip_ctx ctx, float *ms, uint32_t max_n,
                                         uint32_t *n_out);

/* --------------------------------- batching: an uneven experimental plan */
/* (paper section 1: an experimental plan runs sets of replications at
 * different factor levels; here all of them in one persistent launch) */

/* Upload a plan (M/M/1 contexts only). Items keep their index for outputs;
 * the device queue serves them longest-first. Host pointer, n >= 1.
 * Synchronises the context's last stream first (an earlier plan run may
 * still be reading the items it replaces). */
MRIP_API mrip_status mrip_plan_set(mrip_ctx ctx, const mrip_plan_item *items, uint64_t n);

/* Run every item of the plan in one persistent-kernel launch whose waves
 * pop work from a device queue, then reduce per design point. Outputs are
 * indexed like the uploaded items. Asynchronous. In the SIMT and LANE0
 * mappings every working lane pops its own items (the thread-per-
 * replication form, where a wavefront runs as long as its longest item);
 * an item's values equal those of a standalone run in the same mapping. */
MRIP_API mrip_status mrip_run_plan(mrip_ctx ctx, uint64_t seed, void *hip_stream);

/* Resume a plan (section 1: an experimental plan is a set of replication
 * runs; a long one may be stopped and restarted): run every uploaded item
 * i with skip_done[i] == 0, longest first as mrip_run_plan does, and leave
 * the outputs of the others as the output buffers hold them (from an
 * earlier plan run on this context, or results the caller restored into a
 * bound output); then reduce every design point over all items.
 * skip_done: host array of n_items bytes, NULL = run everything.
 * Synchronises the stream before reusing its queue buffer; then
 * asynchronous. */
MRIP_API mrip_status mrip_run_plan_resume(mrip_ctx ctx, uint64_t seed, const uint8_t *skip_done,
                                          void *hip_stream);

/* Stopping and resuming a plan (section 1: an experimental plan is a set
 * of replication runs; a long one may be stopped and restarted). Every
 * replication is a pure function of (seed, item), so recovery is running
 * the items that did not finish.
 *
 * mrip_set_plan_limit: with max_items > 0, every later plan run
 * (mrip_run_plan, mrip_run_plan_resume) stops after the first max_items
 * items of its longest-first order, as a run interrupted there would: those
 * items' outputs and done flags are written, the other items' are left as
 * they were, and no statistics are computed (mrip_stats and
 * mrip_plan_stats return MRIP_E_STATE until a run completes). For fault
 * injection and for splitting a plan over several launches. 0 = no limit
 * (the default). */
MRIP_API mrip_status mrip_set_plan_limit(mrip_ctx ctx, uint64_t max_items);

/* The per-item done flags of the last plan run, set by the device as each
 * item's outputs are stored: done[i] = 1 if item i's outputs in the output
 * buffers are final (run by that plan run, or flagged in the skip_done
 * mask it resumed from), else 0. done: host array of n bytes, n = the
 * plan's item count (MRIP_E_INVAL otherwise); MRIP_E_STATE before a plan
 * run. Synchronises. The flags of a stopped run can be passed as skip_done
 * to mrip_run_plan_resume. */
MRIP_API mrip_status mrip_plan_done(mrip_ctx ctx, uint8_t *done, uint64_t n);

/* Stats of output 0 (mean W) over the items of design point `dp` in the
 * last plan run. Synchronises. */
MRIP_API mrip_status mrip_plan_stats(mrip_ctx ctx, uint32_t dp, double confidence, mrip_stats_t *out);

/* Plans: items of at least long_min customers (0 = 65536) are each split
 * over waves_per_item (1, 2, 4 or 8) wavefronts of a workgroup, served first
 * (longest first) at raised wavefront priority, since the longest items set
 * the plan's makespan; the rest go reps_per_wave per wavefront. Until this
 * call (or mrip_autotune) fixes it, a plan takes the fewest wavefronts per
 * long item, up to 8, that bring its longest item's share of its customers
 * down to its average per wavefront the device holds at once (16 per
 * compute unit), the same in every run of the plan (stopped at an item
 * limit or resumed): a plan of many equal long items is not split. */
MRIP_API mrip_status mrip_set_plan_split(mrip_ctx ctx, uint32_t waves_per_item,
                                         uint64_t long_min);

/* Current launch shape: reps_per_wave, workgroup and wavefronts per
 * replication of mrip_run, wavefronts per long plan item (any may be NULL;
 * before mrip_set_plan_split or mrip_autotune fixes it, the most a plan run
 * may use). */
MRIP_API mrip_status mrip_get_shape(mrip_ctx ctx, uint32_t *reps_per_wave, uint32_t *workgroup,
                                    uint32_t *split, uint32_t *plan_split);

/* Time every (reps_per_wave, workgroup) in {1,2,4} x {64,256,1024}, and,
 * when the plan has long items, every reps_per_wave with long items split
 * over 2, 4 or 8 wavefronts (workgroups of 256 threads, 512 for 8), on the
 * uploaded plan (or on an evenly strided slice of `calib_items` items of
 * its longest-first order, 0 = all; each the best of four runs after a
 * warm-up); keep the fastest as the context's plan
 * shape (mrip_run's shape is left as it is) and report its reps_per_wave,
 * the workgroup size it launches and its time (mrip_get_shape gives the
 * split). WAVE contexts only (MRIP_E_UNSUPPORTED otherwise). Synchronises. */
MRIP_API mrip_status mrip_autotune(mrip_ctx ctx, uint64_t seed, uint64_t calib_items, void *hip_stream,
                          uint32_t *best_rpw, uint32_t *best_workgroup, float *best_ms);

/* The autotuner's cache (the paper's section 6 leaves the block size to
 * tune for occupancy). When the environment variable MRIP_TUNE_CACHE names a
 * file, mrip_autotune first looks up the plan's key there and, when found,
 * installs that shape without timing; otherwise it times the shapes and
 * stores the winner. The file holds one line per key: the key, reps per
 * wavefront, workgroup, wavefronts per long item and milliseconds. */
typedef struct {
  uint32_t reps_per_wave, workgroup, plan_split;
  float ms;
} mrip_tune_entry;

/* The cache key of a plan: model, mapping, log2 buckets of the item count,
 * of the long items + 1 and of the longest item's customers, the GPU's
 * architecture name (blanks and '/' become '_') and its compute-unit count,
 * written to out (at most cap bytes with the terminating 0). Host only;
 * MRIP_E_INVAL on NULL or empty arguments, n_items = 0 or a short buffer. */
MRIP_API mrip_status mrip_tune_key(mrip_model model, mrip_mapping mapping, uint64_t n_items,
                                   uint64_t n_long, uint64_t max_customers, const char *arch,
                                   uint32_t cus, char *out, uint64_t cap);
/* The last entry stored for `key` in the cache file at `path`: MRIP_E_STATE
 * when the file or the key is absent, MRIP_E_INVAL on bad arguments. */
MRIP_API mrip_status mrip_tune_cache_get(const char *path, const char *key, mrip_tune_entry *out);
/* Store (or replace) `key`'s entry: the file is rewritten beside the old one
 * and renamed into place. MRIP_E_INVAL on bad arguments or an unwritable
 * path. */
MRIP_API mrip_status mrip_tune_cache_put(const char *path, const char *key,
                                         const mrip_tune_entry *e);

/* ----------------------------------------- learned control variate (CV) */
/* Not in the paper; it extends MRIP's estimator (section 1: the mean of
 * independent replications with a Student-t interval). Per replication of
 * an M/M/1 context with feature prefix K, the controls are F = (h, z_pre):
 *     h = sum_k g_k(x) z_k,
 * z the first four controls of output 4 (after the prefix) divided by the
 * run length N (the two T-weighted ones also by the service scale
 * (float)(1/mu)), g a small network's four outputs from the prefix features
 * x (output 3, z-scored); z_pre the last four (over the prefix), scaled the
 * same way. Since every control term has mean zero given the past and g
 * depends on customers 0..K-1 only, E[F] = 0 for any network: Y - a . F,
 * with a fixed beforehand per bin of rho, is unbiased for E[Y], and no
 * extra replications estimate E[F]. The plain estimate stays the fallback
 * and the reference for its error. */

#define MRIP_MLP_OUT 4        /* network outputs: one coefficient per control */
#define MRIP_MLP_PARAMS 18436 /* W1[128x10] b1[128] W2[128x128] b2[128] W3[4x128] b3[4] */
#define MRIP_CV_BETA_BINS 16  /* coefficient rows over equal bins of rho */
#define MRIP_CV_COEFS 5       /* per row: the network's control h, then the 4 prefix controls */

/* Forward pass of the 10-128-128-4 ReLU network, bf16 operands with fp32
 * accumulation. theta_dev: MRIP_MLP_PARAMS fp32, 16-byte aligned; x_dev:
 * n x 10 fp32 (normalised features); y_dev: n x 4 fp32, 16-byte aligned;
 * n < 2^30.
 * Device pointers; MRIP_E_INVAL on a NULL or misaligned pointer. */
MRIP_API mrip_status mrip_mlp_forward(const float *theta_dev, const float *x_dev, uint64_t n,
                             float *y_dev, void *hip_stream);

/* Gradient of mean((sum_k g_k(x) z_k - y)^2) over the n rows, with z_dev
 * n x 4 fp32 per-row multipliers (16-byte aligned), or NULL for z = (1, 0,
 * 0, 0) (the first output alone): grad_dev gets MRIP_MLP_PARAMS fp32
 * values, loss_dev one fp32 (nullable). theta_dev 16-byte aligned (the
 * weights are read as 16-byte vectors); n <= 65536. Synchronises. */
MRIP_API mrip_status mrip_mlp_grad(const float *theta_dev, const float *x_dev, const float *z_dev,
                          const float *y_dev, uint64_t n, float *grad_dev, float *loss_dev,
                          void *hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * gradient as mrip_mlp_grad, bit for bit, with its per-64-sample partial
 * rows and its bf16 image of the weights in a fixed device array of the
 * library (MRIP_MLP_GRAD_NOALLOC_MAX / 64 rows of 18440 floats and 82960
 * bytes, about 4.8 MB, held by each GPU the library runs on until the
 * process ends) instead of an allocation. Calls no
 * allocating routine and does not synchronise. n <= MRIP_MLP_GRAD_NOALLOC_MAX
 * (MRIP_E_INVAL beyond it); the other arguments as for mrip_mlp_grad. Every
 * call on one GPU shares that array: calls that overlap on one GPU (other
 * streams, other threads) race and must be ordered by the caller. */
#define MRIP_MLP_GRAD_NOALLOC_MAX 4096
MRIP_API mrip_status mrip_mlp_grad_noalloc(const float *theta_dev, const float *x_dev,
                                           const float *z_dev, const float *y_dev, uint64_t n,
                                           float *grad_dev, float *loss_dev, void *hip_stream);

/* One Adam step (Kingma and Ba 2015, Algorithm 1) on fp32 weights;
 * `step` counts from 1; n_params <= 2^32 - 256. */
MRIP_API mrip_status mrip_adam_step(float *theta_dev, float *m_dev, float *v_dev, const float *grad_dev,
                           uint64_t n_params, uint64_t step, float lr, float beta1, float beta2,
                           float eps, void *hip_stream);

typedef struct {
  uint32_t size;
  uint32_t epochs, batch;      /* default 20, 1024 */
  float lr, beta1, beta2, eps; /* default 1e-3, 0.9, 0.999, 1e-8 */
} mrip_cv_hparams;

/* Generate the training set with the M/M/1 engine (items: design points
 * with at least two replications each, disjoint from later apply items;
 * features over the context's feature_prefix customers, the controls after
 * them; response Y = mean W) and train the network from theta0 (host,
 * MRIP_MLP_PARAMS fp32) with Adam on z-scored features: the target is the
 * replication's standardised deviation within its design point,
 * t = (Y - mean_dp Y) / sd_dp Y, fitted by sum_k g_k(x) z_k / sd_dp, over
 * the first four fifths of the design points (ascending ids). On the
 * held-out fifth, fit the coefficient row of each of MRIP_CV_BETA_BINS
 * equal bins of rho = lambda/mu over the training range: the pooled
 * within-design-point least-squares coefficients of Y on F = (h, z_pre); a
 * column without within-design-point variation in a bin gets 0 there, and a
 * bin without design points takes its nearest neighbour's row (the lower on
 * a tie). hparams nullable (defaults). Host item table; synchronises. */
MRIP_API mrip_status mrip_cv_train(mrip_ctx ctx, const mrip_plan_item *items, uint64_t n,
                          const float *theta0, const mrip_cv_hparams *hparams, uint64_t seed,
                          void *hip_stream);

/* Copy the model to host buffers (any may be NULL): weights
 * (MRIP_MLP_PARAMS), feature mean and std (10 + 10), the coefficient table
 * (MRIP_CV_BETA_BINS x MRIP_CV_COEFS, row-major), its rho range (2) and the
 * last epoch's mean training loss (in units of the standardised target:
 * 1 = no skill). */
MRIP_API mrip_status mrip_cv_model(mrip_ctx ctx, float *theta, float *feat_mean, float *feat_std,
                                   float *coef_table, float *rho_range, float *final_loss);

/* Install a model instead of training one: theta (MRIP_MLP_PARAMS fp32),
 * feature mean / std (10 + 10 fp32, std > 0), the coefficient table
 * (MRIP_CV_BETA_BINS x MRIP_CV_COEFS finite values) over rho in
 * [rho_lo, rho_hi]; the network's coefficients are g(x) = net((x - mean) /
 * std). Host pointers. */
MRIP_API mrip_status mrip_cv_set_model(mrip_ctx ctx, const float *theta, const float *feat_mean,
                                       const float *feat_std, const float *coef_table,
                                       float rho_lo, float rho_hi);

/* Apply the trained control variate to n items (host table, at least two
 * replications per design point): one run of the persistent engine with
 * features and controls, inference, and per design point with n
 * replications and a = the table's row at bin(rho):
 *     Y_cv = mean(Y - a . F),  var = s^2(Y - a . F) / n,  dof n - 1,
 * unbiased for any fixed network and table, beside the plain estimate
 * mean(Y), s^2(Y) / n. Synchronises. */
MRIP_API mrip_status mrip_cv_apply(mrip_ctx ctx, const mrip_plan_item *items, uint64_t n,
                          uint64_t seed, void *hip_stream);

/* Per-replication values, in item order, to a host buffer of at least the
 * output's size. Of the last apply: which = 0 Y (mean W), 1 the network's
 * control h, 2 the network outputs g (4 each), 3 the features (10 each), 4
 * the raw controls (8 each, as output 4 of a run). Of the training run
 * behind the model (MRIP_E_STATE after mrip_cv_set_model): 5 Y, 6 the
 * features, 7 the raw controls, 8 the trained network's outputs.
 * Synchronises. */
MRIP_API mrip_status mrip_cv_outputs(mrip_ctx ctx, uint32_t which, void *dst, uint64_t bytes);

/* CV and plain estimates for design point `dp` of the last apply. */
MRIP_API mrip_status mrip_cv_stats(mrip_ctx ctx, uint32_t dp, double confidence, mrip_stats_t *cv,
                          mrip_stats_t *plain);

/* Milliseconds the last apply spent in the simulation kernel (features and
 * controls included) and in inference with the estimator's reductions. */
MRIP_API mrip_status mrip_cv_times(mrip_ctx ctx, float *run_ms, float *infer_ms);

/* ------------------------------------------------------------ utilities */

/* Raw Philox4x32-10 blocks: out_dev[4i..4i+3] = Philox(ctr_dev[4i..4i+3],
 * key = seed). Device pointers, n blocks, n <= 2^32 - 256. */
MRIP_API mrip_status mrip_philox(uint64_t seed, const uint32_t *ctr_dev, uint64_t n, uint32_t *out_dev,
                        void *hip_stream);

/* Raw taus88 outputs: out_dev[i] = output skip + i of the Random Spacing
 * stream of (model tag, dp, rep) under `seed` (see mrip_rng), each reached by
 * jumping from the stream's start with the generator's power-of-two jump
 * tables. Device pointer, n values, n <= 2^32 - 256. Allocates the tables
 * for the call and synchronises the stream before freeing them. */
MRIP_API mrip_status mrip_taus88(uint64_t seed, uint32_t model, uint32_t dp, uint32_t rep,
                                 uint64_t skip, uint64_t n, uint32_t *out_dev, void *hip_stream);

/* Student-t quantile t_{p, dof} for 0.5 <= p < 1, dof > 0 (host). */
MRIP_API double mrip_t_quantile(double p, double dof);

MRIP_API const char *mrip_status_string(mrip_status s);
MRIP_API const char *mrip_last_error(mrip_ctx ctx); /* valid until the next call on ctx */
MRIP_API const char *mrip_version(void);

#ifdef __cplusplus
}
#endif
#endif /* MRIP_H */
