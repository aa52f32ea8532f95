"""MRIP throughput on one MI355X: simulated events per second, WAVE (one
replication per wavefront) against SIMT (one replication per lane), and the
confidence-interval half-width per GPU-second.

Timed workload (one step = one whole MRIP pass): M/M/1 queue, 1024
replications x 100000 customers, lambda = 0.9, mu = 1, WAVE mapping; the
step runs the replications and the fp64 mean/variance reduction on the
device and builds the 95% interval. Inputs are generated on the device from
the seed (nothing to stage). One JSON line on stdout.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-extras] [--no-cpu]
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

R, N, LAM, MU = 1024, 100000, 0.9, 1.0
SPLIT = 4  # wavefronts per replication (four per SIMD at 1024 replications)
# HBM bytes per launch of mm1_split_kernel<4, false> (reducing the previous
# run, the steady state) from rocprofv3 FETCH_SIZE and WRITE_SIZE, each
# scaled by the same counter on a 256 MiB copy
# (profiles/mm1_split_hbm_counters.md); to be re-measured (or set to None)
# whenever the kernel changes.
TRAFFIC_BYTES = ((212.6 + 203.6) / 2 * 2.00 + 2144.1 * 1.00) * 1024  # taken at SPLIT = 4
# One headline launch in TIMING_EVERY records its kernel's HIP events (the
# kernel duration the roofline uses); the others carry no event.
TIMING_EVERY = 8
# Peak vector issue rate: 256 CUs x 4 SIMDs x 32 lanes x 2.4 GHz, the rate
# behind the published fp32 vector figure (157.3 TFLOP/s counts an FMA as 2).
PEAK_LANE_OPS = 256 * 4 * 32 * 2.4e9

# Issue cost of each instruction class in units of a simple VALU op
# (v_add_u32 / v_xor_b32), from the committed microbenchmark profile
# profiles/valu_rates_gfx950.txt (16 waves per SIMD): v_add_u32 6.12e13/s,
# v_mad_u64_u32 2.89e13/s, v_log_f32 1.94e13/s, v_cvt_f32_u32 ~3.2e13/s.
SLOT_COST = {"mad_u64_u32": 2.12, "log_f32": 3.15, "cvt_f32": 1.9, "simple": 1.0}
# The rate a simple op actually sustains in that microbenchmark (16 waves per
# SIMD, independent chains): the practical ceiling of a slot-weighted mix.
SUSTAINED_LANE_OPS = 6.12e13


def mm1_slots_per_customer(c=SLOT_COST):
    """Algorithmic VALU work per customer, in simple-op slots: half a
    Philox4x32-10 block (10 32x32->64 multiplies, 10 three-input xors), two
    exponential variates (shift, add, convert, scale, log2, scale), the
    Lindley step (two subtract/max pairs and an add) and one add into each of
    the three sums. Scan, compensation and carry instructions are overhead
    and are not counted."""
    philox = 10 * c["mad_u64_u32"] + 10 * c["simple"]
    variates = 2 * (4 * c["simple"] + c["cvt_f32"] + c["log_f32"])
    lindley = 5 * c["simple"]
    sums = 3 * c["simple"]
    return philox + variates + lindley + sums


def philox_block_slots(c=SLOT_COST):
    """One Philox4x32-10 block: 20 32x32->64 multiplies, 20 three-input xors
    (the key schedule runs on the scalar unit)."""
    return 20 * c["mad_u64_u32"] + 20 * c["simple"]


def pi_slots_per_point(c=SLOT_COST):
    """Half a block, each coordinate's odd 25-bit integer (shift, or), the two
    squares summed on v_mad_u64_u32, one 64-bit compare, one add into the
    count."""
    return philox_block_slots(c) / 2 + 4 * c["simple"] + 2 * c["mad_u64_u32"] + 2 * c["simple"]


def ff_slots_per_cell(c=SLOT_COST):
    """A quarter block, the two threshold tests, and the rule on 32-cell
    bit-plane words (about 8 word operations per 32 cells)."""
    return philox_block_slots(c) / 4 + 2 * c["simple"] + 8 / 32 * c["simple"]


def rw_slots_per_step(c=SLOT_COST):
    """1/64 block and about 8 move, unwrapped-offset and wrap operations (the
    LDS or that marks the site is not a VALU op)."""
    return philox_block_slots(c) / 64 + 8 * c["simple"]


def taus88_output_slots(c=SLOT_COST):
    """One taus88 output: three components of shift, xor, shift, and, shift,
    xor each, combined by one three-input xor."""
    return 3 * 6 * c["simple"] + c["simple"]


def taus88_slots(model, c=SLOT_COST):
    """Algorithmic slots per event on taus88 streams: the Philox share of
    each model's count replaced by its taus88 outputs."""
    if model == "mm1":  # two outputs per customer
        return mm1_slots_per_customer(c) - philox_block_slots(c) / 2 + 2 * taus88_output_slots(c)
    if model == "pi":  # two outputs per point
        return pi_slots_per_point(c) - philox_block_slots(c) / 2 + 2 * taus88_output_slots(c)
    return rw_slots_per_step(c) - philox_block_slots(c) / 64 + taus88_output_slots(c) / 16


def alu_roofline(events_per_s, slots):
    achieved = events_per_s * slots
    return {"bound": "alu", "slots_per_event": round(slots, 2), "achieved": achieved / 1e12,
            "peak": PEAK_LANE_OPS / 1e12, "unit": "Tlane-op/s", "frac": achieved / PEAK_LANE_OPS}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=300,
                    help="untimed steps first, back to back like the timed ones: the GPU "
                         "reaches its sustained clock after ~20 ms of continuous work")
    ap.add_argument("--no-extras", action="store_true", help="skip the secondary configs")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=20.0,
                    help="target thread time (CPU seconds) of the CPU-oracle sample")
    ap.add_argument("--copy-calib", action="store_true",
                    help="end with a 256 MiB device-to-device copy (calibrates HBM counters)")
    ap.add_argument("--full-size-counters", action="store_true",
                    help="only run each WAVE workload once at its bench size (for counter runs)")
    ap.add_argument("--split", type=int, default=SPLIT, choices=(2, 4, 8),
                    help="wavefronts per replication of the headline M/M/1 kernel")
    ap.add_argument("--mapping-counters", action="store_true",
                    help="only run the walk and the forest fire once per mapping (for "
                         "rocprofv3 memory counters, the paper's TLP vs WLP table)")
    return ap.parse_args()


def mapping_counters(mrip):
    """The random walk (1024 x 64 walkers x 1000 steps, the paper's model for
    its TLP vs WLP memory-access table), the forest fire (256 x 128^2 x 200)
    and the M/M/1 workload once in each mapping, so that a counter run sees
    one launch of each."""
    maps = (("simt", mrip.MRIP_MAP_SIMT), ("lane0", mrip.MRIP_MAP_LANE0),
            ("wave", mrip.MRIP_MAP_WAVE))
    out = {}
    for name, mp in maps:
        ctx = mrip.Context(mrip.MRIP_RW, mrip.rw_params(64, 64, 1000), mp)
        ctx.run(1024, seed=42)
        out["rw_" + name] = ctx.last_ms()
    for name, mp in (maps[0], maps[2]):
        ctx = mrip.Context(mrip.MRIP_FF, mrip.ff_params(128, 200, 0.01, 1e-5), mp)
        ctx.run(256, seed=42)
        out["ff_" + name] = ctx.last_ms()
    # the headline M/M/1 workload in its three forms (one-lane: 1e4 customers)
    for name, mp, n in (("simt", mrip.MRIP_MAP_SIMT, N), ("lane0", mrip.MRIP_MAP_LANE0, 10000),
                        ("wave", mrip.MRIP_MAP_WAVE, N)):
        ctx = mrip.Context(mrip.MRIP_MM1, mrip.mm1_params(LAM, MU, n), mp)
        if mp == mrip.MRIP_MAP_WAVE:
            ctx.set_split(SPLIT)
        ctx.run(R, seed=42)
        out["mm1_" + name] = ctx.last_ms()
    print(json.dumps({"mapping_counters_kernel_ms": out}), flush=True)


def full_size_counters(mrip):
    """One WAVE launch of each workload at the size bench.py times it (the
    walk also at 16384 replications), so that a counter run sees how busy
    each kernel keeps the vector ALUs at full size."""
    out = {}
    runs = (("mm1_1024x1e5", mrip.MRIP_MM1, mrip.mm1_params(LAM, MU, N), R),
            ("ff_4096x128x128x2000", mrip.MRIP_FF, mrip.ff_params(128, 2000, 0.01, 1e-5), 4096),
            ("pi_1024x1e7", mrip.MRIP_PI, mrip.pi_params(10_000_000), 1024),
            ("rw_32x64x1000", mrip.MRIP_RW, mrip.rw_params(64, 64, 1000), 32),
            ("rw_16384x64x1000", mrip.MRIP_RW, mrip.rw_params(64, 64, 1000), 16384))
    for name, model, params, n in runs:
        ctx = mrip.Context(model, params, mrip.MRIP_MAP_WAVE)
        if model == mrip.MRIP_MM1:
            ctx.set_split(SPLIT)
        ctx.run(n, seed=42)
        out[name] = ctx.last_ms()
    print(json.dumps({"full_size_counters_kernel_ms": out}), flush=True)


def timed_steps(ctx, steps, warmup, torch, mrip):
    """K whole MRIP passes (replications, device reduction, interval). Run
    k's statistics are reduced inside run k + 1's kernel, so reading run k's
    interval waits for that kernel: run k + 2 is enqueued first (the library
    keeps each run's statistics in its own slot of a 4-run ring), and the
    device never waits for the host between steps; every step's interval is
    still read."""
    stream = torch.cuda.current_stream().cuda_stream
    # the kernel's own HIP events on one launch in TIMING_EVERY: each timed
    # launch costs a dispatch gap before the next kernel, the others run
    # back to back
    ctx.set_timing(TIMING_EVERY)

    def loop(n, seed0):
        for i in range(n):
            ctx.run(R, seed=seed0 + i, stream=stream)
            if i >= 2:
                ctx.stats_back(2, 0)  # the interval of step i - 2
        half = None
        for back in range(min(n, 2) - 1, -1, -1):  # the last one or two
            half = ctx.stats_back(back, 0)
        return half

    # warm-up in the same pipelined form: under continuous work the kernel
    # settles within ~20 ms (about 130 runs) at its sustained speed, 5-10 %
    # faster than in the first milliseconds
    if warmup > 0:
        loop(warmup, 1000)
    torch.cuda.synchronize()
    ctx.set_timing(TIMING_EVERY)  # timed launches: steps 0, TIMING_EVERY, ...
    t0 = time.perf_counter()
    half = loop(steps, 42)  # the last step's interval closes the timed region
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    kernel_ms = ctx.history_ms((steps + TIMING_EVERY - 1) // TIMING_EVERY)
    return elapsed, kernel_ms, half


def cpu_baseline(seconds, per_workload=True):
    """The CPU oracle, unchanged, on the same workload: the whole 1024 x 1e5
    run (replication ids 0..1023, one per host thread at a time), repeated
    with new seeds until about `seconds` of thread time (CPU seconds) are spent.
    With per_workload, also the oracle on bounded samples of the secondary
    workloads (each a few hundred ms of wall time), in events per second on
    the same threads, for the GPU/CPU ratios beside each extras row."""
    from oracle import core
    threads = min(core.default_threads(), 16)
    core.mm1_many(7, 1, N, LAM, MU)  # load and warm up
    t0 = time.perf_counter()
    core.mm1_many(7, 4, N, LAM, MU)  # calibrate on four replications
    one = (time.perf_counter() - t0) / 4
    passes = int(min(max(1, round(seconds / max(one * R, 1e-4))), 32))
    t0 = time.perf_counter()
    for k in range(passes):
        core.mm1_many(42 + k, R, N, LAM, MU, threads=threads)
    dt = time.perf_counter() - t0
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    out = {"value": passes * R * N / dt, "unit": "customers/s", "cores": threads,
           "kind": "oracle",
           "sample": "the whole workload (%d replications x %d customers), %d passes "
                     "(seeds 42..%d), %.1f s wall" % (R, N, passes, 41 + passes, dt),
           "single_core": {"value": N / one, "unit": "customers/s", "cores": 1,
                           "sample": "4 replications of the workload (ids 0..3) on one "
                                     "thread, one after the other"},
           "cpu_model": model, "host_cpus": os.cpu_count()}
    if per_workload:
        out["per_workload"] = oracle_workloads(core, threads)
    return out


def oracle_workloads(core, threads):
    """The oracle on the secondary workloads: events/s on `threads` threads."""
    from paper_1501_01405_amd import inputs

    def timed(fn):
        t0 = time.perf_counter()
        fn()
        return time.perf_counter() - t0

    res = {}
    dt = timed(lambda: core.rw_many(42, 32, 64, 64, 1000, threads=threads))
    one = timed(lambda: core.rw_many(42, 4, 64, 64, 1000, threads=1))
    res["rw_32x64x1000"] = {"walker_steps_per_s": 32 * 64 * 1000 / dt,
                            "single_core_walker_steps_per_s": 4 * 64 * 1000 / one,
                            "sample": "the whole workload (32 replications); one core: 4"}
    # pi: one replication of 1e7 points on one core (the paper's CPU-vs-GPU
    # crossover), then one replication per thread
    one = timed(lambda: core.pi_hits(7, 0, 10_000_000))
    dt = timed(lambda: core.pi_many(42, threads, 10_000_000, threads=threads))
    res["pi_1e7"] = {"points_per_s": threads * 1e7 / dt, "s_per_rep_one_core": one,
                     "sample": "%d replications of 1e7 points (of 1024)" % threads}
    n_ff = 2 * threads
    dt = timed(lambda: core.ff_many(42, n_ff, 128, 2000, 0.01, 1e-5, threads=threads))
    one = timed(lambda: core.ff_many(42, 1, 128, 2000, 0.01, 1e-5, threads=1))
    res["ff_4096x128x128x2000"] = {
        "cell_updates_per_s": n_ff * 128 * 128 * 2000 / dt,
        "single_core_cell_updates_per_s": 128 * 128 * 2000 / one,
        "sample": "%d whole replications (of 4096); one core: 1" % n_ff}
    items = inputs.plan_table()
    rows = [(int(i["dp"]), int(i["rep"]), int(i["customers"]), float(i["lambda_"]),
             float(i["mu"])) for i in items]
    dt = timed(lambda: core.mm1_items(42, rows, threads=threads))
    sub = rows[::64]  # every 64th item, the length mix kept
    one = timed(lambda: core.mm1_items(42, sub, threads=1))
    res["plan_64x32"] = {"customers_per_s": float(items["customers"].sum()) / dt,
                         "single_core_customers_per_s": float(sum(r[2] for r in sub)) / one,
                         "sample": "the whole plan (2048 items); one core: every 64th item"}
    return res


def cv_experiment(mrip, inputs, customers, K=1000, runs=3):
    """Learned control variate: train on 1e5 replications (3125 design points
    x 32, rho ~ U[0.5, 0.95]), apply to 256 new design points x 64
    replications; report the pooled variance reduction against plain MRIP on
    the same replications, the half-width ratio at equal GPU time (the plain
    estimate timed on the same items in the feature-free plan kernel, the
    control variate with its features, controls, inference and reductions),
    and the bias z-score of CV - plain over the design points."""
    train, items = inputs.cv_design(n_train=100000, train_reps=32, n_apply_dp=256, reps=64,
                                    customers=customers)
    ctx = mrip.Context(mrip.MRIP_MM1, mrip.mm1_params(0.9, 1.0, customers, K),
                       mrip.MRIP_MAP_WAVE)
    t0 = time.perf_counter()
    mrip.mrip_cv_train(ctx.ctx, train, inputs.he_uniform_init(), mrip.cv_hparams(), seed=42,
                       stream=mrip.current_stream())
    train_s = time.perf_counter() - t0
    model = mrip.mrip_cv_model(ctx.ctx)
    t_cv = []
    for _ in range(runs):  # same seed each time: the same estimates, warm timings
        mrip.mrip_cv_apply(ctx.ctx, items, seed=43, stream=mrip.current_stream())
        run_ms, inf_ms = mrip.mrip_cv_times(ctx.ctx)
        t_cv.append((run_ms + inf_ms, run_ms, inf_ms))
    t_cv_ms, run_ms, inf_ms = min(t_cv)
    plain = mrip.Context(mrip.MRIP_MM1, mrip.mm1_params(0.9, 1.0, customers, 0),
                         mrip.MRIP_MAP_WAVE)
    plain.plan_set(items)
    t_plain = []
    for _ in range(runs):
        plain.run_plan(seed=43)
        t_plain.append(plain.last_ms())
    t_plain_ms = min(t_plain)
    v_cv = v_pl = 0.0
    diffs = []
    for dp in sorted(set(int(d) for d in items["dp"])):
        c, p = mrip.mrip_cv_stats(ctx.ctx, dp)
        v_cv += c["var"] / c["n"]
        v_pl += p["var"] / p["n"]
        diffs.append(c["mean"] - p["mean"])
    n_dp = len(diffs)
    mean_d = sum(diffs) / n_dp
    sd_d = math.sqrt(sum((d - mean_d) ** 2 for d in diffs) / (n_dp - 1))
    vrf = v_pl / v_cv
    return {"customers_per_rep": customers, "prefix": K, "train_s_wall": train_s,
            "train_final_loss": model["final_loss"],
            "coef_h_per_bin": [round(float(b), 4) for b in model["coef"][:, 0]],
            "variance_reduction": vrf, "half_width_ratio_plain_over_cv": math.sqrt(vrf),
            "gpu_ms": {"cv_run": run_ms, "cv_inference": inf_ms, "plain_run": t_plain_ms},
            "equal_time_gain": math.sqrt(vrf * t_plain_ms / t_cv_ms),
            "bias_z": mean_d / (sd_d / math.sqrt(n_dp)) if sd_d > 0 else 0.0}


def extras(torch, mrip, inputs):
    """Secondary configurations, each timed by the library's kernel events."""
    out = {}

    def rate(ctx, n, events, runs=3, seed=42):
        ms = []
        for i in range(runs):
            ctx.run(n, seed=seed + i)
            ms.append(ctx.last_ms())
        return events / (min(ms) * 1e-3), min(ms)

    maps = (("wave", mrip.MRIP_MAP_WAVE), ("simt", mrip.MRIP_MAP_SIMT),
            ("lane0", mrip.MRIP_MAP_LANE0))
    # random walk: 32 reps x 64 walkers x 1000 steps on a 64x64 torus
    for name, mp in maps:
        ctx = mrip.Context(mrip.MRIP_RW, mrip.rw_params(64, 64, 1000), mp)
        v, ms = rate(ctx, 32, 32 * 64 * 1000)
        out.setdefault("rw_32x64x1000", {})[name] = {"walker_steps_per_s": v, "kernel_ms": ms}
    rw = out["rw_32x64x1000"]
    rw["wave"]["roofline"] = alu_roofline(rw["wave"]["walker_steps_per_s"], rw_slots_per_step())
    rw["wave_over_simt"] = rw["wave"]["walker_steps_per_s"] / rw["simt"]["walker_steps_per_s"]
    rw["lane0_over_simt"] = rw["lane0"]["walker_steps_per_s"] / rw["simt"]["walker_steps_per_s"]
    # the paper's replication sweep (its random-walk figure): kernel ms per mapping
    sweep = {}
    for name, mp in maps:
        ctx = mrip.Context(mrip.MRIP_RW, mrip.rw_params(64, 64, 1000), mp)
        for n in (1, 8, 32, 64, 256, 1024, 4096, 16384):
            sweep.setdefault(str(n), {})[name] = rate(ctx, n, n * 64 * 1000, runs=2)[1]
    rw["sweep_kernel_ms"] = sweep
    # the chip filled: 16384 replications in the wavefront mapping
    rw["wave_16384_roofline"] = alu_roofline(16384 * 64 * 1000 / (sweep["16384"]["wave"] * 1e-3),
                                             rw_slots_per_step())

    # Monte Carlo pi, 1e7 draws per replication (the paper's first model):
    # kernel ms against replications per mapping (the oracle's single-core
    # time per replication, for the paper's CPU-vs-GPU crossover, is in
    # cpu_baseline.per_workload)
    psweep = {}
    for name, mp in maps:
        ctx = mrip.Context(mrip.MRIP_PI, mrip.pi_params(10_000_000), mp)
        for n in (1, 8, 32, 64, 256, 1024):
            if name != "wave" and n > 256:
                continue
            psweep.setdefault(str(n), {})[name] = rate(ctx, n, n * 10_000_000, runs=2)[1]
    ctx = mrip.Context(mrip.MRIP_PI, mrip.pi_params(10_000_000), mrip.MRIP_MAP_WAVE)
    v, ms = rate(ctx, 1024, 1024 * 10_000_000, runs=2)
    s_pi = ctx.stats(1)
    out["pi_1e7"] = {"wave_points_per_s_1024reps": v, "sweep_kernel_ms": psweep,
                     "pi_estimate_1024reps": s_pi["mean"], "half_width": s_pi["half_width"],
                     "roofline": alu_roofline(v, pi_slots_per_point())}

    # M/M/1 with the paper's one-working-lane WLP form
    ctx = mrip.Context(mrip.MRIP_MM1, mrip.mm1_params(LAM, MU, N), mrip.MRIP_MAP_LANE0)
    v, ms = rate(ctx, R, R * N, runs=2)
    out["mm1_lane0"] = {"customers_per_s": v, "kernel_ms": ms}
    # the M/M/1 replication sweep (10^4 customers each) in the three mappings
    msweep = {}
    for name, mp in maps:
        ctx = mrip.Context(mrip.MRIP_MM1, mrip.mm1_params(LAM, MU, 10_000), mp)
        for n in (1, 8, 32, 64, 256, 1024, 4096, 16384):
            msweep.setdefault(str(n), {})[name] = rate(ctx, n, n * 10_000, runs=2)[1]
    out["mm1_sweep_1e4_kernel_ms"] = msweep

    # forest fire: 4096 reps x 128^2 x 2000 steps
    ev = 4096 * 128 * 128 * 2000
    ctx = mrip.Context(mrip.MRIP_FF, mrip.ff_params(128, 2000, 0.01, 1e-5), mrip.MRIP_MAP_WAVE)
    v, ms = rate(ctx, 4096, ev, runs=2)
    s = ctx.stats(0)
    ff = {"wave": {"cell_updates_per_s": v, "kernel_ms": ms, "mean_burnt": s["mean"],
                   "half_width": s["half_width"], "roofline": alu_roofline(v, ff_slots_per_cell())}}
    ctx = mrip.Context(mrip.MRIP_FF, mrip.ff_params(128, 2000, 0.01, 1e-5), mrip.MRIP_MAP_SIMT)
    v, ms = rate(ctx, 4096, ev, runs=1)
    ff["simt"] = {"cell_updates_per_s": v, "kernel_ms": ms}
    ff["wave_over_simt"] = ff["wave"]["cell_updates_per_s"] / ff["simt"]["cell_updates_per_s"]
    out["ff_4096x128x128x2000"] = ff

    out["cv_1e5"] = cv_experiment(mrip, inputs, 100000)
    out["cv_1e4"] = cv_experiment(mrip, inputs, 10000)
    out["cv_2e3"] = cv_experiment(mrip, inputs, 2000)  # prefix = half the run

    # the second generator (taus88 with Random Spacing): the same replications
    # on both generators, their kernel times and the z-score of the difference
    # of the two estimates (section 5.3: a second generator checks that the
    # streams do not bias the results)
    cases = (("mm1_1024x1e5_wait", mrip.MRIP_MM1, mrip.mm1_params(LAM, MU, N), 0, R * N,
              min(SPLIT, 4)),  # taus88 replications split over at most 4 wavefronts
             ("pi_1024x1e6", mrip.MRIP_PI, mrip.pi_params(1_000_000), 1, 1024 * 10**6, 1),
             ("rw_1024x64x1000_ssd", mrip.MRIP_RW, mrip.rw_params(64, 64, 1000), 0,
              1024 * 64 * 1000, 1))
    tau = {}
    for name, model, params, o, events, split in cases:
        row = {}
        for gname, g in (("philox", mrip.MRIP_RNG_PHILOX), ("taus88", mrip.MRIP_RNG_TAUS88)):
            ctx = mrip.Context(model, params, mrip.MRIP_MAP_WAVE)
            ctx.set_rng(g)
            ctx.set_split(split)
            v, ms = rate(ctx, 1024, events, runs=2)
            st = ctx.stats(o)
            slots = {"mm1": mm1_slots_per_customer(), "pi": pi_slots_per_point(),
                     "rw": rw_slots_per_step()}[name.split("_")[0]]
            if gname == "taus88":
                slots = taus88_slots(name.split("_")[0])
            row[gname] = {"kernel_ms": ms, "events_per_s": v, "mean": st["mean"],
                          "half_width": st["half_width"], "var": st["var"],
                          "roofline": alu_roofline(v, slots)}
        a, b = row["philox"], row["taus88"]
        row["z_difference"] = (a["mean"] - b["mean"]) / math.sqrt((a["var"] + b["var"]) / 1024)
        tau[name] = row
    out["taus88_vs_philox"] = tau

    # uneven plan: 64 dp x 32 reps, N log-uniform in [1e4, 1e6], one launch
    items = inputs.plan_table()
    ctx = mrip.Context(mrip.MRIP_MM1, mrip.mm1_params(), mrip.MRIP_MAP_WAVE)
    ctx.plan_set(items)
    rpw, wg, tune_ms = ctx.autotune(42)
    ms = []
    for i in range(3):
        ctx.run_plan(42 + i)
        ms.append(ctx.last_ms())
    total = float(items["customers"].sum())
    # the same plan in the thread-per-replication forms (every working lane
    # pops its own items)
    thread_forms = {}
    for name, mp in (("simt", mrip.MRIP_MAP_SIMT), ("lane0", mrip.MRIP_MAP_LANE0)):
        c = mrip.Context(mrip.MRIP_MM1, mrip.mm1_params(), mp)
        c.plan_set(items)
        c.run_plan(42)
        t_ms = c.last_ms()
        thread_forms[name] = {"kernel_ms": t_ms, "customers_per_s": total / (t_ms * 1e-3)}
    out["plan_64x32"] = {"customers": total, "kernel_ms": min(ms),
                         "customers_per_s": total / (min(ms) * 1e-3),
                         "roofline": alu_roofline(total / (min(ms) * 1e-3),
                                                  mm1_slots_per_customer()),
                         "tuned_shape": {"reps_per_wave": rpw, "workgroup": wg},
                         "thread_forms": thread_forms,
                         "wave_over_simt": thread_forms["simt"]["kernel_ms"] / min(ms),
                         "longest_item": int(items["customers"].max())}
    return out


def main():
    global SPLIT
    args = parse()
    SPLIT = args.split
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (replications "
              "would shard by id ranges, with one all-gather of outputs)", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_1501_01405_amd import inputs, mrip
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    mrip.load()
    if args.mapping_counters:
        mapping_counters(mrip)
        return
    if args.full_size_counters:
        full_size_counters(mrip)
        return

    ctx = mrip.Context(mrip.MRIP_MM1, mrip.mm1_params(LAM, MU, N), mrip.MRIP_MAP_WAVE)
    ctx.set_split(SPLIT)
    elapsed, kernel_ms, ci = timed_steps(ctx, args.steps, args.warmup, torch, mrip)
    customers = R * N
    value = customers * args.steps / elapsed
    ms_step = elapsed / args.steps * 1e3
    avg_kernel_ms = sum(kernel_ms) / len(kernel_ms)
    kernel_med = sorted(kernel_ms)[len(kernel_ms) // 2]

    slots = mm1_slots_per_customer()
    achieved = slots * customers / (avg_kernel_ms * 1e-3)

    # SIMT mapping on the same workload (kernel events, outside the timed loop)
    simt = mrip.Context(mrip.MRIP_MM1, mrip.mm1_params(LAM, MU, N), mrip.MRIP_MAP_SIMT)
    simt_ms = []
    for i in range(3):
        simt.run(R, seed=42 + i)
        simt_ms.append(simt.last_ms())
    simt_rate = customers / (min(simt_ms) * 1e-3)
    simt_ci = simt.stats(0)

    line = {
        "metric": "simulated events/sec on 1 MI355X (WLP vs SIMT); CI half-width per GPU-second",
        "value": value,
        "unit": "customers/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (Philox4x32-10 streams generated on the device, seed 42+step)",
        "config": {"workload": "M/M/1 MRIP, 1024 replications x 100000 customers, "
                               "lambda=0.9, mu=1, one replication per %d wavefronts" % SPLIT,
                   "replications": R, "customers": N, "mapping": "WAVE",
                   "waves_per_replication": SPLIT},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12,
                     "peak": PEAK_LANE_OPS / 1e12, "unit": "Tlane-op/s",
                     "frac": achieved / PEAK_LANE_OPS,
                     "traffic": TRAFFIC_BYTES if SPLIT == 4 else None,
                     "kernel": "mm1_split_kernel<%d, false>" % SPLIT, "avg_kernel_ms": avg_kernel_ms,
                     "slots_per_customer": slots,
                     "frac_of_sustained_simple_op_rate": achieved / SUSTAINED_LANE_OPS},
        "kernel_only": {"median_kernel_ms": kernel_med,
                        "customers_per_s": customers / (kernel_med * 1e-3)},
        "ci": {"mean_wq": ci["mean"], "half_width_95": ci["half_width"],
               "gpu_seconds_per_step": ms_step * 1e-3,
               "half_width_x_sqrt_gpu_s": ci["half_width"] * math.sqrt(ms_step * 1e-3)},
        "simt": {"customers_per_s": simt_rate, "kernel_ms": min(simt_ms),
                 "half_width_x_sqrt_gpu_s": simt_ci["half_width"] *
                 math.sqrt(min(simt_ms) * 1e-3)},
        "wave_over_simt": (customers / (avg_kernel_ms * 1e-3)) / simt_rate,
        "paper_reference": "WLP up to ~6x faster than SIMT: Tesla C2050 (Fermi), random walk, "
                           "1000 steps, taus88 PRNG (context, not a target)",
    }
    if not args.no_extras:
        line["extras"] = extras(torch, mrip, inputs)
    if args.copy_calib:
        src = torch.empty(64 * 1024 * 1024, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(args.cpu_seconds, per_workload=not args.no_extras)
        if "extras" in line:
            # GPU (WAVE, kernel events) over the oracle on the host threads
            ex, cpu = line["extras"], line["cpu_baseline"]["per_workload"]
            gpu = {"rw_32x64x1000": ex["rw_32x64x1000"]["wave"]["walker_steps_per_s"],
                   "pi_1e7": ex["pi_1e7"]["wave_points_per_s_1024reps"],
                   "ff_4096x128x128x2000": ex["ff_4096x128x128x2000"]["wave"]["cell_updates_per_s"],
                   "plan_64x32": ex["plan_64x32"]["customers_per_s"]}
            for k, v in gpu.items():
                rate = [x for key, x in cpu[k].items() if key.endswith("_per_s")][0]
                cpu[k]["gpu_over_oracle"] = v / rate
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
