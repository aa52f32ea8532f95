"""The learned control variate end to end on the GPU, against the oracle:
the per-replication values an apply produces (response, features, controls,
network outputs, the network's control), the per-design-point estimator on
those values, the training run's host steps (feature z-scores, coefficient
table) on the library's own training data, training that learns, the
estimator's unbiasedness, and the gain over plain MRIP at equal GPU time."""
import math

import numpy as np
import pytest

from gpu_util import WAVE, announce, rel_err
from oracle import core
from oracle import cv as ocv
from oracle import mlp as omlp
from paper_1501_01405_amd import inputs, mrip

pytestmark = pytest.mark.gpu

K = 1000
BINS, NC = mrip.MRIP_CV_BETA_BINS, mrip.MRIP_CV_COEFS


def _ctx(customers=100000):
    return mrip.Context(mrip.MRIP_MM1, mrip.mm1_params(0.9, 1.0, customers, K), WAVE)


def _model(seed=1):
    theta = inputs.he_uniform_init(seed)
    mean = np.array([0.72, 1, 1.4, 1, 3, 4, 0.3, 20, 0.4, 5], np.float32)
    std = np.array([0.13, 1, 0.1, 0.03, 2, 2, 0.15, 10, 0.1, 5], np.float32)
    return theta, mean, std


def _tuple(items):
    return [(int(i["dp"]), int(i["rep"]), int(i["customers"]), float(i["lambda_"]),
             float(i["mu"])) for i in items]


def _multipliers(ctl, items):
    return np.stack([ocv.control_multipliers(ctl[i], int(items["customers"][i]),
                                             float(items["mu"][i])) for i in range(len(items))])


def _controls_F(G, ctl, items):
    """F = (h, z_pre) from the library's network outputs and raw controls,
    the multipliers rounded to fp32 as the library stores them."""
    Z = _multipliers(ctl, items).astype(np.float32).astype(np.float64)
    h = ocv.control_value(G, Z[:, :4])
    return np.column_stack([h, Z[:, 4:]]), h


def test_apply_matches_oracle_estimator(gpu):
    announce("cv apply vs oracle")
    ctx = _ctx()
    theta, mean, std = _model()
    rng = np.random.default_rng(4)
    coef = rng.normal(size=(BINS, NC)).astype(np.float32)
    mrip.mrip_cv_set_model(ctx.ctx, theta, mean, std, coef, 0.5, 0.95)
    _, items = inputs.cv_design(n_train=10, train_reps=2, n_apply_dp=16, reps=16,
                                customers=20000, seed=11)
    mrip.mrip_cv_apply(ctx.ctx, items, seed=42, stream=mrip.current_stream())
    n = len(items)
    Y = mrip.mrip_cv_outputs(ctx.ctx, 0, n)
    H = mrip.mrip_cv_outputs(ctx.ctx, 1, n)
    G = mrip.mrip_cv_outputs(ctx.ctx, 2, n)
    X = mrip.mrip_cv_outputs(ctx.ctx, 3, n)
    C = mrip.mrip_cv_outputs(ctx.ctx, 4, n)
    # response, features and controls against the oracle M/M/1 (sampled items)
    ids = [0, 5, 77, n - 1]
    ry, rf, rc = core.mm1_items(42, _tuple(items[ids]), features=K, ctl=True)
    assert rel_err(Y[ids], ry[:, 0]).max() <= 1e-5
    cont = [0, 1, 2, 3, 4, 5, 7, 8, 9]
    assert rel_err(X[ids][:, cont], rf[:, cont]).max() <= 1e-5
    es = core.variate_mean(1.0)
    for j, i in enumerate(ids):
        sc = 20000 * es * (1 + float(ry[j, 1]))
        assert np.abs(C[i] - rc[j]).max() <= 1e-5 * sc
    # network outputs against the oracle network on the GPU's own features
    ref_g = omlp.forward(theta, omlp.normalize(X, mean, std), bf16=True)[0]
    assert np.max(np.abs(G - ref_g)) <= 2e-3 * max(1.0, np.max(np.abs(ref_g)))
    # the network's control and the estimator on the GPU's own values
    F, h = _controls_F(G.astype(np.float64), C, items)
    assert np.max(np.abs(H - h)) <= 1e-6 * max(1e-3, np.max(np.abs(h)))
    rho = items["lambda_"] / items["mu"]
    for dp in np.unique(items["dp"]):
        f = items["dp"] == dp
        row = coef[ocv.rho_bin(rho[f][0], 0.5, 0.95, BINS)].astype(np.float64)
        cv_s, plain_s = mrip.mrip_cv_stats(ctx.ctx, int(dp))
        e_cv = ocv.known_mean_control_variate(Y[f], F[f], row)
        e_pl = ocv.plain(Y[f])
        scale = abs(e_pl["mean"]) + np.abs(F[f] @ row).max()
        assert abs(cv_s["mean"] - e_cv["mean"]) <= 1e-6 * scale
        assert abs(cv_s["half_width"] - e_cv["half_width"]) <= 1e-4 * e_cv["half_width"]
        assert abs(plain_s["mean"] - e_pl["mean"]) <= 1e-12 * abs(e_pl["mean"])
        assert abs(plain_s["half_width"] - e_pl["half_width"]) <= 1e-9 * e_pl["half_width"]


def test_zero_table_reduces_to_plain(gpu):
    announce("cv zero coefficients")
    ctx = _ctx()
    theta, mean, std = _model()
    mrip.mrip_cv_set_model(ctx.ctx, theta, mean, std, np.zeros((BINS, NC)), 0.5, 0.95)
    _, items = inputs.cv_design(n_train=10, train_reps=2, n_apply_dp=8, reps=16,
                                customers=5000, seed=3)
    mrip.mrip_cv_apply(ctx.ctx, items, seed=3, stream=mrip.current_stream())
    for dp in np.unique(items["dp"]):
        cv_s, plain_s = mrip.mrip_cv_stats(ctx.ctx, int(dp))
        assert cv_s["mean"] == plain_s["mean"]
        assert abs(cv_s["half_width"] - plain_s["half_width"]) <= 1e-12 * plain_s["half_width"]


def _train(N, n_train=8192, epochs=10, seed=5, n_apply_dp=64, reps=32):
    train, items = inputs.cv_design(n_train=n_train, train_reps=32, n_apply_dp=n_apply_dp,
                                    reps=reps, customers=N, seed=seed)
    ctx = _ctx(N)
    hp = mrip.cv_hparams(epochs=epochs, batch=512, lr=2e-3)
    mrip.mrip_cv_train(ctx.ctx, train, inputs.he_uniform_init(3), hp, seed=42,
                       stream=mrip.current_stream())
    return ctx, train, items


def test_training_host_steps_match_oracle(gpu):
    # the library's own training data through the oracle's host steps:
    # feature z-scores and the per-bin pooled regression on the held-out
    # design points, on the library's network outputs and controls
    announce("cv training host steps vs oracle")
    ctx, train, _ = _train(10000, n_train=4096, epochs=3)
    n = len(train)
    Yt = mrip.mrip_cv_outputs(ctx.ctx, 5, n).astype(np.float64)
    Xt = mrip.mrip_cv_outputs(ctx.ctx, 6, n)
    Ct = mrip.mrip_cv_outputs(ctx.ctx, 7, n)
    Gt = mrip.mrip_cv_outputs(ctx.ctx, 8, n).astype(np.float64)
    model = mrip.mrip_cv_model(ctx.ctx)
    # the training data themselves: sampled items against the oracle M/M/1
    ids = [0, 1000, n - 1]
    ry, rf, _ = core.mm1_items(42, _tuple(train[ids]), features=K, ctl=True)
    assert rel_err(Yt[ids], ry[:, 0]).max() <= 1e-5
    mean, std = ocv.feature_stats(Xt)
    assert rel_err(model["feat_mean"], mean, floor=1e-3).max() <= 1e-6
    assert rel_err(model["feat_std"], std, floor=1e-3).max() <= 1e-6
    # the trained network's outputs are the network's on the z-scored features
    ref_g = omlp.forward(model["theta"], omlp.normalize(Xt[:512], model["feat_mean"],
                                                        model["feat_std"]), bf16=True)[0]
    assert np.max(np.abs(Gt[:512] - ref_g)) <= 2e-3 * max(1.0, np.max(np.abs(ref_g)))
    rho = (train["lambda_"] / train["mu"]).astype(np.float32)
    lo, hi = model["rho_range"]
    assert lo == rho.min() and hi == rho.max()
    hold = np.isin(train["dp"], ocv.holdout_design_points(train["dp"]))
    F, _ = _controls_F(Gt, Ct, train)
    ref = ocv.pooled_regression_table(Yt[hold], F[hold], train["dp"][hold], rho[hold], lo, hi)
    for k in range(BINS):
        assert np.max(np.abs(model["coef"][k] - ref[k])) <= 1e-6 * max(1.0, np.abs(ref[k]).max())


def test_training_learns_and_the_estimator_is_unbiased(gpu):
    announce("cv train + unbiasedness")
    ctx, _, items = _train(10000)
    model = mrip.mrip_cv_model(ctx.ctx)
    # the target is the standardised within-design-point deviation (variance
    # ~1): the controls explain most of it
    assert model["final_loss"] < 0.5
    mrip.mrip_cv_apply(ctx.ctx, items, seed=43, stream=mrip.current_stream())
    diffs, v_cv, v_plain = [], [], []
    for dp in np.unique(items["dp"]):
        cv_s, plain_s = mrip.mrip_cv_stats(ctx.ctx, int(dp))
        diffs.append(cv_s["mean"] - plain_s["mean"])
        v_cv.append(cv_s["var"] / cv_s["n"])
        v_plain.append(plain_s["var"] / plain_s["n"])
    diffs = np.array(diffs)
    # unbiased: the CV - plain differences average to zero
    z = diffs.mean() / (diffs.std(ddof=1) / math.sqrt(len(diffs)))
    vrf = sum(v_plain) / sum(v_cv)
    print("N 1e4: variance reduction", vrf, "bias z", z)
    assert abs(z) < 4.0
    assert vrf > 5.0


def test_gain_at_equal_gpu_time(gpu):
    # runs of 2000 customers, the prefix the first half: the control variate
    # against plain MRIP on the same replications, its half-width ratio
    # scaled to equal GPU time (the plain run in the feature-free plan kernel)
    announce("cv gain at equal time")
    N = 2000
    ctx, _, items = _train(N, epochs=20, seed=11)
    mrip.mrip_cv_apply(ctx.ctx, items, seed=43, stream=mrip.current_stream())
    v_cv, v_plain, diffs = [], [], []
    for dp in np.unique(items["dp"]):
        cv_s, plain_s = mrip.mrip_cv_stats(ctx.ctx, int(dp))
        v_cv.append(cv_s["var"] / cv_s["n"])
        v_plain.append(plain_s["var"] / plain_s["n"])
        diffs.append(cv_s["mean"] - plain_s["mean"])
    run_ms, infer_ms = mrip.mrip_cv_times(ctx.ctx)
    plain = mrip.Context(mrip.MRIP_MM1, mrip.mm1_params(0.9, 1.0, N, 0), WAVE)
    plain.plan_set(items)
    times = []
    for _ in range(5):
        plain.run_plan(seed=43)
        times.append(plain.last_ms())
    t_plain = min(times[1:])
    vrf = sum(v_plain) / sum(v_cv)
    gain = math.sqrt(vrf * t_plain / (run_ms + infer_ms))
    diffs = np.array(diffs)
    z = diffs.mean() / (diffs.std(ddof=1) / math.sqrt(len(diffs)))
    print("N 2000: variance reduction", vrf, "ms", run_ms, infer_ms, t_plain,
          "equal-time gain", gain, "bias z", z)
    assert abs(z) < 4.0
    assert gain > 1.0


def test_apply_rejects_a_design_point_with_one_replication(gpu):
    announce("cv apply input checks")
    ctx = _ctx()
    theta, mean, std = _model()
    mrip.mrip_cv_set_model(ctx.ctx, theta, mean, std, np.zeros((BINS, NC)), 0.5, 0.95)
    items = inputs.uniform_items(2, 2, 2000, [0.6, 0.7])
    with pytest.raises(mrip.MripError):
        mrip.mrip_cv_apply(ctx.ctx, items[:3], seed=1, stream=mrip.current_stream())
    with pytest.raises(mrip.MripError):  # outputs of the training run: none behind this model
        mrip.mrip_cv_outputs(ctx.ctx, 5, 4)
