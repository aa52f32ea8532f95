"""The learned control variate end to end on the GPU: per-design-point CV
and plain statistics against the oracle estimator on the GPU's own
per-replication values, features against the oracle's M/M/1, the constant
network reducing to plain MRIP, training that learns, and unbiasedness."""
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
GAIN_INFORMATIVE = 1.2  # half-width ratio; measured 1.32 with these seeds


def _ctx():
    return mrip.Context(mrip.MRIP_MM1, mrip.mm1_params(0.9, 1.0, 100000, K), WAVE)


def _small_design(n_dp=16, reps=16, pre=64, customers=20000, seed=11):
    _, full, pref = inputs.cv_design(n_train=10, train_reps=2, n_apply_dp=n_dp, reps=reps,
                                     prefix_reps=pre, customers=customers, prefix=K, seed=seed)
    return full, pref


def _model(seed=1):
    theta = inputs.he_uniform_init(seed)
    mean = np.array([0.72, 1, 1.4, 1, 3, 4, 0.3, 20, 0.4, 5], np.float32)
    std = np.array([0.13, 1, 0.1, 0.03, 2, 2, 0.15, 10, 0.1, 5], np.float32)
    return theta, mean, std


def _tuple(items):
    return [(int(i["dp"]), int(i["rep"]), int(i["customers"]), float(i["lambda_"]),
             float(i["mu"])) for i in items]


def test_cv_statistics_match_oracle_estimator(gpu):
    announce("cv apply vs oracle")
    ctx = _ctx()
    theta, mean, std = _model()
    mrip.mrip_cv_set_model(ctx.ctx, theta, mean, std, 1.0, 0.5, 0.95)
    full, pref = _small_design()
    mrip.mrip_cv_apply(ctx.ctx, full, pref, seed=42, stream=mrip.current_stream())
    Y = mrip.mrip_cv_outputs(ctx.ctx, 0, len(full))
    G = mrip.mrip_cv_outputs(ctx.ctx, 1, len(full))
    Gp = mrip.mrip_cv_outputs(ctx.ctx, 2, len(pref))
    X = mrip.mrip_cv_outputs(ctx.ctx, 3, len(full))
    Xp = mrip.mrip_cv_outputs(ctx.ctx, 4, len(pref))
    # features and targets against the oracle M/M/1 (sampled items)
    ids = [0, 5, len(full) - 1]
    ry, rf = core.mm1_items(42, _tuple(full[ids]), features=K)
    assert rel_err(Y[ids], ry[:, 0]).max() <= 1e-5
    cont = [0, 1, 2, 3, 4, 5, 7, 8, 9]
    assert rel_err(X[ids][:, cont], rf[:, cont]).max() <= 1e-5
    pids = [0, 17, len(pref) - 1]
    _, rfp = core.mm1_items(42, _tuple(pref[pids]), features=K)
    assert rel_err(Xp[pids][:, cont], rfp[:, cont]).max() <= 1e-5
    # predictions against the oracle network on the GPU's own features
    xn = omlp.normalize(X, mean, std)
    ref_g = omlp.forward(theta, xn, bf16=True)[0]
    assert np.max(np.abs(G - ref_g)) <= 2e-3 * max(1.0, np.max(np.abs(ref_g)))
    # per-dp estimators against the oracle's, on the same per-rep values
    for dp in np.unique(full["dp"])[:6]:
        f = full["dp"] == dp
        p = pref["dp"] == dp
        cv_s, plain_s = mrip.mrip_cv_stats(ctx.ctx, int(dp))
        beta = 1.0 * p.sum() / (p.sum() + f.sum())  # beta * M / (M + n)
        e_cv = ocv.control_variate(Y[f], G[f], Gp[p], beta=beta)
        e_pl = ocv.plain(Y[f])
        assert abs(cv_s["mean"] - e_cv["mean"]) <= 1e-6 * abs(e_cv["mean"])
        assert abs(cv_s["half_width"] - e_cv["half_width"]) <= 1e-5 * e_cv["half_width"]
        assert abs(plain_s["mean"] - e_pl["mean"]) <= 1e-12 * abs(e_pl["mean"])
        assert abs(plain_s["half_width"] - e_pl["half_width"]) <= 1e-9 * e_pl["half_width"]


def test_constant_network_reduces_to_plain(gpu):
    announce("cv constant network")
    ctx = _ctx()
    theta, mean, std = _model()
    d = omlp.unpack(theta.astype(np.float64))
    d = {k: v.copy() for k, v in d.items()}
    d["W3"][:] = 0.0
    d["b3"][:] = 0.25
    mrip.mrip_cv_set_model(ctx.ctx, omlp.pack(d).astype(np.float32), mean, std, 2.0, 0.5, 0.95)
    full, pref = _small_design(n_dp=8)
    mrip.mrip_cv_apply(ctx.ctx, full, pref, seed=3, stream=mrip.current_stream())
    for dp in np.unique(full["dp"]):
        cv_s, plain_s = mrip.mrip_cv_stats(ctx.ctx, int(dp))
        assert abs(cv_s["mean"] - plain_s["mean"]) <= 1e-6 * plain_s["mean"]
        assert abs(cv_s["half_width"] - plain_s["half_width"]) <= 1e-5 * plain_s["half_width"]


def test_training_learns_and_cv_is_unbiased(gpu):
    announce("cv train + unbiasedness")
    train, full, pref = inputs.cv_design(n_train=8192, train_reps=32, n_apply_dp=64, reps=32,
                                         prefix_reps=128, customers=10000, prefix=K, seed=5)
    ctx = mrip.Context(mrip.MRIP_MM1, mrip.mm1_params(0.9, 1.0, 10000, K), WAVE)
    hp = mrip.cv_hparams(epochs=10, batch=512, lr=2e-3)
    mrip.mrip_cv_train(ctx.ctx, train, inputs.he_uniform_init(3), hp, seed=42,
                       stream=mrip.current_stream())
    model = mrip.mrip_cv_model(ctx.ctx)
    # the target is the standardised within-design-point deviation (variance
    # ~1): a loss below 1 means the prefix features carry information
    assert model["final_loss"] < 1.0
    assert np.all(model["beta"] >= 0.0)
    mrip.mrip_cv_apply(ctx.ctx, full, pref, seed=43, stream=mrip.current_stream())
    diffs, v_cv, v_plain = [], [], []
    for dp in np.unique(full["dp"]):
        cv_s, plain_s = mrip.mrip_cv_stats(ctx.ctx, int(dp))
        diffs.append(cv_s["mean"] - plain_s["mean"])
        v_cv.append(cv_s["var"] / cv_s["n"])
        v_plain.append(plain_s["var"] / plain_s["n"])
    diffs = np.array(diffs)
    # unbiased: the CV - plain differences average to zero
    z = diffs.mean() / (diffs.std(ddof=1) / math.sqrt(len(diffs)))
    assert abs(z) < 4.0
    # the prefix of a 1e4-customer run carries a little information; with the
    # fitted coefficients the pooled variance is not worse than plain MRIP
    gain = math.sqrt(sum(v_plain) / sum(v_cv))
    print("pooled half-width gain", gain, "beta", model["beta"])
    assert gain > 0.97


def test_network_gains_when_the_prefix_is_informative(gpu):
    # runs of 2000 customers whose features cover the first 1000: the prefix
    # carries much of the run's mean wait, and the trained control variate
    # must narrow the interval against plain MRIP on the same replications
    # (the full-size configuration's modest gain is reported by the bench)
    announce("cv gain, informative prefix")
    train, full, pref = inputs.cv_design(n_train=8192, train_reps=32, n_apply_dp=64, reps=32,
                                         prefix_reps=256, customers=2000, prefix=K, seed=11)
    ctx = mrip.Context(mrip.MRIP_MM1, mrip.mm1_params(0.9, 1.0, 2000, K), WAVE)
    hp = mrip.cv_hparams(epochs=20, batch=512, lr=2e-3)
    mrip.mrip_cv_train(ctx.ctx, train, inputs.he_uniform_init(3), hp, seed=42,
                       stream=mrip.current_stream())
    mrip.mrip_cv_apply(ctx.ctx, full, pref, seed=43, stream=mrip.current_stream())
    v_cv, v_plain, diffs = [], [], []
    for dp in np.unique(full["dp"]):
        cv_s, plain_s = mrip.mrip_cv_stats(ctx.ctx, int(dp))
        v_cv.append(cv_s["var"] / cv_s["n"])
        v_plain.append(plain_s["var"] / plain_s["n"])
        diffs.append(cv_s["mean"] - plain_s["mean"])
    gain = math.sqrt(sum(v_plain) / sum(v_cv))
    diffs = np.array(diffs)
    z = diffs.mean() / (diffs.std(ddof=1) / math.sqrt(len(diffs)))
    print("informative prefix: half-width gain", gain, "bias z", z)
    assert abs(z) < 4.0
    assert gain > GAIN_INFORMATIVE
