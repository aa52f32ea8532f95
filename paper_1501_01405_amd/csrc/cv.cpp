// Learned control variate (not in the paper; it extends MRIP's estimator):
// training-set generation with the M/M/1 engine, training of the bf16-MFMA
// network with Adam, and the two-phase control-variate estimate per design
// point, next to the plain MRIP estimate that stays its fallback.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/mrip.h"
#include "context.hpp"
#include "kernels.hpp"
#include "mlp.hpp"

namespace mrip {
double t_quantile(double p, double nu);
}

using namespace mrip;

namespace {

mrip_status fail(mrip_ctx c, hipError_t e, const char *what) {
  if (c) c->err = std::string(what) + ": " + hipGetErrorString(e);
  return MRIP_E_HIP;
}

#define CV_TRY(ctx, expr)                                 \
  do {                                                    \
    hipError_t _e = (expr);                               \
    if (_e != hipSuccess) return fail((ctx), _e, #expr);  \
  } while (0)

mrip_status bad(mrip_ctx c, const char *why) {
  if (c) c->err = why;
  return MRIP_E_INVAL;
}

AdamArgs adam_args(float lr, float b1, float b2, float eps, uint64_t step) {
  AdamArgs a;
  a.lr = lr;
  a.beta1 = b1;
  a.beta2 = b2;
  a.eps = eps;
  a.bc1 = (float)(1.0 - std::pow((double)b1, (double)step));
  a.bc2 = (float)(1.0 - std::pow((double)b2, (double)step));
  return a;
}

// Upload items (SoA), their longest-first order and their dp grouping.
mrip_status upload_items(mrip_ctx c, const mrip_plan_item *items, uint64_t n, uint64_t K,
                         ItemBufs &b) {
  if (!items || n == 0) return bad(c, "empty item table");
  if (n > 0xFFFFFFFFull) return bad(c, "item table too large");
  std::vector<uint32_t> dp(n), rep(n), order(n), index(n);
  std::vector<uint64_t> cust(n);
  std::vector<float> lam(n), mu(n);
  for (uint64_t i = 0; i < n; ++i) {
    const mrip_plan_item &it = items[i];
    if (it.customers < 1 || it.customers >= (1ull << 33)) return bad(c, "item customers out of range");
    if (it.customers < K) return bad(c, "item shorter than the feature prefix");
    if (!(it.lambda > 0.0f) || !(it.mu > 0.0f) || !std::isfinite(it.lambda) || !std::isfinite(it.mu))
      return bad(c, "item rates must be finite and > 0");
    dp[i] = it.dp;
    rep[i] = it.rep;
    cust[i] = it.customers;
    lam[i] = it.lambda;
    mu[i] = it.mu;
    order[i] = index[i] = (uint32_t)i;
  }
  std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b2) { return cust[a] > cust[b2]; });
  std::stable_sort(index.begin(), index.end(), [&](uint32_t a, uint32_t b2) { return dp[a] < dp[b2]; });
  b.dp_ids.clear();
  b.group_offsets.clear();
  for (uint64_t j = 0; j < n; ++j) {
    if (j == 0 || dp[index[j]] != dp[index[j - 1]]) {
      b.group_offsets.push_back(j);
      b.dp_ids.push_back(dp[index[j]]);
    }
  }
  b.group_offsets.push_back(n);
  b.index_host = index;
  b.max_customers = *std::max_element(cust.begin(), cust.end());
  CV_TRY(c, b.dp.ensure(4 * n));
  CV_TRY(c, b.rep.ensure(4 * n));
  CV_TRY(c, b.n.ensure(8 * n));
  CV_TRY(c, b.lambda.ensure(4 * n));
  CV_TRY(c, b.mu.ensure(4 * n));
  CV_TRY(c, b.order.ensure(4 * n));
  CV_TRY(c, b.index.ensure(4 * n));
  CV_TRY(c, b.offsets.ensure(8 * b.group_offsets.size()));
  CV_TRY(c, hipMemcpy(b.dp.p, dp.data(), 4 * n, hipMemcpyHostToDevice));
  CV_TRY(c, hipMemcpy(b.rep.p, rep.data(), 4 * n, hipMemcpyHostToDevice));
  CV_TRY(c, hipMemcpy(b.n.p, cust.data(), 8 * n, hipMemcpyHostToDevice));
  CV_TRY(c, hipMemcpy(b.lambda.p, lam.data(), 4 * n, hipMemcpyHostToDevice));
  CV_TRY(c, hipMemcpy(b.mu.p, mu.data(), 4 * n, hipMemcpyHostToDevice));
  CV_TRY(c, hipMemcpy(b.order.p, order.data(), 4 * n, hipMemcpyHostToDevice));
  CV_TRY(c, hipMemcpy(b.index.p, index.data(), 4 * n, hipMemcpyHostToDevice));
  CV_TRY(c, hipMemcpy(b.offsets.p, b.group_offsets.data(), 8 * b.group_offsets.size(),
                      hipMemcpyHostToDevice));
  b.count = n;
  return MRIP_OK;
}

// Run an item table through the persistent M/M/1 kernel with feature
// capture over the first K customers; `ms` (nullable) gets the kernel time.
mrip_status run_items(mrip_ctx c, ItemBufs &b, uint64_t seed, uint64_t K, float *mean_w,
                      float *feat, hipStream_t s, float *ms) {
  CvState &cv = c->cv;
  CV_TRY(c, cv.queue.ensure(256));
  CV_TRY(c, cv.scratch_t.ensure(4 * b.count));
  CV_TRY(c, cv.scratch_i.ensure(4 * b.count));
  Mm1Args a{};
  a.seed = seed;
  a.feature_prefix = K;
  a.items.dp = b.dp.as<uint32_t>();
  a.items.rep = b.rep.as<uint32_t>();
  a.items.customers = b.n.as<uint64_t>();
  a.items.lambda = b.lambda.as<float>();
  a.items.mu = b.mu.as<float>();
  a.items.order = b.order.as<uint32_t>();
  a.queue_head = cv.queue.as<uint32_t>();
  a.mean_w = mean_w;
  a.mean_t = cv.scratch_t.as<float>();
  a.mean_i = cv.scratch_i.as<float>();
  a.features = feat;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (ms) {
    CV_TRY(c, hipEventCreate(&e0));
    CV_TRY(c, hipEventCreate(&e1));
  }
  CV_TRY(c, launch_zero_u32(a.queue_head, 2, s));
  if (ms) CV_TRY(c, hipEventRecord(e0, s));
  // short replications (prefix-only runs) share a wavefront four at a time
  const uint32_t rpw = b.max_customers <= 4096 ? 4u : c->rpw;
  CV_TRY(c, launch_mm1_plan(a, b.count, rpw, c->wg, s));
  if (ms) {
    CV_TRY(c, hipEventRecord(e1, s));
    CV_TRY(c, hipEventSynchronize(e1));
    CV_TRY(c, hipEventElapsedTime(ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
  }
  return MRIP_OK;
}

std::mutex g_grad_mu;
DevBuf g_grad_partial;  // partial-gradient rows for the context-free mrip_mlp_grad

}  // namespace

extern "C" {

mrip_status mrip_mlp_forward(const float *theta_dev, const float *x_dev, uint64_t n, float *y_dev,
                             void *hip_stream) {
  if (n > 0 && (!theta_dev || !x_dev || !y_dev)) return MRIP_E_INVAL;
  if (n >= (1ull << 30)) return MRIP_E_INVAL;  // 4 lanes per row: one launch < 2^32 lanes
  hipError_t e = launch_mlp_forward(theta_dev, x_dev, n, y_dev, 1.0f, 0.0f, (hipStream_t)hip_stream);
  return e == hipSuccess ? MRIP_OK : MRIP_E_HIP;
}

mrip_status mrip_mlp_grad(const float *theta_dev, const float *x_dev, const float *y_dev,
                          uint64_t n, float *grad_dev, float *loss_dev, void *hip_stream) {
  if (n == 0 || n > 65536 || !theta_dev || !x_dev || !y_dev || !grad_dev) return MRIP_E_INVAL;
  std::lock_guard<std::mutex> lock(g_grad_mu);
  hipStream_t s = (hipStream_t)hip_stream;
  const size_t rows = mlp_partial_rows(n);
  if (g_grad_partial.ensure(rows * MLP_PSTRIDE * sizeof(float)) != hipSuccess) return MRIP_E_NOMEM;
  if (launch_mlp_grad(theta_dev, x_dev, y_dev, n, g_grad_partial.as<float>(), s) != hipSuccess)
    return MRIP_E_HIP;
  AdamArgs none{};
  if (launch_grad_reduce(g_grad_partial.as<float>(), (uint32_t)rows, n, grad_dev, loss_dev, nullptr,
                         nullptr, nullptr, none, s) != hipSuccess)
    return MRIP_E_HIP;
  // the shared partial buffer must not be reused before this call's kernels ran
  return hipStreamSynchronize(s) == hipSuccess ? MRIP_OK : MRIP_E_HIP;
}

mrip_status mrip_adam_step(float *theta_dev, float *m_dev, float *v_dev, const float *grad_dev,
                           uint64_t n_params, uint64_t step, float lr, float beta1, float beta2,
                           float eps, void *hip_stream) {
  if (step == 0 || (n_params > 0 && (!theta_dev || !m_dev || !v_dev || !grad_dev)))
    return MRIP_E_INVAL;
  if (n_params > 0xFFFFFF00ull) return MRIP_E_INVAL;  // one lane per parameter
  hipError_t e = launch_adam(theta_dev, m_dev, v_dev, grad_dev, n_params,
                             adam_args(lr, beta1, beta2, eps, step), (hipStream_t)hip_stream);
  return e == hipSuccess ? MRIP_OK : MRIP_E_HIP;
}

mrip_status mrip_cv_train(mrip_ctx ctx, const mrip_plan_item *items, uint64_t n,
                          const float *theta0, const mrip_cv_hparams *hp_in, uint64_t seed,
                          void *hip_stream) {
  if (!ctx) return MRIP_E_INVAL;
  if (ctx->rng != MRIP_RNG_PHILOX)
    return (ctx->err = "the control variate uses Philox streams"), MRIP_E_UNSUPPORTED;
  if (ctx->model != MRIP_MM1) return (ctx->err = "the control variate needs an M/M/1 context"), MRIP_E_UNSUPPORTED;
  const uint64_t K = ctx->mm1.feature_prefix;
  if (K == 0) return bad(ctx, "the context needs feature_prefix > 0");
  if (!theta0) return bad(ctx, "theta0 is NULL");
  mrip_cv_hparams hp{sizeof(mrip_cv_hparams), 20, 1024, 1e-3f, 0.9f, 0.999f, 1e-8f};
  if (hp_in) {
    if (hp_in->size != sizeof(mrip_cv_hparams)) return bad(ctx, "mrip_cv_hparams.size mismatch");
    hp = *hp_in;
  }
  if (hp.epochs < 1 || hp.batch < 1 || hp.batch > 65536 || !(hp.lr > 0.f))
    return bad(ctx, "bad training hyperparameters");
  hipStream_t s = (hipStream_t)hip_stream;
  CvState &cv = ctx->cv;
  cv.trained = false;

  mrip_status st = upload_items(ctx, items, n, K, cv.train_items);
  if (st != MRIP_OK) return st;
  ItemBufs &tb = cv.train_items;
  const size_t G = tb.dp_ids.size();
  if (G < 2) return bad(ctx, "training needs at least two design points");
  for (size_t g = 0; g < G; ++g)
    if (tb.group_offsets[g + 1] - tb.group_offsets[g] < 2)
      return bad(ctx, "every training design point needs two replications");

  CV_TRY(ctx, cv.y_train.ensure(4 * n));
  CV_TRY(ctx, cv.x_train.ensure(40 * n));
  CV_TRY(ctx, cv.xn.ensure(40 * n));
  CV_TRY(ctx, cv.yn.ensure(4 * n));
  CV_TRY(ctx, cv.t_train.ensure(4 * n));
  CV_TRY(ctx, cv.red_y.ensure(sizeof(double) * 3 * G));
  hipEvent_t e0, e1;
  CV_TRY(ctx, hipEventCreate(&e0));
  CV_TRY(ctx, hipEventCreate(&e1));
  CV_TRY(ctx, hipEventRecord(e0, s));
  st = run_items(ctx, tb, seed, K, cv.y_train.as<float>(), cv.x_train.as<float>(), s, nullptr);
  if (st != MRIP_OK) return st;

  // target: the replication's standardised deviation from its design
  // point's mean, so the network models the within-design-point variation a
  // control variate can use, at the same scale for every factor level
  const std::vector<uint32_t> &index = tb.index_host;
  std::vector<uint32_t> group(n);
  for (size_t g = 0; g < G; ++g)
    for (uint64_t j = tb.group_offsets[g]; j < tb.group_offsets[g + 1]; ++j) group[index[j]] = (uint32_t)g;
  DevBuf group_d;
  CV_TRY(ctx, group_d.ensure(4 * n));
  CV_TRY(ctx, hipMemcpy(group_d.p, group.data(), 4 * n, hipMemcpyHostToDevice));
  CV_TRY(ctx, launch_reduce_f64_gather(cv.y_train.p, 1, tb.index.as<uint32_t>(),
                                       tb.offsets.as<uint64_t>(), (uint32_t)G,
                                       cv.red_y.as<double>(), s));
  CV_TRY(ctx, launch_center(cv.y_train.as<float>(), group_d.as<uint32_t>(), cv.red_y.as<double>(),
                            n, cv.t_train.as<float>(), s));

  // feature z-scores over the training set
  CV_TRY(ctx, cv.colstats.ensure(sizeof(double) * 20));
  CV_TRY(ctx, launch_col_stats(cv.x_train.as<float>(), n, 10, cv.colstats.as<double>(), s));
  double cs[20];
  CV_TRY(ctx, hipMemcpyAsync(cs, cv.colstats.p, sizeof(cs), hipMemcpyDeviceToHost, s));
  CV_TRY(ctx, hipStreamSynchronize(s));
  cv.mean.assign(10, 0.f);
  cv.std_.assign(10, 1.f);
  float host_norm[20];
  for (int j = 0; j < 10; ++j) {
    cv.mean[j] = (float)cs[2 * j];
    cv.std_[j] = cs[2 * j + 1] > 1e-12 ? (float)cs[2 * j + 1] : 1.0f;
    host_norm[j] = cv.mean[j];
    host_norm[10 + j] = 1.0f / cv.std_[j];
  }
  CV_TRY(ctx, cv.norm.ensure(sizeof(host_norm)));
  CV_TRY(ctx, hipMemcpy(cv.norm.p, host_norm, sizeof(host_norm), hipMemcpyHostToDevice));

  // hold out the last fifth of the design points (whole groups) to fit the
  // coefficients; rows are permuted so that the training rows come first
  const size_t g_hold = G >= 5 ? G / 5 : 1;
  const size_t g_fit = G - g_hold;
  std::vector<uint32_t> perm;
  perm.reserve(n);
  for (size_t g = 0; g < G; ++g)
    for (uint64_t j = tb.group_offsets[g]; j < tb.group_offsets[g + 1]; ++j) perm.push_back(index[j]);
  const uint64_t n_fit = tb.group_offsets[g_fit];
  const uint64_t n_hold = n - n_fit;
  DevBuf perm_d, one;
  CV_TRY(ctx, perm_d.ensure(4 * n));
  CV_TRY(ctx, hipMemcpy(perm_d.p, perm.data(), 4 * n, hipMemcpyHostToDevice));
  const float unit[2] = {0.0f, 1.0f};
  CV_TRY(ctx, one.ensure(sizeof(unit)));
  CV_TRY(ctx, hipMemcpy(one.p, unit, sizeof(unit), hipMemcpyHostToDevice));
  const float *mean_d = cv.norm.as<float>(), *inv_d = cv.norm.as<float>() + 10;
  CV_TRY(ctx, launch_gather_normalize(cv.x_train.as<float>(), perm_d.as<uint32_t>(), n, 10, mean_d,
                                      inv_d, cv.xn.as<float>(), s));
  CV_TRY(ctx, launch_gather_normalize(cv.t_train.as<float>(), perm_d.as<uint32_t>(), n, 1,
                                      one.as<float>(), one.as<float>() + 1, cv.yn.as<float>(), s));

  // Adam from theta0
  CV_TRY(ctx, cv.theta.ensure(4 * MLP_NPARAMS));
  CV_TRY(ctx, cv.adam_m.ensure(4 * MLP_NPARAMS));
  CV_TRY(ctx, cv.adam_v.ensure(4 * MLP_NPARAMS));
  CV_TRY(ctx, hipMemcpy(cv.theta.p, theta0, 4 * MLP_NPARAMS, hipMemcpyHostToDevice));
  CV_TRY(ctx, hipMemsetAsync(cv.adam_m.p, 0, 4 * MLP_NPARAMS, s));
  CV_TRY(ctx, hipMemsetAsync(cv.adam_v.p, 0, 4 * MLP_NPARAMS, s));
  const uint64_t batches = (n_fit + hp.batch - 1) / hp.batch;
  const uint64_t steps = batches * hp.epochs;
  CV_TRY(ctx, cv.loss_hist.ensure(4 * steps));
  CV_TRY(ctx, cv.partial.ensure(mlp_partial_rows(hp.batch) * MLP_PSTRIDE * sizeof(float)));
  uint64_t step = 0;
  for (uint32_t ep = 0; ep < hp.epochs; ++ep) {
    for (uint64_t b = 0; b < batches; ++b) {
      const uint64_t r0 = b * hp.batch;
      const uint64_t nb = std::min<uint64_t>(hp.batch, n_fit - r0);
      ++step;
      CV_TRY(ctx, launch_mlp_grad(cv.theta.as<float>(), cv.xn.as<float>() + r0 * 10,
                                  cv.yn.as<float>() + r0, nb, cv.partial.as<float>(), s));
      CV_TRY(ctx, launch_grad_reduce(cv.partial.as<float>(), (uint32_t)mlp_partial_rows(nb), nb,
                                     nullptr, cv.loss_hist.as<float>() + (step - 1),
                                     cv.theta.as<float>(), cv.adam_m.as<float>(),
                                     cv.adam_v.as<float>(),
                                     adam_args(hp.lr, hp.beta1, hp.beta2, hp.eps, step), s));
    }
  }
  CV_TRY(ctx, hipEventRecord(e1, s));
  std::vector<float> hist(batches);
  CV_TRY(ctx, hipMemcpyAsync(hist.data(), cv.loss_hist.as<float>() + (steps - batches),
                             4 * batches, hipMemcpyDeviceToHost, s));

  // coefficient table: per bin of rho, the pooled within-design-point slope
  // of Y on g(X) over the held-out design points (never negative)
  CV_TRY(ctx, cv.g_full.ensure(4 * n_hold));
  CV_TRY(ctx, launch_mlp_forward(cv.theta.as<float>(), cv.xn.as<float>() + n_fit * 10, n_hold,
                                 cv.g_full.as<float>(), 1.0f, 0.0f, s));
  std::vector<float> gh(n_hold), yall(n);
  CV_TRY(ctx, hipMemcpyAsync(gh.data(), cv.g_full.p, 4 * n_hold, hipMemcpyDeviceToHost, s));
  CV_TRY(ctx, hipMemcpyAsync(yall.data(), cv.y_train.p, 4 * n, hipMemcpyDeviceToHost, s));
  CV_TRY(ctx, hipStreamSynchronize(s));
  CV_TRY(ctx, hipEventElapsedTime(&cv.train_ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  double lsum = 0.0;
  for (float v : hist) lsum += v;
  cv.final_loss = (float)(lsum / (double)batches);

  float rlo = 1e30f, rhi = -1e30f;
  for (uint64_t i = 0; i < n; ++i) {
    const float r = items[i].lambda / items[i].mu;
    rlo = std::min(rlo, r);
    rhi = std::max(rhi, r);
  }
  cv.rho_lo = rlo;
  cv.rho_hi = rhi > rlo ? rhi : rlo + 1e-6f;
  std::vector<double> sxy(MRIP_CV_BETA_BINS, 0.0), sxx(MRIP_CV_BETA_BINS, 0.0);
  for (size_t g = g_fit; g < G; ++g) {
    const uint64_t a = tb.group_offsets[g], b = tb.group_offsets[g + 1];
    double my = 0.0, mg = 0.0;
    for (uint64_t j = a; j < b; ++j) {
      my += yall[perm[j]];
      mg += gh[j - n_fit];
    }
    my /= (double)(b - a);
    mg /= (double)(b - a);
    const mrip_plan_item &it = items[perm[a]];
    const int bin = cv.bin_of(it.lambda / it.mu);
    for (uint64_t j = a; j < b; ++j) {
      const double dg = gh[j - n_fit] - mg;
      sxy[bin] += (yall[perm[j]] - my) * dg;
      sxx[bin] += dg * dg;
    }
  }
  cv.beta.assign(MRIP_CV_BETA_BINS, 0.0f);
  for (int k = 0; k < MRIP_CV_BETA_BINS; ++k) {
    // an empty bin borrows its nearest non-empty neighbour's coefficient
    int src = -1;
    for (int d = 0; d < MRIP_CV_BETA_BINS && src < 0; ++d) {
      if (k - d >= 0 && sxx[k - d] > 0.0) src = k - d;
      else if (k + d < MRIP_CV_BETA_BINS && sxx[k + d] > 0.0) src = k + d;
    }
    cv.beta[k] = src < 0 ? 0.0f : (float)std::max(0.0, sxy[src] / sxx[src]);
  }
  cv.trained = true;
  cv.applied = false;
  return MRIP_OK;
}

mrip_status mrip_cv_model(mrip_ctx ctx, float *theta, float *feat_mean, float *feat_std,
                          float *beta_table, float *rho_range, float *final_loss) {
  if (!ctx) return MRIP_E_INVAL;
  if (!ctx->cv.trained) return (ctx->err = "no trained control variate"), MRIP_E_STATE;
  if (theta) CV_TRY(ctx, hipMemcpy(theta, ctx->cv.theta.p, 4 * MLP_NPARAMS, hipMemcpyDeviceToHost));
  for (int j = 0; j < 10; ++j) {
    if (feat_mean) feat_mean[j] = ctx->cv.mean[j];
    if (feat_std) feat_std[j] = ctx->cv.std_[j];
  }
  if (beta_table)
    for (int k = 0; k < MRIP_CV_BETA_BINS; ++k) beta_table[k] = ctx->cv.beta[k];
  if (rho_range) {
    rho_range[0] = ctx->cv.rho_lo;
    rho_range[1] = ctx->cv.rho_hi;
  }
  if (final_loss) *final_loss = ctx->cv.final_loss;
  return MRIP_OK;
}

mrip_status mrip_cv_set_model(mrip_ctx ctx, const float *theta, const float *feat_mean,
                              const float *feat_std, const float *beta_table, float rho_lo,
                              float rho_hi) {
  if (!ctx) return MRIP_E_INVAL;
  if (ctx->model != MRIP_MM1) return (ctx->err = "the control variate needs an M/M/1 context"), MRIP_E_UNSUPPORTED;
  if (ctx->mm1.feature_prefix == 0) return bad(ctx, "the context needs feature_prefix > 0");
  if (!theta || !feat_mean || !feat_std || !beta_table) return bad(ctx, "NULL model array");
  if (!(rho_hi > rho_lo) || !std::isfinite(rho_lo) || !std::isfinite(rho_hi))
    return bad(ctx, "bad factor-level range");
  for (int j = 0; j < 10; ++j)
    if (!(feat_std[j] > 0.0f)) return bad(ctx, "feature std must be > 0");
  for (int k = 0; k < MRIP_CV_BETA_BINS; ++k)
    if (!(beta_table[k] >= 0.0f) || !std::isfinite(beta_table[k]))
      return bad(ctx, "coefficients must be finite and >= 0");
  CvState &cv = ctx->cv;
  float host_norm[20];
  cv.mean.assign(feat_mean, feat_mean + 10);
  cv.std_.assign(feat_std, feat_std + 10);
  for (int j = 0; j < 10; ++j) {
    host_norm[j] = feat_mean[j];
    host_norm[10 + j] = 1.0f / feat_std[j];
  }
  CV_TRY(ctx, cv.theta.ensure(4 * MLP_NPARAMS));
  CV_TRY(ctx, hipMemcpy(cv.theta.p, theta, 4 * MLP_NPARAMS, hipMemcpyHostToDevice));
  CV_TRY(ctx, cv.norm.ensure(sizeof(host_norm)));
  CV_TRY(ctx, hipMemcpy(cv.norm.p, host_norm, sizeof(host_norm), hipMemcpyHostToDevice));
  cv.beta.assign(beta_table, beta_table + MRIP_CV_BETA_BINS);
  cv.rho_lo = rho_lo;
  cv.rho_hi = rho_hi;
  cv.final_loss = 0.0f;
  cv.trained = true;
  cv.applied = false;
  return MRIP_OK;
}

mrip_status mrip_cv_outputs(mrip_ctx ctx, uint32_t which, void *dst, uint64_t bytes) {
  if (!ctx || !dst) return MRIP_E_INVAL;
  CvState &cv = ctx->cv;
  if (!cv.applied) return (ctx->err = "no control-variate apply yet"), MRIP_E_STATE;
  const DevBuf *src = nullptr;
  uint64_t need = 0;
  switch (which) {
    case 0: src = &cv.y_full; need = 4 * cv.full_items.count; break;
    case 1: src = &cv.g_full; need = 4 * cv.full_items.count; break;
    case 2: src = &cv.g_pre; need = 4 * cv.pre_items.count; break;
    case 3: src = &cv.x_full; need = 40 * cv.full_items.count; break;
    case 4: src = &cv.x_pre; need = 40 * cv.pre_items.count; break;
    default: return bad(ctx, "no such control-variate output");
  }
  if (bytes < need) return bad(ctx, "destination too small");
  CV_TRY(ctx, hipMemcpy(dst, src->p, need, hipMemcpyDeviceToHost));
  return MRIP_OK;
}

mrip_status mrip_cv_apply(mrip_ctx ctx, const mrip_plan_item *full, uint64_t n_full,
                          const mrip_plan_item *prefix, uint64_t n_prefix, uint64_t seed,
                          void *hip_stream) {
  if (!ctx) return MRIP_E_INVAL;
  if (ctx->rng != MRIP_RNG_PHILOX)
    return (ctx->err = "the control variate uses Philox streams"), MRIP_E_UNSUPPORTED;
  CvState &cv = ctx->cv;
  if (!cv.trained) return (ctx->err = "train the control variate first"), MRIP_E_STATE;
  const uint64_t K = ctx->mm1.feature_prefix;
  hipStream_t s = (hipStream_t)hip_stream;
  cv.applied = false;
  mrip_status st = upload_items(ctx, full, n_full, K, cv.full_items);
  if (st != MRIP_OK) return st;
  st = upload_items(ctx, prefix, n_prefix, K, cv.pre_items);
  if (st != MRIP_OK) return st;
  if (cv.full_items.dp_ids != cv.pre_items.dp_ids)
    return bad(ctx, "full and prefix items must cover the same design points");
  const size_t G = cv.full_items.dp_ids.size();
  for (size_t g = 0; g < G; ++g) {
    if (cv.full_items.group_offsets[g + 1] - cv.full_items.group_offsets[g] < 2 ||
        cv.pre_items.group_offsets[g + 1] - cv.pre_items.group_offsets[g] < 2)
      return bad(ctx, "every design point needs two full and two prefix replications");
  }
  CV_TRY(ctx, cv.y_full.ensure(4 * n_full));
  CV_TRY(ctx, cv.x_full.ensure(40 * n_full));
  CV_TRY(ctx, cv.g_full.ensure(4 * n_full));
  CV_TRY(ctx, cv.d_full.ensure(4 * n_full));
  CV_TRY(ctx, cv.x_pre.ensure(40 * n_prefix));
  CV_TRY(ctx, cv.y_pre.ensure(4 * n_prefix));
  CV_TRY(ctx, cv.g_pre.ensure(4 * n_prefix));
  CV_TRY(ctx, cv.xn.ensure(40 * std::max(n_full, n_prefix)));
  CV_TRY(ctx, cv.red_d.ensure(sizeof(double) * 3 * G));
  CV_TRY(ctx, cv.red_g.ensure(sizeof(double) * 3 * G));
  CV_TRY(ctx, cv.red_y.ensure(sizeof(double) * 3 * G));
  CV_TRY(ctx, cv.red_f.ensure(sizeof(double) * 3 * G));

  st = run_items(ctx, cv.full_items, seed, K, cv.y_full.as<float>(), cv.x_full.as<float>(), s,
                 &cv.full_ms);
  if (st != MRIP_OK) return st;
  st = run_items(ctx, cv.pre_items, seed, K, cv.y_pre.as<float>(), cv.x_pre.as<float>(), s,
                 &cv.prefix_ms);
  if (st != MRIP_OK) return st;

  // inference on both sets: g = net((x - mean) / std)
  hipEvent_t e0, e1;
  CV_TRY(ctx, hipEventCreate(&e0));
  CV_TRY(ctx, hipEventCreate(&e1));
  const float *mean_d = cv.norm.as<float>(), *inv_d = cv.norm.as<float>() + 10;
  CV_TRY(ctx, hipEventRecord(e0, s));
  CV_TRY(ctx, launch_normalize(cv.x_full.as<float>(), n_full, 10, mean_d, inv_d, cv.xn.as<float>(), s));
  CV_TRY(ctx, launch_mlp_forward(cv.theta.as<float>(), cv.xn.as<float>(), n_full,
                                 cv.g_full.as<float>(), 1.0f, 0.0f, s));
  CV_TRY(ctx, launch_normalize(cv.x_pre.as<float>(), n_prefix, 10, mean_d, inv_d, cv.xn.as<float>(), s));
  CV_TRY(ctx, launch_mlp_forward(cv.theta.as<float>(), cv.xn.as<float>(), n_prefix,
                                 cv.g_pre.as<float>(), 1.0f, 0.0f, s));
  CV_TRY(ctx, hipEventRecord(e1, s));

  // per design point: Y, g(X) and Y - g(X) over the full reps, g(X') over the
  // prefix reps; cov(Y, g) follows from the three variances
  CV_TRY(ctx, launch_axpy(cv.y_full.as<float>(), cv.g_full.as<float>(), 1.0f, n_full,
                          cv.d_full.as<float>(), s));
  const uint32_t *fidx = cv.full_items.index.as<uint32_t>();
  const uint64_t *foff = cv.full_items.offsets.as<uint64_t>();
  CV_TRY(ctx, launch_reduce_f64_gather(cv.y_full.p, 1, fidx, foff, (uint32_t)G, cv.red_y.as<double>(), s));
  CV_TRY(ctx, launch_reduce_f64_gather(cv.g_full.p, 1, fidx, foff, (uint32_t)G, cv.red_f.as<double>(), s));
  CV_TRY(ctx, launch_reduce_f64_gather(cv.d_full.p, 1, fidx, foff, (uint32_t)G, cv.red_d.as<double>(), s));
  CV_TRY(ctx, launch_reduce_f64_gather(cv.g_pre.p, 1, cv.pre_items.index.as<uint32_t>(),
                                       cv.pre_items.offsets.as<uint64_t>(), (uint32_t)G,
                                       cv.red_g.as<double>(), s));
  std::vector<double> ry(3 * G), rf(3 * G), rd(3 * G), rg(3 * G);
  CV_TRY(ctx, hipMemcpyAsync(ry.data(), cv.red_y.p, 24 * G, hipMemcpyDeviceToHost, s));
  CV_TRY(ctx, hipMemcpyAsync(rf.data(), cv.red_f.p, 24 * G, hipMemcpyDeviceToHost, s));
  CV_TRY(ctx, hipMemcpyAsync(rd.data(), cv.red_d.p, 24 * G, hipMemcpyDeviceToHost, s));
  CV_TRY(ctx, hipMemcpyAsync(rg.data(), cv.red_g.p, 24 * G, hipMemcpyDeviceToHost, s));
  CV_TRY(ctx, hipStreamSynchronize(s));
  CV_TRY(ctx, hipEventElapsedTime(&cv.infer_ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);

  cv.dp_ids = cv.full_items.dp_ids;
  cv.cv.assign(5 * G, 0.0);
  cv.plain.assign(3 * G, 0.0);
  for (size_t g = 0; g < G; ++g) {
    const double n = ry[3 * g], M = rg[3 * g];
    const uint64_t first = cv.full_items.group_offsets[g];
    const mrip_plan_item &it = full[cv.full_items.index_host[first]];
    const double beta = (double)cv.beta[cv.bin_of(it.lambda / it.mu)] * M / (M + n);
    const double vy = ry[3 * g + 2], vg = rf[3 * g + 2], vd = rd[3 * g + 2];
    const double cov = 0.5 * (vy + vg - vd);
    const double vres = std::max(0.0, vy - 2.0 * beta * cov + beta * beta * vg);
    const double a = vres / n, b = beta * beta * rg[3 * g + 2] / M;
    const double var = a + b;
    const double den = a * a / (n - 1.0) + b * b / (M - 1.0);
    cv.cv[5 * g + 0] = n;
    cv.cv[5 * g + 1] = ry[3 * g + 1] - beta * (rf[3 * g + 1] - rg[3 * g + 1]);
    cv.cv[5 * g + 2] = var;
    cv.cv[5 * g + 3] = den > 0.0 ? var * var / den : n - 1.0;
    cv.cv[5 * g + 4] = beta;
    cv.plain[3 * g + 0] = n;
    cv.plain[3 * g + 1] = ry[3 * g + 1];
    cv.plain[3 * g + 2] = vy;
  }
  cv.applied = true;
  return MRIP_OK;
}

mrip_status mrip_cv_stats(mrip_ctx ctx, uint32_t dp, double confidence, mrip_stats_t *cvs,
                          mrip_stats_t *plain) {
  if (!ctx) return MRIP_E_INVAL;
  if (!(confidence > 0.0 && confidence < 1.0)) return bad(ctx, "confidence must be in (0, 1)");
  CvState &cv = ctx->cv;
  if (!cv.applied) return (ctx->err = "no control-variate apply yet"), MRIP_E_STATE;
  auto it = std::lower_bound(cv.dp_ids.begin(), cv.dp_ids.end(), dp);
  if (it == cv.dp_ids.end() || *it != dp) return bad(ctx, "no such design point");
  const size_t g = (size_t)(it - cv.dp_ids.begin());
  const double p = 0.5 + 0.5 * confidence;
  if (cvs) {
    const double n = cv.cv[5 * g], var = cv.cv[5 * g + 2], dof = cv.cv[5 * g + 3];
    cvs->n = (uint64_t)n;
    cvs->mean = cv.cv[5 * g + 1];
    cvs->var = var * n;  // so that half_width = t * sqrt(var / n)
    cvs->confidence = confidence;
    cvs->t_quantile = mrip::t_quantile(p, dof);
    cvs->half_width = cvs->t_quantile * std::sqrt(var);
  }
  if (plain) {
    const double n = cv.plain[3 * g];
    plain->n = (uint64_t)n;
    plain->mean = cv.plain[3 * g + 1];
    plain->var = cv.plain[3 * g + 2];
    plain->confidence = confidence;
    plain->t_quantile = mrip::t_quantile(p, n - 1.0);
    plain->half_width = plain->t_quantile * std::sqrt(plain->var / n);
  }
  return MRIP_OK;
}

mrip_status mrip_cv_times(mrip_ctx ctx, float *full_ms, float *prefix_ms, float *infer_ms) {
  if (!ctx) return MRIP_E_INVAL;
  if (!ctx->cv.applied) return (ctx->err = "no control-variate apply yet"), MRIP_E_STATE;
  if (full_ms) *full_ms = ctx->cv.full_ms;
  if (prefix_ms) *prefix_ms = ctx->cv.prefix_ms;
  if (infer_ms) *infer_ms = ctx->cv.infer_ms;
  return MRIP_OK;
}

}  // extern "C"
