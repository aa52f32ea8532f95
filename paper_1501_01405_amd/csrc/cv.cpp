// Learned control variate (not in the paper; it extends MRIP's estimator):
// training-set generation with the M/M/1 engine, training of the bf16-MFMA
// network with Adam, and the control-variate estimate per design point,
// next to the plain MRIP estimate that stays its fallback.
//
// The controls of a replication are F = (h, z_pre): h = sum_k g_k(X) z_k
// with z the four martingale controls of its customers after the feature
// prefix (divided by the run length, the T-weighted two also by the service
// scale) and g the network's coefficients from the prefix features X, and
// z_pre the same four controls over the prefix. Every term of a control has
// mean zero given the past, so E[g_k(X) z_k] = 0 for any network, E[z_pre]
// = 0, and Y - a . F with a fixed per bin of rho is unbiased for E[Y] with
// no second sample.
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

// Upload items (SoA), their longest-first order (and how many of its first
// items are long) and their dp grouping.
mrip_status upload_items(mrip_ctx c, const mrip_plan_item *items, uint64_t n, uint64_t K,
                         uint64_t long_min, ItemBufs &b) {
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
  b.total_customers = 0;
  for (uint64_t i = 0; i < n; ++i) b.total_customers += cust[i];
  b.n_long = 0;  // items of at least long_min customers: a prefix of the order
  while (b.n_long < n && cust[order[b.n_long]] >= long_min) ++b.n_long;
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

// Run an item table through the persistent M/M/1 kernels (the plan's form:
// items of at least long_min customers split over plan_split_for wavefronts)
// with feature capture over the first K customers and the controls after
// them; `ms` (nullable) gets the kernel time.
mrip_status run_items(mrip_ctx c, ItemBufs &b, uint64_t seed, uint64_t K, float *mean_w,
                      float *feat, float *ctl, hipStream_t s, float *ms) {
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
  a.controls = ctl;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (ms) {
    CV_TRY(c, hipEventCreate(&e0));
    CV_TRY(c, hipEventCreate(&e1));
  }
  CV_TRY(c, launch_zero_u32(a.queue_head, 2, s));
  if (ms) CV_TRY(c, hipEventRecord(e0, s));
  const uint32_t split = plan_split_for(c, b.max_customers, b.total_customers);
  if (split > 1 && b.n_long > 0)
    CV_TRY(c, launch_mm1_plan_split(a, b.count, b.n_long, split, c->plan_rpw, s));
  else
    CV_TRY(c, launch_mm1_plan(a, b.count, c->plan_rpw, c->plan_wg, s));
  if (ms) {
    CV_TRY(c, hipEventRecord(e1, s));
    CV_TRY(c, hipEventSynchronize(e1));
    CV_TRY(c, hipEventElapsedTime(ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
  }
  return MRIP_OK;
}

// The four (0) and the four (1) the gather-normalise kernel takes as mean
// and inverse std of the multiplier columns, which it copies unchanged.
mrip_status unit_columns(mrip_ctx c) {
  const float u[8] = {0.f, 0.f, 0.f, 0.f, 1.f, 1.f, 1.f, 1.f};
  CV_TRY(c, c->cv.unit4.ensure(sizeof(u)));
  CV_TRY(c, hipMemcpy(c->cv.unit4.p, u, sizeof(u), hipMemcpyHostToDevice));
  return MRIP_OK;
}

// Solve A x = b (p x p, row-major) by Gaussian elimination with partial
// pivoting; false if a pivot vanishes.
bool solve_dense(std::vector<double> A, std::vector<double> b, int p, std::vector<double> &x) {
  for (int c = 0; c < p; ++c) {
    int piv = c;
    for (int r = c + 1; r < p; ++r)
      if (std::fabs(A[r * p + c]) > std::fabs(A[piv * p + c])) piv = r;
    if (A[piv * p + c] == 0.0) return false;
    if (piv != c) {
      for (int k = 0; k < p; ++k) std::swap(A[c * p + k], A[piv * p + k]);
      std::swap(b[c], b[piv]);
    }
    for (int r = c + 1; r < p; ++r) {
      const double f = A[r * p + c] / A[c * p + c];
      for (int k = c; k < p; ++k) A[r * p + k] -= f * A[c * p + k];
      b[r] -= f * b[c];
    }
  }
  x.assign(p, 0.0);
  for (int r = p - 1; r >= 0; --r) {
    double v = b[r];
    for (int k = r + 1; k < p; ++k) v -= A[r * p + k] * x[k];
    x[r] = v / A[r * p + r];
  }
  return true;
}

// The coefficient table on the device (MRIP_CV_BETA_BINS x MRIP_CV_COEFS).
mrip_status upload_coefs(mrip_ctx c) {
  CV_TRY(c, c->cv.coef_d.ensure(sizeof(float) * c->cv.coef.size()));
  CV_TRY(c, hipMemcpy(c->cv.coef_d.p, c->cv.coef.data(), sizeof(float) * c->cv.coef.size(),
                      hipMemcpyHostToDevice));
  return MRIP_OK;
}

std::mutex g_grad_mu;
DevBuf g_grad_partial;  // partial-gradient rows for the context-free mrip_mlp_grad
DevBuf g_grad_image;    // and its weights' image

bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

}  // namespace

extern "C" {

mrip_status mrip_mlp_forward(const float *theta_dev, const float *x_dev, uint64_t n, float *y_dev,
                             void *hip_stream) {
  if (n > 0 && (!theta_dev || !x_dev || !y_dev)) return MRIP_E_INVAL;
  if (n > 0 && (!aligned16(y_dev) || !aligned16(theta_dev))) return MRIP_E_INVAL;
  if (n >= (1ull << 30)) return MRIP_E_INVAL;  // 4 lanes per row: one launch < 2^32 lanes
  hipError_t e = launch_mlp_forward(theta_dev, x_dev, n, y_dev, (hipStream_t)hip_stream);
  return e == hipSuccess ? MRIP_OK : MRIP_E_HIP;
}

mrip_status mrip_mlp_grad(const float *theta_dev, const float *x_dev, const float *z_dev,
                          const float *y_dev, uint64_t n, float *grad_dev, float *loss_dev,
                          void *hip_stream) {
  if (n == 0 || n > 65536 || !theta_dev || !x_dev || !y_dev || !grad_dev) return MRIP_E_INVAL;
  if (!aligned16(theta_dev) || (z_dev && !aligned16(z_dev))) return MRIP_E_INVAL;
  std::lock_guard<std::mutex> lock(g_grad_mu);
  hipStream_t s = (hipStream_t)hip_stream;
  const size_t rows = mlp_partial_rows(n);
  if (g_grad_partial.ensure(rows * MLP_PSTRIDE * sizeof(float)) != hipSuccess ||
      g_grad_image.ensure(MLP_IMAGE_BYTES) != hipSuccess)
    return MRIP_E_NOMEM;
  if (launch_mlp_pack(theta_dev, g_grad_image.p, s) != hipSuccess) return MRIP_E_HIP;
  if (launch_mlp_grad(g_grad_image.p, x_dev, z_dev, y_dev, n, g_grad_partial.as<float>(), s) !=
      hipSuccess)
    return MRIP_E_HIP;
  AdamArgs none{};
  if (launch_grad_reduce(g_grad_partial.as<float>(), (uint32_t)rows, n, grad_dev, loss_dev, nullptr,
                         nullptr, nullptr, none, nullptr, s) != hipSuccess)
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
  cv.applied = false;

  mrip_status st = upload_items(ctx, items, n, K, ctx->long_min, cv.train_items);
  if (st != MRIP_OK) return st;
  ItemBufs &tb = cv.train_items;
  const size_t G = tb.dp_ids.size();
  if (G < 2) return bad(ctx, "training needs at least two design points");
  for (size_t g = 0; g < G; ++g)
    if (tb.group_offsets[g + 1] - tb.group_offsets[g] < 2)
      return bad(ctx, "every training design point needs two replications");
  st = unit_columns(ctx);
  if (st != MRIP_OK) return st;

  CV_TRY(ctx, cv.y_train.ensure(4 * n));
  CV_TRY(ctx, cv.x_train.ensure(40 * n));
  CV_TRY(ctx, cv.c_train.ensure(32 * n));
  CV_TRY(ctx, cv.z_train.ensure(32 * n));
  CV_TRY(ctx, cv.t_train.ensure(4 * n));
  CV_TRY(ctx, cv.zt_train.ensure(16 * n));
  CV_TRY(ctx, cv.g_rows.ensure(16 * n));
  CV_TRY(ctx, cv.g_train.ensure(16 * n));
  CV_TRY(ctx, cv.xn.ensure(40 * n));
  CV_TRY(ctx, cv.yn.ensure(4 * n));
  CV_TRY(ctx, cv.zn.ensure(16 * n));
  CV_TRY(ctx, cv.red_y.ensure(sizeof(double) * 3 * G));
  hipEvent_t e0, e1;
  CV_TRY(ctx, hipEventCreate(&e0));
  CV_TRY(ctx, hipEventCreate(&e1));
  CV_TRY(ctx, hipEventRecord(e0, s));
  st = run_items(ctx, tb, seed, K, cv.y_train.as<float>(), cv.x_train.as<float>(),
                 cv.c_train.as<float>(), s, nullptr);
  if (st != MRIP_OK) return st;

  // target: the replication's standardised deviation from its design
  // point's mean, so the network models the within-design-point variation a
  // control variate can use, at the same scale for every factor level; the
  // multipliers are scaled by the same standard deviation
  const std::vector<uint32_t> &index = tb.index_host;
  std::vector<uint32_t> group(n);
  for (size_t g = 0; g < G; ++g)
    for (uint64_t j = tb.group_offsets[g]; j < tb.group_offsets[g + 1]; ++j) group[index[j]] = (uint32_t)g;
  CV_TRY(ctx, cv.group.ensure(4 * n));
  CV_TRY(ctx, hipMemcpy(cv.group.p, group.data(), 4 * n, hipMemcpyHostToDevice));
  CV_TRY(ctx, launch_reduce_f64_gather(cv.y_train.p, 1, tb.index.as<uint32_t>(),
                                       tb.offsets.as<uint64_t>(), (uint32_t)G,
                                       cv.red_y.as<double>(), s));
  CV_TRY(ctx, launch_multipliers(cv.c_train.as<float>(), tb.n.as<uint64_t>(), tb.mu.as<float>(), n,
                                 cv.z_train.as<float>(), cv.y_train.as<float>(),
                                 cv.group.as<uint32_t>(), cv.red_y.as<double>(),
                                 cv.t_train.as<float>(), cv.zt_train.as<float>(), s));

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
  cv.perm.clear();
  cv.perm.reserve(n);
  for (size_t g = 0; g < G; ++g)
    for (uint64_t j = tb.group_offsets[g]; j < tb.group_offsets[g + 1]; ++j) cv.perm.push_back(index[j]);
  const uint64_t n_fit = tb.group_offsets[g_fit];
  const uint64_t n_hold = n - n_fit;
  cv.n_fit = n_fit;
  DevBuf perm_d;
  CV_TRY(ctx, perm_d.ensure(4 * n));
  CV_TRY(ctx, hipMemcpy(perm_d.p, cv.perm.data(), 4 * n, hipMemcpyHostToDevice));
  const float *mean_d = cv.norm.as<float>(), *inv_d = cv.norm.as<float>() + 10;
  const float *zero4 = cv.unit4.as<float>(), *one4 = cv.unit4.as<float>() + 4;
  const uint32_t *pd = perm_d.as<uint32_t>();
  CV_TRY(ctx, launch_gather_normalize(cv.x_train.as<float>(), pd, n, 10, mean_d, inv_d,
                                      cv.xn.as<float>(), s));
  CV_TRY(ctx, launch_gather_normalize(cv.t_train.as<float>(), pd, n, 1, zero4, one4,
                                      cv.yn.as<float>(), s));
  CV_TRY(ctx, launch_gather_normalize(cv.zt_train.as<float>(), pd, n, 4, zero4, one4,
                                      cv.zn.as<float>(), s));

  // Adam from theta0
  CV_TRY(ctx, cv.theta.ensure(4 * MLP_NPARAMS));
  CV_TRY(ctx, cv.adam_m.ensure(4 * MLP_NPARAMS));
  CV_TRY(ctx, cv.adam_v.ensure(4 * MLP_NPARAMS));
  CV_TRY(ctx, hipMemcpy(cv.theta.p, theta0, 4 * MLP_NPARAMS, hipMemcpyHostToDevice));
  CV_TRY(ctx, hipMemsetAsync(cv.adam_m.p, 0, 4 * MLP_NPARAMS, s));
  CV_TRY(ctx, hipMemsetAsync(cv.adam_v.p, 0, 4 * MLP_NPARAMS, s));
  CV_TRY(ctx, cv.image.ensure(MLP_IMAGE_BYTES));
  CV_TRY(ctx, launch_mlp_pack(cv.theta.as<float>(), cv.image.p, s));
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
      CV_TRY(ctx, launch_mlp_grad(cv.image.p, cv.xn.as<float>() + r0 * 10,
                                  cv.zn.as<float>() + r0 * 4, cv.yn.as<float>() + r0, nb,
                                  cv.partial.as<float>(), s));
      CV_TRY(ctx, launch_grad_reduce(cv.partial.as<float>(), (uint32_t)mlp_partial_rows(nb), nb,
                                     nullptr, cv.loss_hist.as<float>() + (step - 1),
                                     cv.theta.as<float>(), cv.adam_m.as<float>(),
                                     cv.adam_v.as<float>(),
                                     adam_args(hp.lr, hp.beta1, hp.beta2, hp.eps, step),
                                     cv.image.p, s));
    }
  }
  CV_TRY(ctx, hipEventRecord(e1, s));
  std::vector<float> hist(batches);
  CV_TRY(ctx, hipMemcpyAsync(hist.data(), cv.loss_hist.as<float>() + (steps - batches),
                             4 * batches, hipMemcpyDeviceToHost, s));

  // the trained network on every row (training order); the held-out rows'
  // outputs fit the coefficient table
  CV_TRY(ctx, launch_mlp_forward(cv.theta.as<float>(), cv.xn.as<float>(), n, cv.g_rows.as<float>(), s));
  std::vector<float> grow(4 * n), zall(8 * n), yall(n);
  CV_TRY(ctx, hipMemcpyAsync(grow.data(), cv.g_rows.p, 16 * n, hipMemcpyDeviceToHost, s));
  CV_TRY(ctx, hipMemcpyAsync(zall.data(), cv.z_train.p, 32 * n, hipMemcpyDeviceToHost, s));
  CV_TRY(ctx, hipMemcpyAsync(yall.data(), cv.y_train.p, 4 * n, hipMemcpyDeviceToHost, s));
  CV_TRY(ctx, hipStreamSynchronize(s));
  CV_TRY(ctx, hipEventElapsedTime(&cv.train_ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  double lsum = 0.0;
  for (float v : hist) lsum += v;
  cv.final_loss = (float)(lsum / (double)batches);
  // network outputs in item order (an output of the library)
  std::vector<float> gitem(4 * n);
  for (uint64_t j = 0; j < n; ++j)
    for (int k = 0; k < 4; ++k) gitem[4 * (uint64_t)cv.perm[j] + k] = grow[4 * j + k];
  CV_TRY(ctx, hipMemcpy(cv.g_train.p, gitem.data(), 16 * n, hipMemcpyHostToDevice));

  float rlo = 1e30f, rhi = -1e30f;
  for (uint64_t i = 0; i < n; ++i) {
    const float r = items[i].lambda / items[i].mu;
    rlo = std::min(rlo, r);
    rhi = std::max(rhi, r);
  }
  cv.rho_lo = rlo;
  cv.rho_hi = rhi > rlo ? rhi : rlo + 1e-6f;
  // coefficient table: per bin of rho, the pooled within-design-point
  // least-squares coefficients of Y on F = (h, z_4..z_7) over the held-out
  // design points, h = sum_k g_k z_k the network's control
  constexpr int P = MRIP_CV_COEFS, NB = MRIP_CV_BETA_BINS;
  std::vector<double> A((size_t)NB * P * P, 0.0), bv((size_t)NB * P, 0.0);
  std::vector<bool> seen(NB, false);
  std::vector<double> F((size_t)n_hold * P);
  for (size_t g = g_fit; g < G; ++g) {
    const uint64_t a = tb.group_offsets[g], b = tb.group_offsets[g + 1];
    double my = 0.0, mf[P] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (uint64_t j = a; j < b; ++j) {
      const uint64_t i = cv.perm[j];
      double *f = &F[(j - n_fit) * P];
      double hv = 0.0;
      for (int k = 0; k < 4; ++k) hv += (double)grow[4 * j + k] * (double)zall[8 * i + k];
      f[0] = hv;
      for (int k = 0; k < 4; ++k) f[1 + k] = (double)zall[8 * i + 4 + k];
      my += yall[i];
      for (int k = 0; k < P; ++k) mf[k] += f[k];
    }
    my /= (double)(b - a);
    for (int k = 0; k < P; ++k) mf[k] /= (double)(b - a);
    const mrip_plan_item &it = items[cv.perm[a]];
    const int bin = cv.bin_of(it.lambda / it.mu);
    seen[bin] = true;
    for (uint64_t j = a; j < b; ++j) {
      const double *f = &F[(j - n_fit) * P];
      const double dy = yall[cv.perm[j]] - my;
      for (int r = 0; r < P; ++r) {
        const double fr = f[r] - mf[r];
        bv[(size_t)bin * P + r] += fr * dy;
        for (int c = 0; c < P; ++c) A[((size_t)bin * P + r) * P + c] += fr * (f[c] - mf[c]);
      }
    }
  }
  std::vector<double> coef((size_t)NB * P, 0.0);
  for (int k = 0; k < NB; ++k) {
    if (!seen[k]) continue;
    // columns without within-design-point variation get 0 and leave the system
    std::vector<int> live;
    for (int c = 0; c < P; ++c)
      if (A[((size_t)k * P + c) * P + c] > 0.0) live.push_back(c);
    const int q = (int)live.size();
    if (q == 0) continue;
    std::vector<double> Al((size_t)q * q), bl(q), x;
    for (int r = 0; r < q; ++r) {
      bl[r] = bv[(size_t)k * P + live[r]];
      for (int c = 0; c < q; ++c) Al[(size_t)r * q + c] = A[((size_t)k * P + live[r]) * P + live[c]];
    }
    if (!solve_dense(Al, bl, q, x)) continue;
    for (int r = 0; r < q; ++r) coef[(size_t)k * P + live[r]] = x[r];
  }
  cv.coef.assign((size_t)NB * P, 0.0f);
  for (int k = 0; k < NB; ++k) {
    // a bin without design points borrows its nearest neighbour's row
    int src = -1;
    for (int d = 0; d < NB && src < 0; ++d) {
      if (k - d >= 0 && seen[k - d]) src = k - d;
      else if (k + d < NB && seen[k + d]) src = k + d;
    }
    if (src >= 0)
      for (int c = 0; c < P; ++c) cv.coef[(size_t)k * P + c] = (float)coef[(size_t)src * P + c];
  }
  st = upload_coefs(ctx);
  if (st != MRIP_OK) return st;
  cv.trained = true;
  return MRIP_OK;
}

mrip_status mrip_cv_model(mrip_ctx ctx, float *theta, float *feat_mean, float *feat_std,
                          float *coef_table, float *rho_range, float *final_loss) {
  if (!ctx) return MRIP_E_INVAL;
  if (!ctx->cv.trained) return (ctx->err = "no trained control variate"), MRIP_E_STATE;
  if (theta) CV_TRY(ctx, hipMemcpy(theta, ctx->cv.theta.p, 4 * MLP_NPARAMS, hipMemcpyDeviceToHost));
  for (int j = 0; j < 10; ++j) {
    if (feat_mean) feat_mean[j] = ctx->cv.mean[j];
    if (feat_std) feat_std[j] = ctx->cv.std_[j];
  }
  if (coef_table)
    for (size_t k = 0; k < ctx->cv.coef.size(); ++k) coef_table[k] = ctx->cv.coef[k];
  if (rho_range) {
    rho_range[0] = ctx->cv.rho_lo;
    rho_range[1] = ctx->cv.rho_hi;
  }
  if (final_loss) *final_loss = ctx->cv.final_loss;
  return MRIP_OK;
}

mrip_status mrip_cv_set_model(mrip_ctx ctx, const float *theta, const float *feat_mean,
                              const float *feat_std, const float *coef_table, float rho_lo,
                              float rho_hi) {
  if (!ctx) return MRIP_E_INVAL;
  if (ctx->model != MRIP_MM1) return (ctx->err = "the control variate needs an M/M/1 context"), MRIP_E_UNSUPPORTED;
  if (ctx->mm1.feature_prefix == 0) return bad(ctx, "the context needs feature_prefix > 0");
  if (!theta || !feat_mean || !feat_std || !coef_table) return bad(ctx, "NULL model array");
  if (!(rho_hi > rho_lo) || !std::isfinite(rho_lo) || !std::isfinite(rho_hi))
    return bad(ctx, "bad factor-level range");
  for (int j = 0; j < 10; ++j)
    if (!(feat_std[j] > 0.0f)) return bad(ctx, "feature std must be > 0");
  for (int k = 0; k < MRIP_CV_BETA_BINS * MRIP_CV_COEFS; ++k)
    if (!std::isfinite(coef_table[k])) return bad(ctx, "coefficients must be finite");
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
  cv.coef.assign(coef_table, coef_table + MRIP_CV_BETA_BINS * MRIP_CV_COEFS);
  mrip_status st = upload_coefs(ctx);
  if (st != MRIP_OK) return st;
  cv.rho_lo = rho_lo;
  cv.rho_hi = rho_hi;
  cv.final_loss = 0.0f;
  cv.trained = true;
  cv.applied = false;
  cv.train_items.count = 0;  // no training set behind an installed model
  return MRIP_OK;
}

mrip_status mrip_cv_outputs(mrip_ctx ctx, uint32_t which, void *dst, uint64_t bytes) {
  if (!ctx || !dst) return MRIP_E_INVAL;
  CvState &cv = ctx->cv;
  const DevBuf *src = nullptr;
  uint64_t need = 0;
  if (which <= 4) {
    if (!cv.applied) return (ctx->err = "no control-variate apply yet"), MRIP_E_STATE;
    const uint64_t n = cv.items.count;
    switch (which) {
      case 0: src = &cv.y; need = 4 * n; break;
      case 1: src = &cv.h; need = 4 * n; break;
      case 2: src = &cv.g; need = 16 * n; break;
      case 3: src = &cv.x; need = 40 * n; break;
      default: src = &cv.c; need = 32 * n; break;
    }
  } else if (which <= 8) {
    if (!cv.trained || cv.train_items.count == 0)
      return (ctx->err = "no training run behind the model"), MRIP_E_STATE;
    const uint64_t n = cv.train_items.count;
    switch (which) {
      case 5: src = &cv.y_train; need = 4 * n; break;
      case 6: src = &cv.x_train; need = 40 * n; break;
      case 7: src = &cv.c_train; need = 32 * n; break;
      default: src = &cv.g_train; need = 16 * n; break;
    }
  } else {
    return bad(ctx, "no such control-variate output");
  }
  if (bytes < need) return bad(ctx, "destination too small");
  CV_TRY(ctx, hipDeviceSynchronize());
  CV_TRY(ctx, hipMemcpy(dst, src->p, need, hipMemcpyDeviceToHost));
  return MRIP_OK;
}

mrip_status mrip_cv_apply(mrip_ctx ctx, const mrip_plan_item *items, uint64_t n, uint64_t seed,
                          void *hip_stream) {
  if (!ctx) return MRIP_E_INVAL;
  if (ctx->rng != MRIP_RNG_PHILOX)
    return (ctx->err = "the control variate uses Philox streams"), MRIP_E_UNSUPPORTED;
  CvState &cv = ctx->cv;
  if (!cv.trained) return (ctx->err = "train the control variate first"), MRIP_E_STATE;
  const uint64_t K = ctx->mm1.feature_prefix;
  hipStream_t s = (hipStream_t)hip_stream;
  cv.applied = false;
  mrip_status st = upload_items(ctx, items, n, K, ctx->long_min, cv.items);
  if (st != MRIP_OK) return st;
  const size_t G = cv.items.dp_ids.size();
  for (size_t g = 0; g < G; ++g)
    if (cv.items.group_offsets[g + 1] - cv.items.group_offsets[g] < 2)
      return bad(ctx, "every design point needs two replications");
  CV_TRY(ctx, cv.y.ensure(4 * n));
  CV_TRY(ctx, cv.x.ensure(40 * n));
  CV_TRY(ctx, cv.c.ensure(32 * n));
  CV_TRY(ctx, cv.g.ensure(16 * n));
  CV_TRY(ctx, cv.h.ensure(4 * n));
  CV_TRY(ctx, cv.d.ensure(4 * n));
  CV_TRY(ctx, cv.bin_item.ensure(4 * n));
  CV_TRY(ctx, cv.red_y.ensure(sizeof(double) * 3 * G));
  CV_TRY(ctx, cv.red_d.ensure(sizeof(double) * 3 * G));
  // each item's row of the coefficient table: its design point's bin of rho
  std::vector<uint32_t> bins(n);
  for (uint64_t i = 0; i < n; ++i) bins[i] = (uint32_t)cv.bin_of(items[i].lambda / items[i].mu);
  CV_TRY(ctx, hipMemcpy(cv.bin_item.p, bins.data(), 4 * n, hipMemcpyHostToDevice));

  st = run_items(ctx, cv.items, seed, K, cv.y.as<float>(), cv.x.as<float>(), cv.c.as<float>(), s,
                 &cv.run_ms);
  if (st != MRIP_OK) return st;

  // inference in one kernel: g = net((x - mean) / std), the multipliers, h
  // and the residual Y - coef . (h, z_pre); then per design point (n, mean,
  // var) of Y and of the residual in one reduction launch
  hipEvent_t e0, e1;
  CV_TRY(ctx, hipEventCreate(&e0));
  CV_TRY(ctx, hipEventCreate(&e1));
  CvInferArgs ia{};
  ia.mean = cv.norm.as<float>();
  ia.inv_std = cv.norm.as<float>() + 10;
  ia.ctl = cv.c.as<float>();
  ia.customers = cv.items.n.as<uint64_t>();
  ia.mu = cv.items.mu.as<float>();
  ia.bin = cv.bin_item.as<uint32_t>();
  ia.coef = cv.coef_d.as<float>();
  ia.y = cv.y.as<float>();
  ia.g = cv.g.as<float>();
  ia.h = cv.h.as<float>();
  ia.d = cv.d.as<float>();
  CV_TRY(ctx, hipEventRecord(e0, s));
  CV_TRY(ctx, launch_cv_infer(cv.theta.as<float>(), cv.x.as<float>(), n, ia, s));
  CV_TRY(ctx, launch_reduce_f64_gather2(cv.y.as<float>(), cv.d.as<float>(),
                                        cv.items.index.as<uint32_t>(),
                                        cv.items.offsets.as<uint64_t>(), (uint32_t)G,
                                        cv.red_y.as<double>(), cv.red_d.as<double>(), s));
  CV_TRY(ctx, hipEventRecord(e1, s));
  std::vector<double> ry(3 * G), rd(3 * G);
  CV_TRY(ctx, hipMemcpyAsync(ry.data(), cv.red_y.p, 24 * G, hipMemcpyDeviceToHost, s));
  CV_TRY(ctx, hipMemcpyAsync(rd.data(), cv.red_d.p, 24 * G, hipMemcpyDeviceToHost, s));
  CV_TRY(ctx, hipStreamSynchronize(s));
  CV_TRY(ctx, hipEventElapsedTime(&cv.infer_ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);

  cv.dp_ids = cv.items.dp_ids;
  cv.cv.assign(5 * G, 0.0);
  cv.plain.assign(3 * G, 0.0);
  for (size_t g = 0; g < G; ++g) {
    const double nn = ry[3 * g];
    const uint64_t first = cv.items.group_offsets[g];
    const mrip_plan_item &it = items[cv.items.index_host[first]];
    cv.cv[5 * g + 0] = nn;
    cv.cv[5 * g + 1] = rd[3 * g + 1];
    cv.cv[5 * g + 2] = rd[3 * g + 2] / nn;
    cv.cv[5 * g + 3] = nn - 1.0;
    cv.cv[5 * g + 4] = cv.coef[(size_t)cv.bin_of(it.lambda / it.mu) * MRIP_CV_COEFS];
    cv.plain[3 * g + 0] = nn;
    cv.plain[3 * g + 1] = ry[3 * g + 1];
    cv.plain[3 * g + 2] = ry[3 * g + 2];
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

mrip_status mrip_cv_times(mrip_ctx ctx, float *run_ms, float *infer_ms) {
  if (!ctx) return MRIP_E_INVAL;
  if (!ctx->cv.applied) return (ctx->err = "no control-variate apply yet"), MRIP_E_STATE;
  if (run_ms) *run_ms = ctx->cv.run_ms;
  if (infer_ms) *infer_ms = ctx->cv.infer_ms;
  return MRIP_OK;
}

}  // extern "C"
