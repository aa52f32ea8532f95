// Student-t quantile for the replication confidence interval (the paper's
// section 1 interval from at least 30 replications; for fewer, the t law is
// the exact small-sample form of the same interval).
//
// Upper tail: P(T > t) = I_x(nu/2, 1/2) / 2 with x = nu / (nu + t^2), where
// I is the regularised incomplete beta function, evaluated by its continued
// fraction (modified Lentz). The quantile is a safeguarded Newton iteration
// on that tail inside a bisection bracket.
#include <cmath>

namespace mrip {

namespace {

// Continued fraction for I_x(a, b), valid for x < (a + 1) / (a + b + 2).
double beta_cf(double a, double b, double x) {
  const double tiny = 1e-300, eps = 1e-16;
  double c = 1.0, d = 1.0 - (a + b) * x / (a + 1.0);
  if (std::fabs(d) < tiny) d = tiny;
  d = 1.0 / d;
  double h = d;
  for (int m = 1; m <= 10000; ++m) {
    const double m2 = 2.0 * m;
    double num = m * (b - m) * x / ((a + m2 - 1.0) * (a + m2));
    d = 1.0 + num * d;
    if (std::fabs(d) < tiny) d = tiny;
    c = 1.0 + num / c;
    if (std::fabs(c) < tiny) c = tiny;
    d = 1.0 / d;
    h *= d * c;
    num = -(a + m) * (a + b + m) * x / ((a + m2) * (a + m2 + 1.0));
    d = 1.0 + num * d;
    if (std::fabs(d) < tiny) d = tiny;
    c = 1.0 + num / c;
    if (std::fabs(c) < tiny) c = tiny;
    d = 1.0 / d;
    const double del = d * c;
    h *= del;
    if (std::fabs(del - 1.0) < eps) break;
  }
  return h;
}

double inc_beta(double a, double b, double x) {
  if (x <= 0.0) return 0.0;
  if (x >= 1.0) return 1.0;
  const double lbeta = std::lgamma(a + b) - std::lgamma(a) - std::lgamma(b);
  const double front = std::exp(lbeta + a * std::log(x) + b * std::log1p(-x));
  if (x < (a + 1.0) / (a + b + 2.0)) return front * beta_cf(a, b, x) / a;
  return 1.0 - front * beta_cf(b, a, 1.0 - x) / b;
}

double t_upper_tail(double t, double nu) {  // t >= 0
  return 0.5 * inc_beta(0.5 * nu, 0.5, nu / (nu + t * t));
}

double t_pdf(double t, double nu) {
  const double lc = std::lgamma(0.5 * (nu + 1.0)) - std::lgamma(0.5 * nu) -
                    0.5 * std::log(nu * M_PI);
  return std::exp(lc - 0.5 * (nu + 1.0) * std::log1p(t * t / nu));
}

}  // namespace

double t_quantile(double p, double nu) {
  if (!(p >= 0.5 && p < 1.0) || !(nu > 0.0)) return std::nan("");
  if (p == 0.5) return 0.0;
  const double target = 1.0 - p;  // upper-tail probability
  double lo = 0.0, hi = 1.0;
  while (t_upper_tail(hi, nu) > target) {
    lo = hi;
    hi *= 2.0;
    if (hi > 1e300) return INFINITY;
  }
  double t = 0.5 * (lo + hi);
  for (int it = 0; it < 200; ++it) {
    const double f = t_upper_tail(t, nu) - target;  // decreasing in t
    if (f > 0) lo = t;
    else hi = t;
    double next = t + f / t_pdf(t, nu);  // Newton step on the tail
    if (!(next > lo && next < hi)) next = 0.5 * (lo + hi);
    if (std::fabs(next - t) <= 1e-15 * std::fabs(t) || hi - lo <= 1e-15 * hi) {
      t = next;
      break;
    }
    t = next;
  }
  return t;
}

}  // namespace mrip
