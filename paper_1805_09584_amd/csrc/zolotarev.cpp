// Zolotarev's optimal rational approximation of 1/sqrt(y) and the application
// x ~ (Q^2)^{-1/2} b through the multi-shift solve (section "Rational
// approximation": eq:rational, eq:deviation, eq:zolotarev_shifts, eq:ratapp).
//
// The Jacobi elliptic functions come from the arithmetic-geometric mean with
// descending Landen transformations (the method of Abramowitz and Stegun,
// section 16.4), the complete elliptic integral from K(m) = pi / (2 AGM(1, sqrt(1-m))).
// The maximal deviation is delta = d^2 / (1 + sqrt(1 - d^2))^2, the value the
// approximation attains (the printed formula lacks the square of the denominator).
#include <cmath>
#include <vector>

#include "ctx.h"

namespace ndtm {
namespace {

constexpr int kAgmMax = 64;

// K(m), parameter m = k^2 < 1
double ellip_k(double m) {
  double a = 1.0, b = std::sqrt(1.0 - m);
  for (int i = 0; i < kAgmMax && std::fabs(a - b) > 1e-16 * a; ++i) {
    const double an = 0.5 * (a + b);
    b = std::sqrt(a * b);
    a = an;
  }
  return M_PI / (2.0 * a);
}

// sn, cn of (u | m), 0 <= m < 1, by the AGM scale and backward recurrence of the amplitude
void ellip_sn_cn(double u, double m, double* sn, double* cn) {
  double a[kAgmMax + 1], c[kAgmMax + 1];
  a[0] = 1.0;
  double b = std::sqrt(1.0 - m);
  c[0] = std::sqrt(m);
  int nn = 0;
  while (nn < kAgmMax && std::fabs(c[nn]) > 1e-16 * a[nn]) {
    a[nn + 1] = 0.5 * (a[nn] + b);
    c[nn + 1] = 0.5 * (a[nn] - b);
    b = std::sqrt(a[nn] * b);
    ++nn;
  }
  double phi = std::ldexp(a[nn] * u, nn);
  for (int i = nn; i > 0; --i) phi = 0.5 * (phi + std::asin(c[i] / a[i] * std::sin(phi)));
  *sn = std::sin(phi);
  *cn = std::cos(phi);
}

}  // namespace

// c[0..2n-1] = c_1..c_2n, *a, *delta of order n on [eps, 1]
int zolotarev_coefficients(int n, double eps, double* c, double* a, double* delta) {
  if (n < 0 || n > NDTM_MAX_SHIFTS || !(eps > 0.0 && eps < 1.0) || (n > 0 && !c) || !a || !delta)
    return NDTM_EINVAL;
  const double m = 1.0 - eps;
  const double v = ellip_k(m) / (2 * n + 1);
  std::vector<double> s(2 * n);
  for (int k = 1; k <= 2 * n; ++k) {
    double sn, cn;
    ellip_sn_cn(k * v, m, &sn, &cn);
    s[k - 1] = sn * sn;
    c[k - 1] = (cn / sn) * (cn / sn);
  }
  double d = std::pow(1.0 - eps, 0.5 * (2 * n + 1));
  double ratio = 1.0;
  for (int j = 0; j < n; ++j) {
    d *= s[2 * j] * s[2 * j];
    ratio *= s[2 * j] / s[2 * j + 1];
  }
  const double root = 1.0 + std::sqrt(1.0 - d * d);
  *a = 2.0 / root * ratio;
  *delta = d * d / (root * root);
  return NDTM_OK;
}

}  // namespace ndtm

using namespace ndtm;

extern "C" {

int ndtm_zolotarev(int n, double eps, double* c, double* a, double* delta) {
  return zolotarev_coefficients(n, eps, c, a, delta);
}

int ndtm_solve_rational(ndtm_ctx* c, void* y_dev, const void* b_dev, int n, double eps, double lambda,
                        const ndtm_solve_params* p, ndtm_solve_report* rep, void* stream) {
  if (!c) return NDTM_EINVAL;
  if (!y_dev || !b_dev || !p || !rep || y_dev == b_dev) return fail(c, NDTM_EINVAL, "solve_rational: bad pointers");
  if (n < 1 || n > NDTM_MAX_SHIFTS || !(eps > 0.0 && eps < 1.0) || !(lambda > 0.0) || !std::isfinite(lambda))
    return fail(c, NDTM_EINVAL, "solve_rational: 1 <= n <= 16, 0 < eps < 1, lambda > 0");
  std::vector<double> cc(2 * n);
  double a = 0, delta = 0;
  if (zolotarev_coefficients(n, eps, cc.data(), &a, &delta) != NDTM_OK)
    return fail(c, NDTM_EINVAL, "solve_rational: coefficients");
  // shifts m_i^2 = c_{2i} and weights q_i of eq:ratapp, scaled to the spectrum [eps lambda, lambda]
  std::vector<double> sig(n), q(n);
  for (int i = 0; i < n; ++i) {
    sig[i] = lambda * cc[2 * i + 1];
    q[i] = cc[2 * i] - cc[2 * i + 1];
    for (int j = 0; j < n; ++j)
      if (j != i) q[i] *= (cc[2 * j] - cc[2 * i + 1]) / (cc[2 * j + 1] - cc[2 * i + 1]);
  }
  int rc = ndtm_set_shifts(c, n, sig.data());
  if (rc != NDTM_OK) return rc;
  NDTM_HIP(c, hipSetDevice(c->device));
  hipStream_t st = static_cast<hipStream_t>(stream);
  const size_t elems = (size_t)c->g.vh * 24;  // canonical odd-site doublet
  std::vector<void*> xs(n);
  for (int i = 0; i < n; ++i) {
    xs[i] = ws_get(c, "rat_x" + std::to_string(i), elems * sizeof(double2));
    if (!xs[i]) return fail(c, NDTM_ENOMEM, "solve_rational: workspace");
  }
  rc = ndtm_solve(c, xs.data(), b_dev, p, rep, stream);
  if (rc != NDTM_OK && rc != NDTM_ENOCONV) return rc;
  // y = lambda^{-1/2} a (b + sum_i q_i lambda x_i)
  std::vector<const double2*> V(n + 1);
  std::vector<double2> w(n + 1);
  const double s = a / std::sqrt(lambda);
  V[0] = static_cast<const double2*>(b_dev);
  w[0] = make_double2(s, 0.0);
  for (int i = 0; i < n; ++i) {
    V[1 + i] = static_cast<const double2*>(xs[i]);
    w[1 + i] = make_double2(s * lambda * q[i], 0.0);
  }
  blas_lincomb(static_cast<double2*>(y_dev), V.data(), w.data(), n + 1, elems, st);
  NDTM_HIP(c, hipStreamSynchronize(st));
  return rc;
}

}  // extern "C"
