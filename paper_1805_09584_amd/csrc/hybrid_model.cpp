// The hybrid split of section 4.4: the number n of (largest) shifts solved by
// multi-shift CG, chosen by the cost model eq:costwo,
//   c_HY(n) = t_CG(m_n^2) + sum_{i > n} t_MG(m_i^2),
// where the multi-shift solve costs what CG costs at its smallest shift m_n^2.
// t_CG(sigma) is the CG iteration bound for the spectrum [lmin + sigma, lmax + sigma],
//   k(sigma) = 0.5 sqrt(kappa) ln(2 / tol),  kappa = (lmax + sigma) / (lmin + sigma),
// times the measured cost of one multi-shift iteration; t_MG is the measured
// cost of one multigrid shift.  The spectrum comes from the Lanczos tridiagonal
// matrix that the base system's CG coefficients define (the multi-shift solve
// records them), its extreme eigenvalues found by Sturm-sequence bisection.
#include <algorithm>
#include <cmath>
#include <vector>

#include "ctx.h"

namespace ndtm {

namespace {

// number of eigenvalues of the symmetric tridiagonal (d, e) below x
int sturm_count(const std::vector<double>& d, const std::vector<double>& e, double x) {
  int cnt = 0;
  double q = 1.0;
  for (size_t i = 0; i < d.size(); ++i) {
    const double off = i ? e[i - 1] * e[i - 1] : 0.0;
    q = d[i] - x - (i ? off / q : 0.0);
    if (q == 0.0) q = 1e-300;
    if (q < 0) ++cnt;
  }
  return cnt;
}

double tridiag_eig(const std::vector<double>& d, const std::vector<double>& e, int which, double lo, double hi) {
  // which-th eigenvalue (0-based, ascending) by bisection on [lo, hi]
  for (int it = 0; it < 200 && hi - lo > 1e-15 * std::max(1.0, std::fabs(hi)); ++it) {
    const double mid = 0.5 * (lo + hi);
    if (sturm_count(d, e, mid) > which) hi = mid;
    else lo = mid;
  }
  return 0.5 * (lo + hi);
}

}  // namespace

// Extreme eigenvalues of the Lanczos matrix of CG with coefficients alpha_k, beta_k
// (k < K): T_kk = 1/alpha_k + beta_{k-1}/alpha_{k-1}, T_{k,k+1} = sqrt(beta_k)/alpha_k.
bool lanczos_extremes(const std::vector<double>& alpha, const std::vector<double>& beta, double* lo, double* hi) {
  const size_t K = alpha.size();
  if (K < 2) return false;
  std::vector<double> d(K), e(K - 1);
  for (size_t k = 0; k < K; ++k) {
    if (!(alpha[k] > 0)) return false;
    d[k] = 1.0 / alpha[k] + (k ? beta[k - 1] / alpha[k - 1] : 0.0);
    if (k + 1 < K) e[k] = std::sqrt(std::max(beta[k], 0.0)) / alpha[k];
  }
  double glo = d[0], ghi = d[0];
  for (size_t k = 0; k < K; ++k) {
    const double r = (k ? std::fabs(e[k - 1]) : 0.0) + (k + 1 < K ? std::fabs(e[k]) : 0.0);
    glo = std::min(glo, d[k] - r);
    ghi = std::max(ghi, d[k] + r);
  }
  *lo = tridiag_eig(d, e, 0, glo, ghi);
  *hi = tridiag_eig(d, e, (int)K - 1, glo, ghi);
  return true;
}

int hybrid_choose(int N, const double* sig, double lmin, double lmax, double tol, double ms_iter, double ms_mg,
                  int* n_out, double* cost_out) {
  if (N < 1 || N > NDTM_MAX_SHIFTS || !sig || !n_out || !(lmin > 0) || !(lmax >= lmin) || !(tol > 0 && tol < 1) ||
      !(ms_iter > 0) || !(ms_mg >= 0))
    return NDTM_EINVAL;
  for (int i = 1; i < N; ++i)
    if (!(sig[i] < sig[i - 1]) || !(sig[i] > 0)) return NDTM_EINVAL;
  int best = N;
  double best_cost = 0;
  for (int n = N; n >= 1; --n) {
    const double s = sig[n - 1];
    const double kappa = (lmax + s) / (lmin + s);
    const double iters = 0.5 * std::sqrt(kappa) * std::log(2.0 / tol);
    const double cost = iters * ms_iter + (N - n) * ms_mg;
    if (n == N || cost < best_cost) {
      best = n;
      best_cost = cost;
    }
  }
  *n_out = best;
  if (cost_out) *cost_out = best_cost;
  return NDTM_OK;
}

}  // namespace ndtm

using namespace ndtm;

extern "C" {

int ndtm_hybrid_split(int n_shifts, const double* sigma_desc, double lambda_min, double lambda_max, double tol,
                      double ms_per_iteration, double ms_per_mg_shift, int* n_out) {
  return hybrid_choose(n_shifts, sigma_desc, lambda_min, lambda_max, tol, ms_per_iteration, ms_per_mg_shift, n_out,
                       nullptr);
}

int ndtm_spectrum_estimate(const ndtm_ctx* c, double* lambda_min, double* lambda_max) {
  if (!c || !lambda_min || !lambda_max) return NDTM_EINVAL;
  if (!(c->est_lmin > 0)) return NDTM_ESTATE;
  *lambda_min = c->est_lmin;
  *lambda_max = c->est_lmax;
  return NDTM_OK;
}

}  // extern "C"
