// Minimal-residual initial guess over the converged solutions.
//
// Generalises the interpolated guesses of section 4.2: instead of the
// Lagrange coefficients, the coefficients c (complex) minimise the residual
// || b - (Q^2 + sigma_t) sum_i c_i x_i || over the span of the converged
// solutions x_i of the shifts sigma_i.  By the identity of appendix B,
// (Q^2 + sigma_t) x_i = b - r_i - (sigma_i - sigma_t) x_i, so with the node
// residuals r_i (below the solver tolerance) left out the residual of any
// combination is b + sum_i c_i w_i, w_i = (sigma_i - sigma_t) x_i - b, and the
// whole minimisation needs only the Gram matrix of [b, x_1..x_K] and the
// overlaps of the current residual with b and the x_i: no operator
// application per node.
//
// Starting from the Lagrange guess x_L, each step computes the true residual
// r of the current guess (one application of Q^2), solves the K x K normal
// equations G y = -g, G_ij = <w_i, w_j>, g_i = <w_i, r>, with a small
// Tikhonov term for the nearly collinear solutions, and sets x += sum y_i x_i.
// The true residual of the result decides whether the step is kept; a step
// that does not reduce it is undone.  Because each step starts from the exact
// residual, the cancellation of the Gram form only limits how far one step
// gets, not the accuracy of the result.
#include <cmath>
#include <complex>
#include <vector>

#include "ctx.h"
#include "vec.h"

namespace ndtm {

namespace {

using cd = std::complex<double>;

// Solves (A + eps I) y = rhs for Hermitian positive semidefinite A (n x n,
// row-major) by Cholesky; eps = rel_eps * max diag.  Returns false on failure.
bool hpd_solve(std::vector<cd> A, std::vector<cd> rhs, int n, double rel_eps, std::vector<cd>* y) {
  double dmax = 0;
  for (int i = 0; i < n; ++i) dmax = std::max(dmax, A[i * n + i].real());
  if (!(dmax > 0)) return false;
  for (int i = 0; i < n; ++i) A[i * n + i] += rel_eps * dmax;
  // A = L L^H
  std::vector<cd> L(n * n, 0.0);
  for (int j = 0; j < n; ++j) {
    double d = A[j * n + j].real();
    for (int k = 0; k < j; ++k) d -= std::norm(L[j * n + k]);
    if (!(d > 0)) return false;
    const double ljj = std::sqrt(d);
    L[j * n + j] = ljj;
    for (int i = j + 1; i < n; ++i) {
      cd s = A[i * n + j];
      for (int k = 0; k < j; ++k) s -= L[i * n + k] * std::conj(L[j * n + k]);
      L[i * n + j] = s / ljj;
    }
  }
  // L z = rhs, L^H y = z
  for (int i = 0; i < n; ++i) {
    cd s = rhs[i];
    for (int k = 0; k < i; ++k) s -= L[i * n + k] * rhs[k];
    rhs[i] = s / L[i * n + i];
  }
  for (int i = n - 1; i >= 0; --i) {
    cd s = rhs[i];
    for (int k = i + 1; k < n; ++k) s -= std::conj(L[k * n + i]) * rhs[k];
    rhs[i] = s / L[i * n + i];
  }
  *y = rhs;
  return true;
}

}  // namespace

void gram_extend(ndtm_ctx* c, GramCache* g, const HalfField& b, const std::vector<HalfField>& xs, int K,
                 hipStream_t st) {
  const size_t n = half_elems(c);
  if ((int)g->M.size() != 17 * 17) {
    g->M.assign(17 * 17, 0.0);
    g->count = 0;
  }
  double* d = c->dscal + 2048;
  // vectors B_0 = b, B_j = x_{j-1}; each new column j holds <B_i, B_j> for i <= j
  for (int j = g->count; j <= K; ++j) {
    std::vector<const void*> B(j + 1);
    B[0] = b.v;
    for (int i = 1; i <= j; ++i) B[i] = xs[i - 1].v;
    vmultidot(P64, B.data(), j + 1, B[j], n, c->vred, d, st);
    (void)hipMemcpyAsync(c->hscal, d, 2 * (j + 1) * sizeof(double), hipMemcpyDeviceToHost, st);
    (void)hipStreamSynchronize(st);
    for (int i = 0; i <= j; ++i) {
      const cd v(c->hscal[2 * i], c->hscal[2 * i + 1]);
      g->M[i * 17 + j] = v;
      g->M[j * 17 + i] = std::conj(v);
    }
  }
  g->count = std::max(g->count, K + 1);
}

int guess_projection(ndtm_ctx* c, const std::vector<double>& nodes, const std::vector<HalfField>& xs, double sig_t,
                     const HalfField& b, const HalfField& x, GramCache* gram, double* lag_res, double* proj_res,
                     hipStream_t st) {
  const int K = (int)nodes.size();
  if (K < 1) return fail(c, NDTM_EINVAL, "projection guess: no converged solutions");
  if (K + 1 > 16) return fail(c, NDTM_EINVAL, "projection guess: at most 15 nodes");
  const size_t n = half_elems(c);
  HalfField r = half_field(c, "pg_r", P64), xb = half_field(c, "pg_xb", P64);
  if (!r.v || !xb.v) return fail(c, NDTM_ENOMEM, "projection guess: workspace");
  // start: the Lagrange guess over the nodes the interpolation keeps
  const int first = guess_first_node(nodes, sig_t);
  {
    std::vector<double> sub(nodes.begin() + first, nodes.end());
    std::vector<double> l(sub.size(), 1.0);
    for (size_t i = 0; i < sub.size(); ++i)
      for (size_t j = 0; j < sub.size(); ++j)
        if (j != i) l[i] *= (sig_t - sub[j]) / (sub[i] - sub[j]);
    std::vector<const double2*> V(sub.size());
    std::vector<double2> cc(sub.size());
    for (size_t i = 0; i < sub.size(); ++i) {
      V[i] = (const double2*)xs[first + i].v;
      cc[i] = make_double2(l[i], 0.0);
    }
    blas_lincomb((double2*)x.v, V.data(), cc.data(), (int)sub.size(), n, st);
  }
  double res = true_residual(c, x, b, sig_t, r, st);
  *lag_res = res;
  // Gram matrix of B = [b, x_1..x_K], kept across the targets of one solve
  gram_extend(c, gram, b, xs, K, st);
  auto M = [&](int i, int j) { return gram->M[i * 17 + j]; };
  std::vector<const void*> B(K + 1);
  B[0] = b.v;
  for (int i = 0; i < K; ++i) B[1 + i] = xs[i].v;
  double* d = c->dscal + 2048;
  std::vector<double> dl(K);
  for (int i = 0; i < K; ++i) dl[i] = nodes[i] - sig_t;
  // G_ij = <w_i, w_j>, w_i = dl_i x_i - b
  std::vector<cd> G(K * K);
  for (int i = 0; i < K; ++i)
    for (int j = 0; j < K; ++j)
      G[i * K + j] = M(0, 0) - dl[j] * M(0, j + 1) - dl[i] * M(i + 1, 0) + dl[i] * dl[j] * M(i + 1, j + 1);
  for (int step = 0; step < 3 && std::isfinite(res) && res > 0; ++step) {
    // g_i = <w_i, r> = dl_i <x_i, r> - <b, r>
    vmultidot(P64, B.data(), K + 1, r.v, n, c->vred, d, st);
    NDTM_HIP(c, hipMemcpyAsync(c->hscal, d, 2 * (K + 1) * sizeof(double), hipMemcpyDeviceToHost, st));
    NDTM_HIP(c, hipStreamSynchronize(st));
    const cd hb(c->hscal[0], c->hscal[1]);
    std::vector<cd> g(K);
    for (int i = 0; i < K; ++i) g[i] = -(dl[i] * cd(c->hscal[2 * (1 + i)], c->hscal[2 * (1 + i) + 1]) - hb);
    std::vector<cd> y;
    if (!hpd_solve(G, g, K, 1e-13, &y)) break;
    blas_copy((double2*)xb.v, (const double2*)x.v, n, st);
    // x += sum_i y_i x_i in one pass (coefficients staged through pinned memory)
    for (int i = 0; i < K; ++i) {
      c->hscal[2 * i] = y[i].real();
      c->hscal[2 * i + 1] = y[i].imag();
    }
    NDTM_HIP(c, hipMemcpyAsync(d, c->hscal, 2 * K * sizeof(double), hipMemcpyHostToDevice, st));
    vlincomb_dev(P64, x.v, B.data() + 1, K, d, 1, n, st);
    const double nres = true_residual(c, x, b, sig_t, r, st);
    if (!(nres < 0.9 * res)) {
      blas_copy((double2*)x.v, (const double2*)xb.v, n, st);
      break;
    }
    res = nres;
  }
  *proj_res = res;
  return NDTM_OK;
}

}  // namespace ndtm
