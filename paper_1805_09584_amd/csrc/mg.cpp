// Two-level aggregation multigrid for the shifted single systems, the
// difference-of-single-solves form (case C) with FP64 defect correction, the
// Lagrange-interpolated initial guesses and the hybrid driver (sections 3.1,
// 3.2, 4.2 and 4.4 of the paper).
//
// Single systems.  (Q +- i m) x = c with Q = Gamma5 tau1 S is equivalent to
// (S +- i m Gamma5 tau1) x = Gamma5 tau1 c, and S +- i m Gamma5 tau1 is the odd
// Schur complement of the full-lattice operator
//   D'_+- = D_ND +- i m (Gamma5 x tau1) P_odd
// (the even-even block is unchanged).  The outer solver is FGMRES in FP64 on
// the odd system; each preconditioner application is one two-level cycle on
// the full lattice for D'_+- applied to (0, r_o), returning the odd part:
//   coarse correction z = P D'_c^-1 P^+ r   (the coarse system by a fixed
//   number of GMRES iterations on the device), then post-smoothing on D'_+-
//   (0 pre- and smooth_iters post-smoothing iterations): minimal-residual steps
//   on the whole lattice, or sweeps of the Schwarz alternating procedure (SAP)
//   over the aggregates as blocks, each block solved by minimal-residual steps.
// The cycle runs in FP32 (FP16 storage of P and links on request), or FP64.
//
// Coarse operator (eq:non-degenerate_coarse with P_ND = P x I2 and the
// odd-site shift term): D'_c = D_W,c x I2 + i d mubar Gamma5_c x tau3
//   - epsbar tau1 +- i m (Gamma5_c P^+ P_odd P) x tau1.
//
// Setup: N_v test vectors by inverse iteration; each sweep replaces v by
// setup_smooth CG steps on the normal equations D^+ D x = v and normalises x.
// By default (setup_nd = 1) D is the doublet operator itself and both flavour
// components of each field become test vectors; with setup_nd = 0 the doublet
// kernel runs at epsbar = 0, so flavour 0 iterates D_W + i mubar Gamma5 and
// flavour 1 D_W - i mubar Gamma5 (section 3.2: the one-flavour twisted-mass
// setup reused for the doublet).
//
// Case C (eq:lindif): (Q^2 + m^2)^-1 r = (i/2m)[(Q + i m)^-1 r - (Q - i m)^-1 r].
// The squared residual of case C grows by up to sqrt(lambda_max + m^2)/m over
// the single residuals (appendix A), so each multigrid shift is refined by
// FP64 defect correction on the true residual b - (Q^2 + m^2) x until it
// reaches the tolerance.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstring>

#include "ctx.h"
#include "vec.h"

namespace ndtm {

struct MGData {
  MGGeom g{};
  ndtm_mg_params prm{};
  int cprec = P32;  // precision of the cycle's fields and coarse operator
  int sprec = P32;  // precision of its stencil: cprec, or P32H (FP32 fields on FP16 links)
  float* Psc = nullptr;  // FP16-storage cycle: Pc holds FP16 entries with these per-site scales
  double2* P64 = nullptr;
  double2* D64 = nullptr;
  double2* Bo64 = nullptr;
  void* Pc = nullptr;   // P in cycle precision (aliases P64 for FP64)
  void* Dc = nullptr;
  void* Boc = nullptr;
  size_t ncoarse = 0;   // complex elements of a coarse doublet vector
  std::vector<void*> cV;  // coarse basis (cycle precision), coarse_iters + 1
  void* cW = nullptr;     // Arnoldi work vectors: step j's new direction in cW (j even) or cW2 (odd)
  void* cW2 = nullptr;
  void* cR = nullptr;
  void* cT = nullptr;     // coarse residual of the restarted solve
  void* cX = nullptr;     // coarse solution
  double* dH = nullptr;   // Hessenberg columns, coarse_iters x (coarse_iters+1) complex
  double* dsub = nullptr; // subdiagonal norms^2
  double* dy = nullptr;   // least-squares coefficients
  double* dbeta = nullptr;
  double* dtmp = nullptr;
  double* dh2 = nullptr;  // second Gram-Schmidt pass coefficients, laid out as dH
  double* dpart = nullptr;  // smoother: stencil partials of <D'S, S>, ||D'S||^2 ([3][2 nblk])
  // even-odd coarsest level: -A_ee^-1 per value of m (null when that m's site terms
  // could not be inverted), the Schur complement's work vectors and the build scratch
  bool eo = false;
  std::vector<std::pair<double, void*>> einv;
  void *cU = nullptr, *cT2 = nullptr, *cR2 = nullptr;
  double2* einv_scratch = nullptr;
  int einv_chunk = 0;
  unsigned* einv_bad = nullptr;
  std::vector<void*> owned;
  bool ready = false;
  // cycle graphs: one per value of the odd-site shift m, replayed on the caller's stream
  hipStream_t cap = nullptr;
  std::vector<std::pair<double, hipGraphExec_t>> graphs;
  bool use_graphs = true;
};

static void* mg_alloc(ndtm_ctx* c, MGData* M, size_t bytes) {
  void* p = dev_alloc(c, bytes);
  if (!p) return nullptr;
  (void)hipMemset(p, 0, bytes);
  M->owned.push_back(p);
  return p;
}

static size_t csz(int prec) { return prec == P64 ? sizeof(double2) : sizeof(float2); }

// views of a full-lattice field stored as one buffer (even half then odd half)
struct Full {
  HalfField e, o;
  void* base = nullptr;
};

// k FP64 coarse systems D'_c(m_r) x_r = b_r at once (x, b: [k][Vc][2][2Nv]); the batched
// solve of ndtm_mg_coarse_solve_multi (FP64 coarse blocks)
int coarse_solve_multi(ndtm_ctx* c, MGData* M, void* xc, const void* bc, int k, const double* m, hipStream_t st);

static Full full_field(ndtm_ctx* c, const std::string& name, int prec) {
  Full f;
  const size_t n = half_elems(c);
  const size_t es = prec == P64 ? 16 : 8;
  f.base = ws_get(c, name + (prec == P64 ? "#f64" : "#f32"), 2 * n * es);
  f.e.prec = f.o.prec = prec;
  f.e.v = f.base;
  f.o.v = f.base ? static_cast<char*>(f.base) + n * es : nullptr;
  return f;
}

// Algorithmic bytes of the cycle's transfer and coarse kernels (element size es
// of a complex number in the cycle precision): restriction and prolongation
// stream P (V x 12 x Nv) and one full doublet field (V x 24) and touch one
// coarse vector; the coarse stencil streams the 9 blocks (2Nv)^2 of every coarse
// site and the odd-projector block (2 x Nv^2), and reads/writes a coarse vector.
static double transfer_bytes(const MGData* M) {
  const double es = (double)csz(M->cprec), Nv = M->g.Nv;
  const double V = (double)M->g.Vc * M->g.nloc;
  // FP16 storage of P: 4 bytes an entry and one scale per site
  const double pb = M->Psc ? 12.0 * Nv * 4.0 + 4.0 : 12.0 * Nv * es;
  return V * (pb + 24.0 * es) + (double)M->ncoarse * es;
}
static double coarse_bytes(const MGData* M) {
  const double es = (double)csz(M->cprec), n2 = 2.0 * M->g.Nv;
  // five stored blocks and the odd-projector block read per coarse site (the backward
  // hops come from the neighbours' forward blocks), the input and output vectors
  return (double)M->g.Vc * (5.0 * n2 * n2 + 0.5 * n2 * n2) * es + 2.0 * (double)M->ncoarse * es;
}

// ---- even-odd coarsest level ------------------------------------------------
// -A_ee^-1 of D'_c(m)'s even site terms, built on first use of m (outside any graph
// capture: mg_cycle asks for it before capturing) and kept until the next setup.
static const void* einv_for(ndtm_ctx* c, MGData* M, double m, hipStream_t st) {
  for (auto& e : M->einv)
    if (e.first == m) return e.second;
  const int N = 4 * M->g.Nv;
  const size_t bytes = (size_t)(M->g.Vc / 2) * N * N * csz(M->cprec);
  void* E = dev_alloc(c, bytes);
  if (E) M->owned.push_back(E);
  bool ok = E != nullptr;
  if (ok) {
    (void)hipMemsetAsync(M->einv_bad, 0, sizeof(unsigned), st);
    const double mubar_c = M->prm.coarse_mu_factor * c->mubar;
    for (int X0 = 0; X0 < M->g.Vc; X0 += M->einv_chunk)
      mg_einv_build(M->cprec, M->g, X0, std::min(M->einv_chunk, M->g.Vc - X0), M->Dc, M->Boc, mubar_c, c->epsbar, m,
                    M->einv_scratch, E, M->einv_bad, st);
    unsigned bad = 0;
    (void)hipMemcpyAsync(&bad, M->einv_bad, sizeof(unsigned), hipMemcpyDeviceToHost, st);
    (void)hipStreamSynchronize(st);
    ok = bad == 0;
  }
  M->einv.push_back({m, ok ? E : nullptr});
  return ok ? E : nullptr;
}

// w_o = S v_o with S = D_oo - D_oe A_ee^-1 D_eo the odd Schur complement of D'_c(m), for
// coarse vectors whose even part is zero (v) or stays zero (w)
static void schur_apply(ndtm_ctx* c, MGData* M, const void* E, const void* v, void* w, double m, double eps,
                        hipStream_t st) {
  const int cp = M->cprec;
  const double mubar_c = M->prm.coarse_mu_factor * c->mubar;
  ProfScope ps(c, NDTM_PROF_COARSE, coarse_bytes(M), st);
  mg_coarse_apply(cp, M->g, M->Dc, M->Boc, v, M->cU, mubar_c, eps, m, st, nullptr, nullptr, 0);  // D_eo v_o
  mg_einv_apply(cp, M->g, E, M->cU, v, M->cT2, st);  // (-A_ee^-1 D_eo v_o) + v_o
  mg_coarse_apply(cp, M->g, M->Dc, M->Boc, M->cT2, w, mubar_c, eps, m, st, nullptr, nullptr, 1);
}

// One GMRES(kc) cycle from zero on S y_o = src_o (src's even part zero), as coarse_gmres_cycle
static void eo_gmres_cycle(ndtm_ctx* c, MGData* M, const void* E, const void* src, const double* src2, void* sol,
                           int accumulate, double m, double eps, hipStream_t st) {
  const int cp = M->cprec;
  const size_t n = M->ncoarse;
  const int kc = M->prm.coarse_iters;
  // the Schur complement writes the odd sites only: the work vectors' even parts are
  // cleared (the full coarse solve may have left values there)
  mg_coarse_zero_parity(cp, M->g, M->cW, 0, st);
  mg_coarse_zero_parity(cp, M->g, M->cW2, 0, st);
  vscale_inv_sqrt(cp, M->cV[0], src, src2, n, st);
  for (int j = 0; j < kc; ++j) {
    void* w = (j & 1) ? M->cW2 : M->cW;
    schur_apply(c, M, E, M->cV[j], w, m, eps, st);
    double* hcol = M->dH + 2 * (size_t)j * (kc + 1);
    double* hcol2 = M->dh2 + 2 * (size_t)j * (kc + 1);
    vmultidot(cp, (const void* const*)M->cV.data(), j + 1, w, n, c->vred, hcol, st);
    vmulti_axpy_multidot(cp, w, (const void* const*)M->cV.data(), j + 1, hcol, n, c->vred, hcol2, st);
    vmulti_axpy_norm_dev(cp, w, (const void* const*)M->cV.data(), j + 1, hcol2, n, c->vred, M->dsub + j, st);
    if (j + 1 < kc) vscale_inv_sqrt(cp, M->cV[j + 1], w, M->dsub + j, n, st);
  }
  hess_lsq(M->dH, M->dh2, kc + 1, kc, src2, M->dsub, M->dy, st);
  vlincomb_dev(cp, sol, (const void* const*)M->cV.data(), kc, M->dy, accumulate, n, st);
}

// sol ~ D'_c(m)^-1 rhs through the odd Schur complement: rhs_o' = rhs_o - D_oe A_ee^-1 rhs_e,
// GMRES on S sol_o = rhs_o' (restarted on its true residual when coarse_tol > 0), then
// sol_e = A_ee^-1 (rhs_e - D_eo sol_o).  Returns false if this m has no even inverse.
static bool coarse_solve_eo(ndtm_ctx* c, MGData* M, const void* rhs, void* sol, double m, double eps,
                            hipStream_t st) {
  const void* E = einv_for(c, M, m, st);
  if (!E) return false;
  const int cp = M->cprec;
  const size_t n = M->ncoarse;
  const double mubar_c = M->prm.coarse_mu_factor * c->mubar;
  // cR2 = rhs_o - D_oe A_ee^-1 rhs_e on the odd sites, zero on the even ones
  mg_einv_apply(cp, M->g, E, rhs, nullptr, M->cT2, st);
  {
    ProfScope ps(c, NDTM_PROF_COARSE, coarse_bytes(M), st);
    mg_coarse_apply(cp, M->g, M->Dc, M->Boc, M->cT2, M->cR2, mubar_c, eps, m, st, nullptr, nullptr, 1);
  }
  vaxpby(cp, M->cR2, make_double2(1, 0), rhs, make_double2(1, 0), n, st);
  mg_coarse_zero_parity(cp, M->g, M->cR2, 0, st);
  vnorm2(cp, M->cR2, n, c->vred, M->dbeta, st);
  eo_gmres_cycle(c, M, E, M->cR2, M->dbeta, sol, 0, m, eps, st);
  if (M->prm.coarse_tol > 0.0) {
    // the full coarse residual equals the Schur residual on the odd sites (its even part
    // vanishes by the construction of sol_e): the tolerance is relative to ||rhs||
    vnorm2(cp, rhs, n, c->vred, M->dbeta + 2, st);
    (void)hipMemcpyAsync(c->hscal, M->dbeta + 2, sizeof(double), hipMemcpyDeviceToHost, st);
    (void)hipStreamSynchronize(st);
    const double rhs2 = c->hscal[0];
    const double tol2 = M->prm.coarse_tol * M->prm.coarse_tol * rhs2;
    for (int cyc = 1; cyc < M->prm.coarse_cycles && rhs2 > 0.0; ++cyc) {
      mg_coarse_zero_parity(cp, M->g, M->cT, 0, st);
      schur_apply(c, M, E, sol, M->cT, m, eps, st);
      vaxpby(cp, M->cT, make_double2(1, 0), M->cR2, make_double2(-1, 0), n, st);  // cT = rhs' - S sol
      vnorm2(cp, M->cT, n, c->vred, M->dbeta + 1, st);
      (void)hipMemcpyAsync(c->hscal, M->dbeta + 1, sizeof(double), hipMemcpyDeviceToHost, st);
      (void)hipStreamSynchronize(st);
      const double res2 = c->hscal[0];
      if (!(res2 > tol2) || !std::isfinite(res2)) break;
      eo_gmres_cycle(c, M, E, M->cT, M->dbeta + 1, sol, 1, m, eps, st);
    }
  }
  // sol_e = A_ee^-1 (rhs_e - D_eo sol_o) = -A_ee^-1 (D_eo sol_o - rhs_e)
  {
    ProfScope ps(c, NDTM_PROF_COARSE, coarse_bytes(M), st);
    mg_coarse_apply(cp, M->g, M->Dc, M->Boc, sol, M->cU, mubar_c, eps, m, st, nullptr, nullptr, 0);
  }
  vaxpby(cp, M->cU, make_double2(-1, 0), rhs, make_double2(1, 0), n, st);
  mg_einv_apply(cp, M->g, E, M->cU, sol, sol, st);
  return true;
}

// ---- coarse solve: GMRES on the device ------------------------------------
// One GMRES(kc) cycle from zero on D'_c y = src; *src2 = ||src||^2 on the device.
// The solution is written (accumulate = 0) or added (1) to sol, which must not be
// cW or cW2, the Arnoldi work vectors.  Step j's direction w_j is orthogonalised in
// place; the coarse stencil of step j + 1 reads it, normalises it as it reads, and
// stores the basis vector V_{j+1} (the last w is never normalised: no step reads it).
static void coarse_gmres_cycle(ndtm_ctx* c, MGData* M, const void* src, const double* src2, void* sol,
                               int accumulate, double m, double eps, hipStream_t st) {
  const int cp = M->cprec;
  const size_t n = M->ncoarse;
  const int kc = M->prm.coarse_iters;
  const double mubar_c = M->prm.coarse_mu_factor * c->mubar;
  vscale_inv_sqrt(cp, M->cV[0], src, src2, n, st);
  for (int j = 0; j < kc; ++j) {
    void* w = (j & 1) ? M->cW2 : M->cW;
    {
      ProfScope ps(c, NDTM_PROF_COARSE, coarse_bytes(M), st);
      if (j == 0)
        mg_coarse_apply(cp, M->g, M->Dc, M->Boc, M->cV[0], w, mubar_c, eps, m, st);
      else
        mg_coarse_apply(cp, M->g, M->Dc, M->Boc, (j & 1) ? M->cW : M->cW2, w, mubar_c, eps, m, st, M->dsub + j - 1,
                        M->cV[j]);
    }
    // classical Gram-Schmidt with one reorthogonalisation; the second pass's
    // coefficients go to their own Hessenberg array, added to the first by the
    // least-squares step
    double* hcol = M->dH + 2 * (size_t)j * (kc + 1);
    double* hcol2 = M->dh2 + 2 * (size_t)j * (kc + 1);
    vmultidot(cp, (const void* const*)M->cV.data(), j + 1, w, n, c->vred, hcol, st);
    vmulti_axpy_multidot(cp, w, (const void* const*)M->cV.data(), j + 1, hcol, n, c->vred, hcol2, st);
    vmulti_axpy_norm_dev(cp, w, (const void* const*)M->cV.data(), j + 1, hcol2, n, c->vred, M->dsub + j, st);
  }
  hess_lsq(M->dH, M->dh2, kc + 1, kc, src2, M->dsub, M->dy, st);
  vlincomb_dev(cp, sol, (const void* const*)M->cV.data(), kc, M->dy, accumulate, n, st);
}

// sol ~ D'_c(m)^-1 rhs.  coarse_tol = 0: one cycle from zero, a fixed launch
// sequence with no host synchronisation.  coarse_tol > 0: restarted on the true
// coarse residual (read by the host after each cycle) until it is below
// coarse_tol ||rhs|| or coarse_cycles cycles have run.
static void coarse_solve(ndtm_ctx* c, MGData* M, const void* rhs, void* sol, double m, double eps,
                         hipStream_t st) {
  if (M->eo && coarse_solve_eo(c, M, rhs, sol, m, eps, st)) return;
  const int cp = M->cprec;
  const size_t n = M->ncoarse;
  const double mubar_c = M->prm.coarse_mu_factor * c->mubar;
  vnorm2(cp, rhs, n, c->vred, M->dbeta, st);
  coarse_gmres_cycle(c, M, rhs, M->dbeta, sol, 0, m, eps, st);
  if (!(M->prm.coarse_tol > 0.0)) return;
  (void)hipMemcpyAsync(c->hscal, M->dbeta, sizeof(double), hipMemcpyDeviceToHost, st);
  (void)hipStreamSynchronize(st);
  const double rhs2 = c->hscal[0];
  const double tol2 = M->prm.coarse_tol * M->prm.coarse_tol * rhs2;
  for (int cyc = 1; cyc < M->prm.coarse_cycles && rhs2 > 0.0; ++cyc) {
    {
      ProfScope ps(c, NDTM_PROF_COARSE, coarse_bytes(M), st);
      mg_coarse_apply(cp, M->g, M->Dc, M->Boc, sol, M->cT, mubar_c, eps, m, st);
    }
    vaxpby(cp, M->cT, make_double2(1, 0), rhs, make_double2(-1, 0), n, st);  // cT = rhs - D sol
    vnorm2(cp, M->cT, n, c->vred, M->dbeta + 1, st);
    (void)hipMemcpyAsync(c->hscal, M->dbeta + 1, sizeof(double), hipMemcpyDeviceToHost, st);
    (void)hipStreamSynchronize(st);
    const double res2 = c->hscal[0];
    if (!(res2 > tol2) || !std::isfinite(res2)) break;
    coarse_gmres_cycle(c, M, M->cT, M->dbeta + 1, sol, 1, m, eps, st);
  }
}

// full-lattice D' in the cycle precision
static void dprime(ndtm_ctx* c, int prec, const Full& y, const Full& x, double m, hipStream_t st) {
  apply_dfull(c, prec, y.e, y.o, x.e, x.o, m, st);
}

// y = D' x, with the partials of <y, x> and ||y||^2 of both parity passes in
// part[q * 2 nblk + i] (the two hops of apply_dfull, each reducing over its sites)
static void dprime_mr(ndtm_ctx* c, int prec, const Full& y, const Full& x, double m, double* part, hipStream_t st) {
  const int hg = hop_grid(c->g);
  hop(c, prec, EPI_SITE, RED_MR, 0, x.o, y.e, &x.e, nullptr, 0.0, -0.5, 0, part, st);
  hop(c, prec, EPI_SITE, RED_MR, 1, x.e, y.o, &x.o, nullptr, m, -0.5, 0, part + hg, st);
}

// Post-smoothing of D'(m) z = R from the coarse correction in Z: smooth_iters
// minimal-residual steps on the whole lattice, or with SAP (section 3's smoother)
// smooth_iters sweeps; in each, the blocks of colour 0 and then of colour 1 solve
// D'_B e = s_B by minimal-residual steps in the block kernel, with the residual
// S = R - D'Z formed again before each colour but the first.
static void mg_smooth(ndtm_ctx* c, MGData* M, const Full& R, const Full& Z, double m, hipStream_t st) {
  const int cp = M->cprec;
  const size_t nh = half_elems(c);
  const int nu = M->prm.smooth_iters;
  if (nu <= 0) return;
  Full S = full_field(c, "mg_S", cp), Tt = full_field(c, "mg_T", cp);
  dprime(c, M->sprec, S, Z, m, st);
  vaxpby(cp, S.base, make_double2(1, 0), R.base, make_double2(-1, 0), 2 * nh, st);  // S = R - D'Z
  if (M->prm.smoother == NDTM_SMOOTH_SAP) {
    const int lp = M->sprec == P32H ? P16 : M->sprec;
    for (int sw = 0; sw < nu; ++sw)
      for (int col = 0; col < 2; ++col) {
        if (sw + col > 0) {
          dprime(c, M->sprec, S, Z, m, st);
          vaxpby(cp, S.base, make_double2(1, 0), R.base, make_double2(-1, 0), 2 * nh, st);
        }
        launch_sap_block(M->sprec, c->g, M->prm.block, col, M->prm.sap_mr_iters, c->op, c->U[lp][0], c->U[lp][1],
                         S.e, S.o, Z.e, Z.o, m, -0.5, st);
      }
    return;
  }
  for (int it = 0; it < nu; ++it) {
    // T = D' S with <T, S>, ||T||^2 reduced in the stencil epilogue; the update
    // kernel forms omega from those partials
    dprime_mr(c, M->sprec, Tt, S, m, M->dpart, st);
    vmr_update_part(cp, Z.base, S.base, Tt.base, M->dpart, 2 * hop_grid(c->g), it + 1 < nu, 2 * nh, st);
  }
}

// Z ~ D'^-1 R on the full lattice (cycle precision): coarse correction then the
// post-smoother (mg_smooth).  The fine operator is the one in c->op (D'(m)); eps
// is the flavour-mixing term the coarse operator uses with it.
static void mg_vcycle(ndtm_ctx* c, MGData* M, const Full& R, const Full& Z, double m, double eps, hipStream_t st) {
  const int cp = M->cprec;
  {
    ProfScope ps(c, NDTM_PROF_RESTRICT, transfer_bytes(M), st);
    mg_restrict(cp, M->g, M->Pc, M->Psc, R.e.v, R.o.v, M->cR, st);
  }
  coarse_solve(c, M, M->cR, M->cX, m, eps, st);
  {
    ProfScope ps(c, NDTM_PROF_PROLONG, transfer_bytes(M), st);
    mg_prolong(cp, M->g, M->Pc, M->Psc, M->cX, Z.e.v, Z.o.v, st);
  }
  mg_smooth(c, M, R, Z, m, st);
}

// z_o ~ S'^-1 r_o : the cycle for D'(m) applied to (0, r_o), odd part; FP64 in/out
// The cycle between fixed buffers (mg_R with a zero even half, mg_Z) is a fixed
// sequence of about a hundred small launches for a given m; it is captured once
// per m into a HIP graph (on the context's own stream, with timing events off)
// and replayed on the caller's stream.  Every buffer it touches is allocated at
// setup, so nothing is allocated or cleared by memset inside the capture.
static hipGraphExec_t cycle_graph(ndtm_ctx* c, MGData* M, double m) {
  for (auto& g : M->graphs)
    if (g.first == m) return g.second;
  const int cp = M->cprec;
  Full R = full_field(c, "mg_R", cp), Z = full_field(c, "mg_Z", cp);
  if (!M->cap && hipStreamCreateWithFlags(&M->cap, hipStreamNonBlocking) != hipSuccess) return nullptr;
  const int mask = c->prof_mask;
  c->prof_mask = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  if (hipStreamBeginCapture(M->cap, hipStreamCaptureModeRelaxed) == hipSuccess) {
    mg_vcycle(c, M, R, Z, m, c->epsbar, M->cap);
    if (hipStreamEndCapture(M->cap, &graph) == hipSuccess && graph) {
      if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) exec = nullptr;
      (void)hipGraphDestroy(graph);
    }
  }
  c->prof_mask = mask;
  if (exec) M->graphs.push_back({m, exec});
  return exec;
}

static void mg_cycle(ndtm_ctx* c, MGData* M, const HalfField& r64, const HalfField& z64, double m, hipStream_t st) {
  const int cp = M->cprec;
  const size_t nh = half_elems(c);
  Full R = full_field(c, "mg_R", cp), Z = full_field(c, "mg_Z", cp);
  vconvert_field(cp, R.o.v, P64, r64.v, 1, c->g.vh, c->g.stride, st);
  if (M->eo) (void)einv_for(c, M, m, st);  // built now, never inside a graph capture
  hipGraphExec_t g = M->use_graphs ? cycle_graph(c, M, m) : nullptr;
  if (g)
    (void)hipGraphLaunch(g, st);
  else
    mg_vcycle(c, M, R, Z, m, c->epsbar, st);
  vconvert_field(P64, z64.v, cp, Z.o.v, 1, c->g.vh, c->g.stride, st);
}

// The cycles of D'(+m) and D'(-m) side by side (case C's two signs): both residuals
// restricted, the two coarse systems solved together by the batched FP64 coarse solve
// (one matrix-core stencil launch per Arnoldi step for both), each correction
// prolonged and smoothed with its own sign.  FP64 in/out on the odd sites.
static bool mg_cycle_pair(ndtm_ctx* c, MGData* M, const HalfField* r64, const HalfField* z64, double m, hipStream_t st) {
  const int cp = M->cprec;
  const size_t nc = M->ncoarse;
  Full R[2] = {full_field(c, "mg_R", cp), full_field(c, "mg_R2", cp)};
  Full Z[2] = {full_field(c, "mg_Z", cp), full_field(c, "mg_Z2", cp)};
  double2* B = static_cast<double2*>(ws_get(c, "mp_B", 2 * nc * sizeof(double2)));
  double2* X = static_cast<double2*>(ws_get(c, "mp_X", 2 * nc * sizeof(double2)));
  if (!R[1].base || !Z[1].base || !B || !X) return false;
  for (int s = 0; s < 2; ++s) {
    // the even halves of R stay zero (the second pair's from its allocation)
    vconvert_field(cp, R[s].o.v, P64, r64[s].v, 1, c->g.vh, c->g.stride, st);
    ProfScope ps(c, NDTM_PROF_RESTRICT, transfer_bytes(M), st);
    mg_restrict(cp, M->g, M->Pc, M->Psc, R[s].e.v, R[s].o.v, M->cR, st);
    vconvert(P64, B + s * nc, cp, M->cR, nc, st);
  }
  const double ms[2] = {m, -m};
  if (coarse_solve_multi(c, M, X, B, 2, ms, st) != NDTM_OK) return false;
  for (int s = 0; s < 2; ++s) {
    vconvert(cp, M->cX, P64, X + s * nc, nc, st);
    {
      ProfScope ps(c, NDTM_PROF_PROLONG, transfer_bytes(M), st);
      mg_prolong(cp, M->g, M->Pc, M->Psc, M->cX, Z[s].e.v, Z[s].o.v, st);
    }
    mg_smooth(c, M, R[s], Z[s], ms[s], st);
    vconvert_field(P64, z64[s].v, cp, Z[s].o.v, 1, c->g.vh, c->g.stride, st);
  }
  return true;
}

// FGMRES in FP64 for (S + i m Gamma5 tau1) x = rhs, x starting from zero.
// Stops when the recursive residual <= tol * ||rhs||.  Returns iterations.
// Case C takes 5 FP64 half fields of the solve's phase region, FGMRES(k) 2k + 4 more.
static int fgmres_restart_clamp(int restart) { return std::max(2, std::min(restart, 32)); }
// case C's five fields, then FGMRES(k)'s 2k + 4 (twice with the signs paired)
int mg_region_fields(int fgmres_restart, bool pair) {
  return 5 + (pair ? 2 : 1) * (2 * fgmres_restart_clamp(fgmres_restart) + 4);
}

// FP64 half field j of the solve's phase region, else the named workspace buffer
static HalfField region_field(ndtm_ctx* c, size_t j, const std::string& name) {
  if (c->region && j < c->region_fields) {
    HalfField f;
    f.prec = P64;
    f.v = static_cast<double2*>(c->region) + j * half_elems(c);
    return f;
  }
  return half_field(c, name, P64);
}

static int fgmres(ndtm_ctx* c, MGData* M, const HalfField& rhs, const HalfField& x, double m, double tol, int restart,
                  int maxiter, double* res_out, hipStream_t st) {
  const size_t n = half_elems(c);
  restart = fgmres_restart_clamp(restart);
  std::vector<HalfField> V(restart + 1), Z(restart);
  size_t j0 = 5;  // after case C's five fields
  for (int j = 0; j <= restart; ++j) V[j] = region_field(c, j0++, "fg_v" + std::to_string(j));
  for (int j = 0; j < restart; ++j) Z[j] = region_field(c, j0++, "fg_z" + std::to_string(j));
  HalfField W = region_field(c, j0, "fg_w"), te = region_field(c, j0 + 1, "fg_te"),
            r = region_field(c, j0 + 2, "fg_r");
  bool have = W.v && te.v && r.v;
  for (auto& f : V) have = have && f.v;
  for (auto& f : Z) have = have && f.v;
  if (!have) {  // workspace exhausted: the caller reports NDTM_ENOMEM
    *res_out = INFINITY;
    return -1;
  }
  std::vector<const void*> Vp(restart + 1), Zp(restart);
  for (int j = 0; j <= restart; ++j) Vp[j] = V[j].v;
  for (int j = 0; j < restart; ++j) Zp[j] = Z[j].v;
  double* dh = c->dscal;  // [0, 2*restart): h, [2*restart, 4*restart): second pass, then norm2
  const double bn = std::sqrt(norm2_host(c, (const double2*)rhs.v, n, st));
  blas_zero(x.v, n * sizeof(double2), st);
  if (bn == 0) {
    *res_out = 0;
    return 0;
  }
  int total = 0;
  double res = bn;
  while (total < maxiter) {
    // r = rhs - A x
    apply_sshift(c, P64, r, x, te, m, st);
    blas_axpby((double2*)r.v, make_double2(1, 0), (const double2*)rhs.v, make_double2(-1, 0), n, st);
    const double beta = std::sqrt(norm2_host(c, (const double2*)r.v, n, st));
    res = beta;
    if (beta <= tol * bn) break;
    blas_axpby((double2*)V[0].v, make_double2(1.0 / beta, 0), (const double2*)r.v, make_double2(0, 0), n, st);
    std::vector<std::complex<double>> H((restart + 1) * restart, 0.0), cs(restart), sn(restart),
        g(restart + 1, 0.0);
    g[0] = beta;
    int k = 0;
    for (; k < restart && total < maxiter; ++k) {
      mg_cycle(c, M, V[k], Z[k], m, st);
      apply_sshift(c, P64, W, Z[k], te, m, st);
      // classical Gram-Schmidt, two passes
      vmultidot(P64, Vp.data(), k + 1, W.v, n, c->vred, dh, st);
      vmulti_axpy_multidot(P64, W.v, Vp.data(), k + 1, dh, n, c->vred, dh + 2 * restart, st);
      vmulti_axpy_norm_dev(P64, W.v, Vp.data(), k + 1, dh + 2 * restart, n, c->vred, dh + 4 * restart, st);
      vscale_inv_sqrt(P64, V[k + 1].v, W.v, dh + 4 * restart, n, st);
      (void)hipMemcpyAsync(c->hscal, dh, (4 * restart + 1) * sizeof(double), hipMemcpyDeviceToHost, st);
      (void)hipStreamSynchronize(st);
      ++total;
      for (int i = 0; i <= k; ++i)
        H[k * (restart + 1) + i] = std::complex<double>(c->hscal[2 * i] + c->hscal[2 * restart + 2 * i],
                                                        c->hscal[2 * i + 1] + c->hscal[2 * restart + 2 * i + 1]);
      const double hn = std::sqrt(std::max(0.0, c->hscal[4 * restart]));
      H[k * (restart + 1) + k + 1] = hn;
      for (int i = 0; i < k; ++i) {
        auto& a = H[k * (restart + 1) + i];
        auto& b = H[k * (restart + 1) + i + 1];
        const auto t = std::conj(cs[i]) * a + std::conj(sn[i]) * b;
        b = -sn[i] * a + cs[i] * b;
        a = t;
      }
      auto& a = H[k * (restart + 1) + k];
      auto& b = H[k * (restart + 1) + k + 1];
      const double den = std::sqrt(std::norm(a) + std::norm(b));
      if (!(den > 0) || !std::isfinite(den)) break;
      cs[k] = a / den;
      sn[k] = b / den;
      a = den;
      b = 0;
      g[k + 1] = -sn[k] * g[k];
      g[k] = std::conj(cs[k]) * g[k];
      res = std::abs(g[k + 1]);
      if (res <= tol * bn || hn == 0) {
        ++k;
        break;
      }
    }
    // y = R^-1 g, x += Z y
    std::vector<std::complex<double>> y(k);
    for (int i = k - 1; i >= 0; --i) {
      auto s = g[i];
      for (int j = i + 1; j < k; ++j) s -= H[j * (restart + 1) + i] * y[j];
      y[i] = s / H[i * (restart + 1) + i];
    }
    std::vector<double> yc(2 * k);
    for (int i = 0; i < k; ++i) {
      yc[2 * i] = y[i].real();
      yc[2 * i + 1] = y[i].imag();
    }
    (void)hipMemcpyAsync(c->dscal + 6 * restart, yc.data(), 2 * k * sizeof(double), hipMemcpyHostToDevice, st);
    vlincomb_dev(P64, x.v, Zp.data(), k, c->dscal + 6 * restart, 1, n, st);
    if (res <= tol * bn) {
      // confirm with the true residual at the top of the loop
      continue;
    }
  }
  *res_out = res / bn;
  return total;
}

// The FGMRES solves of (S + i m Gamma5 tau1) x_+ = rhs and (S - i m Gamma5 tau1) x_- = rhs
// in lock-step: while both are inside an Arnoldi cycle their preconditioner steps run as
// one paired cycle (mg_cycle_pair); a system that has converged (or whose cycle ended)
// waits, and the other continues with single cycles.  Each system follows the single
// fgmres exactly otherwise (same restarts, same stopping rule on its own ||rhs||).
// Returns the iterations of both (its[0] for +m, its[1] for -m), -1 without workspace.
static int fgmres_pair(ndtm_ctx* c, MGData* M, const HalfField& rhs, const HalfField* x, double m, double tol,
                       int restart, int maxiter, double* res_out, int* its, hipStream_t st) {
  const size_t n = half_elems(c);
  restart = fgmres_restart_clamp(restart);
  const int per = 2 * restart + 4;
  struct Sys {
    std::vector<HalfField> V, Z;
    HalfField W, te, r;
    std::vector<const void*> Vp, Zp;
    std::vector<std::complex<double>> H, cs, sn, g;
    double sgn = 1, res = 0;
    int total = 0, k = 0;
    bool done = false, in_cycle = false;
  } S[2];
  for (int s = 0; s < 2; ++s) {
    Sys& y = S[s];
    y.sgn = s == 0 ? 1.0 : -1.0;
    size_t j0 = 5 + (size_t)s * per;
    y.V.resize(restart + 1);
    y.Z.resize(restart);
    bool have = true;
    for (int j = 0; j <= restart; ++j) have &= (y.V[j] = region_field(c, j0++, "fp_v" + std::to_string(s) + "_" + std::to_string(j))).v != nullptr;
    for (int j = 0; j < restart; ++j) have &= (y.Z[j] = region_field(c, j0++, "fp_z" + std::to_string(s) + "_" + std::to_string(j))).v != nullptr;
    y.W = region_field(c, j0, "fp_w" + std::to_string(s));
    y.te = region_field(c, j0 + 1, "fp_te" + std::to_string(s));
    y.r = region_field(c, j0 + 2, "fp_r" + std::to_string(s));
    if (!have || !y.W.v || !y.te.v || !y.r.v) {
      res_out[0] = res_out[1] = INFINITY;
      return -1;
    }
    for (auto& f : y.V) y.Vp.push_back(f.v);
    for (auto& f : y.Z) y.Zp.push_back(f.v);
    blas_zero(x[s].v, n * sizeof(double2), st);
  }
  const double bn = std::sqrt(norm2_host(c, (const double2*)rhs.v, n, st));
  if (bn == 0) {
    res_out[0] = res_out[1] = 0;
    its[0] = its[1] = 0;
    return 0;
  }
  // per system: [0, 2 restart) h, [2 restart, 4 restart) second pass, 4 restart: norm2,
  // [6 restart, 8 restart): the update coefficients
  auto dh = [&](int s) { return c->dscal + (size_t)s * 8 * (restart + 1); };
  while (!(S[0].done && S[1].done)) {
    // start a cycle for every system that is not done: r = rhs - A x, V_0 = r / beta
    for (int s = 0; s < 2; ++s) {
      Sys& y = S[s];
      if (y.done) continue;
      if (y.total >= maxiter) {
        y.done = true;
        continue;
      }
      apply_sshift(c, P64, y.r, x[s], y.te, y.sgn * m, st);
      blas_axpby((double2*)y.r.v, make_double2(1, 0), (const double2*)rhs.v, make_double2(-1, 0), n, st);
      const double beta = std::sqrt(norm2_host(c, (const double2*)y.r.v, n, st));
      y.res = beta;
      if (beta <= tol * bn) {
        y.done = true;
        continue;
      }
      blas_axpby((double2*)y.V[0].v, make_double2(1.0 / beta, 0), (const double2*)y.r.v, make_double2(0, 0), n, st);
      y.H.assign((size_t)(restart + 1) * restart, 0.0);
      y.cs.assign(restart, 0.0);
      y.sn.assign(restart, 0.0);
      y.g.assign(restart + 1, 0.0);
      y.g[0] = beta;
      y.k = 0;
      y.in_cycle = true;
    }
    if (S[0].done && S[1].done) break;
    // Arnoldi steps, paired while both systems are inside a cycle
    while (S[0].in_cycle || S[1].in_cycle) {
      if (S[0].in_cycle && S[1].in_cycle) {
        const HalfField rv[2] = {S[0].V[S[0].k], S[1].V[S[1].k]}, zv[2] = {S[0].Z[S[0].k], S[1].Z[S[1].k]};
        if (!mg_cycle_pair(c, M, rv, zv, m, st)) {
          res_out[0] = res_out[1] = INFINITY;
          return -1;
        }
      } else {
        const int s = S[0].in_cycle ? 0 : 1;
        mg_cycle(c, M, S[s].V[S[s].k], S[s].Z[S[s].k], S[s].sgn * m, st);
      }
      for (int s = 0; s < 2; ++s) {
        Sys& y = S[s];
        if (!y.in_cycle) continue;
        const int k = y.k;
        apply_sshift(c, P64, y.W, y.Z[k], y.te, y.sgn * m, st);
        vmultidot(P64, y.Vp.data(), k + 1, y.W.v, n, c->vred, dh(s), st);
        vmulti_axpy_multidot(P64, y.W.v, y.Vp.data(), k + 1, dh(s), n, c->vred, dh(s) + 2 * restart, st);
        vmulti_axpy_norm_dev(P64, y.W.v, y.Vp.data(), k + 1, dh(s) + 2 * restart, n, c->vred, dh(s) + 4 * restart,
                             st);
        vscale_inv_sqrt(P64, y.V[k + 1].v, y.W.v, dh(s) + 4 * restart, n, st);
        (void)hipMemcpyAsync(c->hscal + (size_t)s * 8 * (restart + 1), dh(s), (4 * restart + 1) * sizeof(double),
                             hipMemcpyDeviceToHost, st);
      }
      (void)hipStreamSynchronize(st);
      for (int s = 0; s < 2; ++s) {
        Sys& y = S[s];
        if (!y.in_cycle) continue;
        const int k = y.k;
        const double* hs = c->hscal + (size_t)s * 8 * (restart + 1);
        ++y.total;
        auto Hk = [&](int i) -> std::complex<double>& { return y.H[(size_t)k * (restart + 1) + i]; };
        for (int i = 0; i <= k; ++i)
          Hk(i) = std::complex<double>(hs[2 * i] + hs[2 * restart + 2 * i], hs[2 * i + 1] + hs[2 * restart + 2 * i + 1]);
        const double hn = std::sqrt(std::max(0.0, hs[4 * restart]));
        Hk(k + 1) = hn;
        for (int i = 0; i < k; ++i) {
          const auto t = std::conj(y.cs[i]) * Hk(i) + std::conj(y.sn[i]) * Hk(i + 1);
          Hk(i + 1) = -y.sn[i] * Hk(i) + y.cs[i] * Hk(i + 1);
          Hk(i) = t;
        }
        const double den = std::sqrt(std::norm(Hk(k)) + std::norm(Hk(k + 1)));
        bool stop = false;
        if (!(den > 0) || !std::isfinite(den)) {
          stop = true;  // breakdown: the cycle ends with the columns before this one
        } else {
          y.cs[k] = Hk(k) / den;
          y.sn[k] = Hk(k + 1) / den;
          Hk(k) = den;
          Hk(k + 1) = 0;
          y.g[k + 1] = -y.sn[k] * y.g[k];
          y.g[k] = std::conj(y.cs[k]) * y.g[k];
          y.res = std::abs(y.g[k + 1]);
          y.k = k + 1;
          stop = y.res <= tol * bn || hn == 0 || y.k == restart || y.total >= maxiter;
        }
        if (stop) {
          y.in_cycle = false;
          // x += Z y with y = R^-1 g over the columns of this cycle
          const int kk = y.k;
          std::vector<std::complex<double>> yy(kk);
          for (int i = kk - 1; i >= 0; --i) {
            auto sum = y.g[i];
            for (int j = i + 1; j < kk; ++j) sum -= y.H[(size_t)j * (restart + 1) + i] * yy[j];
            yy[i] = sum / y.H[(size_t)i * (restart + 1) + i];
          }
          std::vector<double> yc(2 * kk);
          for (int i = 0; i < kk; ++i) {
            yc[2 * i] = yy[i].real();
            yc[2 * i + 1] = yy[i].imag();
          }
          if (kk > 0) {
            (void)hipMemcpyAsync(dh(s) + 6 * restart, yc.data(), 2 * kk * sizeof(double), hipMemcpyHostToDevice, st);
            vlincomb_dev(P64, x[s].v, y.Zp.data(), kk, dh(s) + 6 * restart, 1, n, st);
            // the host buffer yc must outlive the copy
            (void)hipStreamSynchronize(st);
          }
        }
      }
    }
  }
  for (int s = 0; s < 2; ++s) {
    res_out[s] = S[s].res / bn;
    its[s] = S[s].total;
  }
  return its[0] + its[1];
}

// upper estimate of the spectrum of Q^2: the context's estimate (largest Ritz value of
// the base system's Lanczos matrix, from a multi-shift solve or ndtm_spectrum_estimate,
// which approaches lambda_max from below) with a 10% margin; without one, 28 (the free
// field's 25.6 with a margin)
static double lambda_max_estimate(const ndtm_ctx* c) { return c->est_lmax > 0 ? 1.1 * c->est_lmax : 28.0; }

// Solves (Q^2 + sigma) x = b for one multigrid shift by case C with FP64 defect
// correction, starting from x (initial guess).  Returns NDTM_OK when the true
// relative residual reaches tol.
static int case_c_solve(ndtm_ctx* c, MGData* M, const HalfField& x, const HalfField& b, double sigma,
                        const ndtm_solve_params* p, double* res_out, int* iters, int* rounds, double* guess_res,
                        hipStream_t st) {
  const size_t n = half_elems(c);
  const double m = std::sqrt(sigma);
  HalfField r = region_field(c, 0, "cc_r"), cr = region_field(c, 1, "cc_c"), ep = region_field(c, 2, "cc_ep"),
            em = region_field(c, 3, "cc_em");
  HalfField xb = region_field(c, 4, "cc_xb");
  if (!r.v || !cr.v || !ep.v || !em.v || !xb.v) return fail(c, NDTM_ENOMEM, "multigrid shift: workspace");
  double res = true_residual(c, x, b, sigma, r, st);
  *guess_res = res;
  const double amp = m / std::sqrt(lambda_max_estimate(c) + sigma);
  int it_total = 0, rd = 0;
  while (res > p->tol && rd < p->max_rounds) {
    blas_copy((double2*)xb.v, (const double2*)x.v, n, st);
    // single-solve tolerance so that one round meets tol after the case-C amplification
    double rho = 0.5 * p->tol / res * amp;
    rho = std::max(1e-14, std::min(rho, p->mg_tol));
    launch_g5t1(c->g, (const double2*)r.v, (double2*)cr.v, st);
    double rp = 0, rm = 0;
    if (mg_pairs_signs(c)) {
      const HalfField xe[2] = {ep, em};
      double rr[2];
      int its[2];
      if (fgmres_pair(c, M, cr, xe, m, rho, p->fgmres_restart, p->fgmres_maxiter, rr, its, st) < 0)
        return fail(c, NDTM_ENOMEM, "multigrid shift: paired FGMRES workspace");
      it_total += its[0] + its[1];
    } else {
      const int ip = fgmres(c, M, cr, ep, +m, rho, p->fgmres_restart, p->fgmres_maxiter, &rp, st);
      if (ip < 0) return fail(c, NDTM_ENOMEM, "multigrid shift: FGMRES workspace");
      const int im = fgmres(c, M, cr, em, -m, rho, p->fgmres_restart, p->fgmres_maxiter, &rm, st);
      if (im < 0) return fail(c, NDTM_ENOMEM, "multigrid shift: FGMRES workspace");
      it_total += ip + im;
    }
    // x += (i/2m)(e_+ - e_-)
    blas_axpy((double2*)x.v, make_double2(0, 0.5 / m), (const double2*)ep.v, n, st);
    blas_axpy((double2*)x.v, make_double2(0, -0.5 / m), (const double2*)em.v, n, st);
    const double prev = res;
    res = true_residual(c, x, b, sigma, r, st);
    ++rd;
    if (!std::isfinite(res) || res >= prev) {
      // the round did not converge far enough to help: keep the previous iterate
      blas_copy((double2*)x.v, (const double2*)xb.v, n, st);
      res = prev;
      break;
    }
  }
  *res_out = res;
  *iters = it_total;
  *rounds = rd;
  return res <= p->tol ? NDTM_OK : NDTM_ENOCONV;
}

bool mg_ready(const ndtm_ctx* c) { return c->mg && c->mg->ready; }
bool mg_pairs_signs(const ndtm_ctx* c) { return c->mg && c->mg->ready && c->mg->prm.pair_signs && c->mg->D64; }

// Lagrange coefficients l_i(target) over the nodes (section 4.2, appendix B).
static std::vector<double> lagrange(const std::vector<double>& nodes, double t) {
  const size_t k = nodes.size();
  std::vector<double> c(k, 1.0);
  for (size_t i = 0; i < k; ++i)
    for (size_t j = 0; j < k; ++j)
      if (j != i) c[i] *= (t - nodes[j]) / (nodes[i] - nodes[j]);
  return c;
}

// First node used for the guess of sig_t from the descending nodes: the
// farthest nodes are dropped while the Lebesgue constant sum |l_i| exceeds 4,
// which bounds the growth of the node residuals in the guess (appendix B).
int guess_first_node(const std::vector<double>& nodes, double sig_t) {
  const int t = (int)nodes.size();
  int first = 0;
  for (;;) {
    if (t - first <= 1) return first;
    std::vector<double> sub(nodes.begin() + first, nodes.end());
    double s = 0;
    for (double v : lagrange(sub, sig_t)) s += std::fabs(v);
    if (s <= 4.0) return first;
    ++first;
  }
}

int guess_mlp(ndtm_ctx* c, const std::vector<double>& nodes, const std::vector<HalfField>& xs, int K, double sig_t,
              const HalfField& b, const std::vector<double>& lag, std::vector<double>* coef, double* pred_mlp,
              double* pred_lag, hipStream_t st);
int guess_projection(ndtm_ctx* c, const std::vector<double>& nodes, const std::vector<HalfField>& xs, double sig_t,
                     const HalfField& b, const HalfField& x, GramCache* gram, double* lag_res, double* proj_res,
                     hipStream_t st);

int solve_mg_shifts(ndtm_ctx* c, const std::vector<double>& sig, int n_mms, int n_pred,
                    std::vector<HalfField>& xs, const HalfField& b, const ndtm_solve_params* p,
                    ndtm_solve_report* rep, hipStream_t st) {
  MGData* M = c->mg;
  if (!M || !M->ready) return fail(c, NDTM_ESTATE, "solve: multigrid shifts need ndtm_mg_setup first");
  // a coarse solve to a tolerance reads its residual on the host: no capture
  M->use_graphs = p->use_graphs != 0 && !(M->prm.coarse_tol > 0.0);
  const int nsh = (int)sig.size();
  const size_t n = half_elems(c);
  int status = NDTM_OK;
  GramCache gram;
  HalfField R = half_field(c, "mg_pred_r", P64), Xp = half_field(c, "mg_pred_x", P64);
  if (n_pred > 0 && (!R.v || !Xp.v)) return fail(c, NDTM_ENOMEM, "solve: predicted-guess workspace");
  for (int t = n_mms; t < nsh; ++t) {
    auto tg0 = std::chrono::steady_clock::now();
    // ---- the shift's own multi-shift iterate (section 4.2, guesses via MMS-CG) ----
    double pred_res = -1;
    if (t < n_mms + n_pred) {
      pred_res = true_residual(c, xs[t], b, sig[t], R, st);
      if (pred_res <= p->tol) {
        // already converged along with the multi-shift solve: no guess, no multigrid work
        rep->guess_kind[t] = NDTM_GUESS_MMS;
        rep->lagrange_res[t] = -1;
        rep->method[t] = 1;
        rep->iterations[t] = 0;
        rep->rounds[t] = 0;
        rep->true_res[t] = rep->guess_res[t] = pred_res;
        rep->t_guess_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - tg0).count();
        continue;
      }
      blas_copy((double2*)Xp.v, (const double2*)xs[t].v, n, st);
    }
    // ---- initial guess from the converged solutions (descending shifts) ----
    const int first = guess_first_node(std::vector<double>(sig.begin(), sig.begin() + t), sig[t]);
    std::vector<double> nodes(sig.begin() + first, sig.begin() + t);
    std::vector<double> lag = lagrange(nodes, sig[t]);
    const int K = t - first;
    std::vector<double> coef = lag;
    rep->guess_kind[t] = p->guess;
    rep->lagrange_res[t] = -1;
    if (p->guess == NDTM_GUESS_MLP) {
      std::vector<HalfField> xk(xs.begin() + first, xs.begin() + t);
      double pm = -1, pl = -1;
      int rc = guess_mlp(c, nodes, xk, K, sig[t], b, lag, &coef, &pm, &pl, st);
      rep->mlp_res[t] = pm;
      rep->lagrange_res[t] = pl;
      if (rc != NDTM_OK || !(pm >= 0) || pm > pl) {
        coef = lag;  // fallback to Lagrange
        rep->guess_kind[t] = NDTM_GUESS_LAGRANGE;
      }
    }
    if (p->guess == NDTM_GUESS_PROJECTION) {
      std::vector<double> all(sig.begin(), sig.begin() + t);
      std::vector<HalfField> xall(xs.begin(), xs.begin() + t);
      double lres = -1, pres = -1;
      const int grc = guess_projection(c, all, xall, sig[t], b, xs[t], &gram, &lres, &pres, st);
      if (grc != NDTM_OK) return grc;
      rep->lagrange_res[t] = lres;
    } else if (p->guess == NDTM_GUESS_ZERO) {
      blas_zero(xs[t].v, n * sizeof(double2), st);
    } else {
      std::vector<const double2*> V(K);
      std::vector<double2> cc(K);
      for (int i = 0; i < K; ++i) {
        V[i] = (const double2*)xs[first + i].v;
        cc[i] = make_double2(coef[i], 0.0);
      }
      blas_lincomb((double2*)xs[t].v, V.data(), cc.data(), K, n, st);
    }
    if (pred_res >= 0) {
      // keep whichever start has the smaller true residual
      const double gres = true_residual(c, xs[t], b, sig[t], R, st);
      if (p->guess == NDTM_GUESS_LAGRANGE) rep->lagrange_res[t] = gres;
      if (!(gres <= pred_res)) {
        blas_copy((double2*)xs[t].v, (const double2*)Xp.v, n, st);
        rep->guess_kind[t] = NDTM_GUESS_MMS;
      }
    }
    auto tg1 = std::chrono::steady_clock::now();
    rep->t_guess_ms += std::chrono::duration<double, std::milli>(tg1 - tg0).count();
    // ---- case C with defect correction ----
    double res = 0, gres = 0;
    int iters = 0, rounds = 0;
    int rc = case_c_solve(c, M, xs[t], b, sig[t], p, &res, &iters, &rounds, &gres, st);
    rep->method[t] = 1;
    rep->iterations[t] = iters;
    rep->rounds[t] = rounds;
    rep->true_res[t] = res;
    rep->guess_res[t] = gres;
    if (rep->lagrange_res[t] < 0 && p->guess == NDTM_GUESS_LAGRANGE) rep->lagrange_res[t] = gres;
    auto tg2 = std::chrono::steady_clock::now();
    rep->t_mg_ms += std::chrono::duration<double, std::milli>(tg2 - tg1).count();
    if (rc == NDTM_ENOMEM) return rc;
    if (rc != NDTM_OK) {
      // the multigrid did not reach the tolerance: finish this shift with FP64 CG
      // from the best iterate, so that every shift still converges
      double pres = 0;
      int pits = 0;
      const int prc = cg_shift(c, xs[t], b, sig[t], p->tol, p->maxiter, &pres, &pits, st);
      rep->method[t] = 2;
      rep->iterations[t] += pits;
      rep->true_res[t] = pres;
      rep->t_mg_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - tg2).count();
      if (prc == NDTM_EBREAKDOWN) return prc;
      if (prc != NDTM_OK) status = prc;
    }
  }
  return status;
}

// ---- setup ----------------------------------------------------------------
static int mg_build(ndtm_ctx* c, const ndtm_mg_params* prm, const void* tv_dev, hipStream_t st) {
  ndtm_mg_free(c);
  // with hipMalloc storage, the solve's phase region (sized to the free memory it found)
  // is given back; the next solve sizes it again around the multigrid data
  if (!c->arena) {
    ws_free_prefix(c, "sv_region");
    ws_free_prefix(c, "cg_ring");
  }
  MGData* M = new MGData();
  c->mg = M;
  M->prm = *prm;
  MGGeom& g = M->g;
  g.T = c->g.T;
  g.Lz = c->g.Lz;
  g.Ly = c->g.Ly;
  g.Lx = c->g.Lx;
  g.bt = prm->block[0];
  g.bz = prm->block[1];
  g.by = prm->block[2];
  g.bx = prm->block[3];
  g.CT = g.T / g.bt;
  g.CZ = g.Lz / g.bz;
  g.CY = g.Ly / g.by;
  g.CX = g.Lx / g.bx;
  g.Vc = g.CT * g.CZ * g.CY * g.CX;
  g.nloc = g.bt * g.bz * g.by * g.bx;
  g.Nv = prm->n_vec;
  g.stride = c->g.stride;
  M->cprec = prm->precision == NDTM_PREC_F64 ? P64 : P32;
  // FP16 storage: the cycle's stencil reads the FP16 links and P is kept in FP16 with
  // one scale per fine site; fields, coarse operator and arithmetic stay FP32
  const bool f16 = prm->precision == NDTM_PREC_F16;
  M->sprec = f16 ? P32H : M->cprec;
  const int Nv = g.Nv, n2 = 2 * Nv;
  const size_t nP = (size_t)g.Vc * g.nloc * 12 * Nv;
  const size_t nD = (size_t)g.Vc * 5 * n2 * n2;  // self block and the four forward hops
  const size_t nB = (size_t)g.Vc * 2 * Nv * Nv;
  M->ncoarse = (size_t)g.Vc * 2 * n2;
  M->P64 = (double2*)mg_alloc(c, M, nP * 16);
  M->D64 = (double2*)mg_alloc(c, M, nD * 16);
  M->Bo64 = (double2*)mg_alloc(c, M, nB * 16);
  if (!M->P64 || !M->D64 || !M->Bo64) return fail(c, NDTM_ENOMEM, "mg_setup: P / coarse operator");
  const size_t nh = half_elems(c);
  if (M->cprec == P64) {
    M->Pc = M->P64;
    M->Dc = M->D64;
    M->Boc = M->Bo64;
  } else {
    M->Pc = mg_alloc(c, M, nP * (f16 ? 4 : 8));
    M->Dc = mg_alloc(c, M, nD * 8);
    M->Boc = mg_alloc(c, M, nB * 8);
    if (f16) M->Psc = (float*)mg_alloc(c, M, (size_t)g.Vc * g.nloc * sizeof(float));
    if (!M->Pc || !M->Dc || !M->Boc || (f16 && !M->Psc)) return fail(c, NDTM_ENOMEM, "mg_setup: cycle copies");
  }
  const int kc = prm->coarse_iters;
  M->cV.resize(kc + 1);
  for (int j = 0; j <= kc; ++j) {
    M->cV[j] = mg_alloc(c, M, M->ncoarse * csz(M->cprec));
    if (!M->cV[j]) return fail(c, NDTM_ENOMEM, "mg_setup: coarse basis");
  }
  M->cW = mg_alloc(c, M, M->ncoarse * csz(M->cprec));
  M->cW2 = mg_alloc(c, M, M->ncoarse * csz(M->cprec));
  M->cR = mg_alloc(c, M, M->ncoarse * csz(M->cprec));
  M->cT = mg_alloc(c, M, M->ncoarse * csz(M->cprec));
  M->cX = mg_alloc(c, M, M->ncoarse * csz(M->cprec));
  M->dH = (double*)mg_alloc(c, M, 2 * (size_t)(kc + 1) * (kc + 1) * sizeof(double));
  M->dsub = (double*)mg_alloc(c, M, (kc + 1) * sizeof(double));
  M->dy = (double*)mg_alloc(c, M, 2 * (kc + 1) * sizeof(double));
  M->dbeta = (double*)mg_alloc(c, M, 8 * sizeof(double));
  M->dtmp = (double*)mg_alloc(c, M, 16 * sizeof(double));
  M->dh2 = (double*)mg_alloc(c, M, 2 * (size_t)(kc + 1) * (kc + 1) * sizeof(double));
  M->dpart = (double*)mg_alloc(c, M, 6 * (size_t)hop_grid(c->g) * sizeof(double));
  if (!M->dpart || !M->dh2 || !M->cW || !M->cW2 || !M->cR || !M->cT || !M->cX || !M->dH || !M->dsub || !M->dy || !M->dbeta || !M->dtmp)
    return fail(c, NDTM_ENOMEM, "mg_setup: coarse workspace");
  M->eo = prm->coarse_eo && g.CT % 2 == 0 && g.CZ % 2 == 0 && g.CY % 2 == 0 && g.CX % 2 == 0;
  if (M->eo) {
    const size_t N = 4 * (size_t)Nv;
    M->einv_chunk = (int)std::max<size_t>(2, std::min<size_t>(g.Vc, ((size_t)1 << 30) / (N * 2 * N * 16) * 2)) & ~1;
    M->cU = mg_alloc(c, M, M->ncoarse * csz(M->cprec));
    M->cT2 = mg_alloc(c, M, M->ncoarse * csz(M->cprec));
    M->cR2 = mg_alloc(c, M, M->ncoarse * csz(M->cprec));
    M->einv_scratch = (double2*)mg_alloc(c, M, (size_t)(M->einv_chunk / 2) * N * 2 * N * 16);
    M->einv_bad = (unsigned*)mg_alloc(c, M, 256);
    if (!M->cU || !M->cT2 || !M->cR2 || !M->einv_scratch || !M->einv_bad)
      return fail(c, NDTM_ENOMEM, "mg_setup: even-odd coarse workspace");
  }
  double2* scratch = (double2*)ws_get(c, "mg_scratch", (size_t)g.Vc * 8 * n2 * n2 * 16);
  if (!scratch) return fail(c, NDTM_ENOMEM, "mg_setup: scratch");
  // P from the vectors currently in M->P64: orthonormalise, Galerkin products, cycle-precision copies
  auto rebuild = [&]() {
    mg_orthonormalize(g, M->P64, st);
    mg_galerkin(g, (const double2*)c->U[P64][0], (const double2*)c->U[P64][1], c->g.antiperiodic, c->op.a, M->P64,
                M->D64, scratch, M->Bo64, st);
    if (c->op.clover)
      mg_galerkin_clover(g, M->P64, (const double*)c->clv_m[0][0], (const double*)c->clv_m[0][1], c->op.a, M->D64, st);
    if (M->cprec != P64) {
      if (M->Psc)
        mg_p_to_half(g, M->P64, M->Pc, M->Psc, st);
      else
        vconvert(P32, M->Pc, P64, M->P64, nP, st);
      vconvert(P32, M->Dc, P64, M->D64, nD, st);
      vconvert(P32, M->Boc, P64, M->Bo64, nB, st);
    }
  };
  if (tv_dev) {
    mg_tv_to_P(g, static_cast<const double2*>(tv_dev), M->P64, st);
    rebuild();
  } else {
    // inverse iteration on the one-flavour operators D_W +- i mubar Gamma5 (doublet kernel at epsbar = 0)
    const int nf = (Nv + 1) / 2;
    std::vector<Full> F(nf);
    for (int i = 0; i < nf; ++i) {
      F[i] = full_field(c, "su_v" + std::to_string(i), P64);
      if (!F[i].base) return fail(c, NDTM_ENOMEM, "mg_setup: test vectors");
      mg_random_fill(g, c->g.vh, (double2*)F[i].e.v, (double2*)F[i].o.v, prm->seed * 1000003ull + i, st);
    }
    Full X = full_field(c, "su_x", P64), R = full_field(c, "su_r", P64), Tt = full_field(c, "su_t", P64);
    if (!X.base || !R.base || !Tt.base) return fail(c, NDTM_ENOMEM, "mg_setup: workspace");
    double* d = c->dscal + 64;
    const OpParams saved = c->op;
    const double a = c->op.a;
    const double eps_setup = prm->setup_nd ? c->epsbar : 0.0;
    auto setup_op = [&]() {
      c->op.epsbar = eps_setup;
      c->op.inv_den = 1.0 / (a * a + c->mubar * c->mubar - eps_setup * eps_setup);
    };
    setup_op();
    // x ~ (D^+ D)^-1 v by CG on the normal equations, D^+ = Gamma5 tau1 D Gamma5 tau1
    // (eq:g5tau1-hermiticity), then v = x / ||x||: inverse iteration towards the
    // smallest singular vectors, which span the near-null space the coarse grid
    // has to represent
    Full Pp = full_field(c, "su_p", P64), W = full_field(c, "su_w", P64);
    if (!Pp.base || !W.base) return fail(c, NDTM_ENOMEM, "mg_setup: workspace");
    const size_t nf2 = 2 * nh;
    // y = Gamma5 tau1 D x (Hermitian), Gamma5 tau1 taken in the stencil's site epilogue;
    // D^+ D = (Gamma5 tau1 D)^2
    auto apply_q = [&](const Full& y, const Full& x) {
      hop(c, P64, EPI_SITE_Q, RED_NONE, 0, x.o, y.e, &x.e, nullptr, 0.0, -0.5, 0, nullptr, st);
      hop(c, P64, EPI_SITE_Q, RED_NONE, 1, x.e, y.o, &x.o, nullptr, 0.0, -0.5, 0, nullptr, st);
    };
    auto apply_normal = [&](const Full& w, const Full& v) {
      apply_q(Tt, v);
      apply_q(w, Tt);
    };
    if (prm->setup_prec == NDTM_PREC_F32) {
      // the same inverse iteration with the CG in FP32 fields and links; the test vectors
      // stay FP64 (each sweep's x is normalised into them)
      Full X3 = full_field(c, "su_x", P32), R3 = full_field(c, "su_r", P32), T3 = full_field(c, "su_t", P32);
      Full P3 = full_field(c, "su_p", P32), W3 = full_field(c, "su_w", P32);
      if (!X3.base || !R3.base || !T3.base || !P3.base || !W3.base) return fail(c, NDTM_ENOMEM, "mg_setup: workspace");
      auto apply_q32 = [&](const Full& y, const Full& x) {
        hop(c, P32, EPI_SITE_Q, RED_NONE, 0, x.o, y.e, &x.e, nullptr, 0.0, -0.5, 0, nullptr, st);
        hop(c, P32, EPI_SITE_Q, RED_NONE, 1, x.e, y.o, &x.o, nullptr, 0.0, -0.5, 0, nullptr, st);
      };
      auto to_host = [&](const double* dv, int k) {
        (void)hipMemcpyAsync(c->hscal, dv, k * sizeof(double), hipMemcpyDeviceToHost, st);
        (void)hipStreamSynchronize(st);
      };
      const size_t n32 = 2 * nh;  // complex elements of a full FP32 field
      for (int sweep = 0; sweep < prm->setup_iters; ++sweep) {
        for (int i = 0; i < nf; ++i) {
          vzero(P32, X3.base, n32, st);
          vconvert_field(P32, R3.base, P64, F[i].base, 2, c->g.vh, c->g.stride, st);
          vconvert(P32, P3.base, P32, R3.base, n32, st);
          vnorm2(P32, R3.base, n32, c->vred, d, st);
          to_host(d, 1);
          double rr = c->hscal[0];
          for (int it = 0; it < prm->setup_smooth && rr > 0; ++it) {
            apply_q32(T3, P3);
            apply_q32(W3, T3);
            vdot(P32, P3.base, W3.base, n32, c->vred, d, st);
            to_host(d, 1);
            const double pw = c->hscal[0];
            if (!(pw > 0)) break;
            const double alpha = rr / pw;
            vaxpby(P32, X3.base, make_double2(alpha, 0), P3.base, make_double2(1, 0), n32, st);
            vaxpby(P32, R3.base, make_double2(-alpha, 0), W3.base, make_double2(1, 0), n32, st);
            vnorm2(P32, R3.base, n32, c->vred, d, st);
            to_host(d, 1);
            const double rn = c->hscal[0];
            vaxpby(P32, P3.base, make_double2(1, 0), R3.base, make_double2(rn / rr, 0), n32, st);
            rr = rn;
          }
          vconvert_field(P64, X.base, P32, X3.base, 2, c->g.vh, c->g.stride, st);
          vnorm2(P64, X.base, nf2, c->vred, d + 6, st);
          vscale_inv_sqrt(P64, F[i].base, X.base, d + 6, nf2, st);
        }
      }
    }
    for (int sweep = 0; sweep < (prm->setup_prec == NDTM_PREC_F32 ? 0 : prm->setup_iters); ++sweep) {
      for (int i = 0; i < nf; ++i) {
        vzero(P64, X.base, nf2, st);
        blas_copy((double2*)R.base, (const double2*)F[i].base, nf2, st);
        blas_copy((double2*)Pp.base, (const double2*)R.base, nf2, st);
        double rr = norm2_host(c, (const double2*)R.base, nf2, st);
        for (int it = 0; it < prm->setup_smooth && rr > 0; ++it) {
          apply_normal(W, Pp);
          const double pw = dot_host(c, (const double2*)Pp.base, (const double2*)W.base, nf2, st).x;
          if (!(pw > 0)) break;
          const double alpha = rr / pw;
          blas_axpy((double2*)X.base, make_double2(alpha, 0), (const double2*)Pp.base, nf2, st);
          blas_axpy((double2*)R.base, make_double2(-alpha, 0), (const double2*)W.base, nf2, st);
          const double rn = norm2_host(c, (const double2*)R.base, nf2, st);
          blas_axpby((double2*)Pp.base, make_double2(1, 0), (const double2*)R.base, make_double2(rn / rr, 0), nf2, st);
          rr = rn;
        }
        vnorm2(P64, X.base, nf2, c->vred, d + 6, st);
        vscale_inv_sqrt(P64, F[i].base, X.base, d + 6, nf2, st);
      }
    }
    std::vector<const double2*> fp(nf);
    for (int i = 0; i < nf; ++i) fp[i] = (const double2*)F[i].base;
    c->op = saved;
    mg_fields_to_P(g, fp.data(), nf, M->P64, st);
    rebuild();
    // refinement: v <- (two-level cycle of the setup operator) v, then rebuild P and D_c
    Full Rc = full_field(c, "su_rc", M->cprec), Zc = full_field(c, "su_zc", M->cprec);
    if (!Rc.base || !Zc.base) return fail(c, NDTM_ENOMEM, "mg_setup: workspace");
    for (int r = 0; r < prm->setup_refine; ++r) {
      setup_op();
      for (int i = 0; i < nf; ++i) {
        vconvert_field(M->cprec, Rc.base, P64, F[i].base, 2, c->g.vh, c->g.stride, st);
        mg_vcycle(c, M, Rc, Zc, 0.0, eps_setup, st);
        vconvert_field(P64, X.base, M->cprec, Zc.base, 2, c->g.vh, c->g.stride, st);
        vnorm2(P64, X.base, 2 * nh, c->vred, d + 6, st);
        vscale_inv_sqrt(P64, F[i].base, X.base, d + 6, 2 * nh, st);
      }
      c->op = saved;
      mg_fields_to_P(g, fp.data(), nf, M->P64, st);
      rebuild();
    }
    c->op = saved;
    NDTM_HIP(c, hipStreamSynchronize(st));
    ws_free_prefix(c, "su_");
  }
  NDTM_HIP(c, hipGetLastError());
  NDTM_HIP(c, hipStreamSynchronize(st));
  // the partial self blocks are only needed during setup
  ws_free_prefix(c, "mg_scratch");
  {
    // cycle buffers exist before any graph capture; the even half of mg_R stays zero
    Full R = full_field(c, "mg_R", M->cprec), Z = full_field(c, "mg_Z", M->cprec);
    Full S = full_field(c, "mg_S", M->cprec), Tt = full_field(c, "mg_T", M->cprec);
    if (!R.base || !Z.base || !S.base || !Tt.base) return fail(c, NDTM_ENOMEM, "mg_setup: cycle workspace");
    vzero(M->cprec, R.base, 2 * nh, st);
    NDTM_HIP(c, hipStreamSynchronize(st));
  }
  if (M->cprec != P64 && !prm->keep_f64) {
    // the FP32 cycle reads only the FP32 copies: give the FP64 ones back
    for (void* q : {(void*)M->P64, (void*)M->D64, (void*)M->Bo64}) {
      M->owned.erase(std::remove(M->owned.begin(), M->owned.end(), q), M->owned.end());
      dev_free(c, q);
    }
    M->P64 = nullptr;
    M->D64 = nullptr;
    M->Bo64 = nullptr;
  }
  M->ready = true;
  return NDTM_OK;
}

}  // namespace ndtm

using namespace ndtm;

extern "C" {

void ndtm_mg_free(ndtm_ctx* c) {
  if (!c || !c->mg) return;
  (void)hipDeviceSynchronize();
  for (auto& g : c->mg->graphs) (void)hipGraphExecDestroy(g.second);
  if (c->mg->cap) (void)hipStreamDestroy(c->mg->cap);
  for (void* p : c->mg->owned) dev_free(c, p);
  delete c->mg;
  c->mg = nullptr;
}

void ndtm_mg_default_params(ndtm_mg_params* p) {
  if (!p) return;
  p->block[0] = p->block[1] = p->block[2] = p->block[3] = 4;
  p->n_vec = 24;
  p->setup_iters = 6;
  p->setup_smooth = 30;
  p->setup_refine = 0;
  p->setup_nd = 1;
  p->smooth_iters = 8;
  p->coarse_iters = 12;
  p->coarse_mu_factor = 1.0;
  p->seed = 32;
  p->precision = NDTM_PREC_F32;
  p->coarse_tol = 0.0;
  p->coarse_cycles = 20;
  p->coarse_eo = 1;
  p->pair_signs = 1;
  p->keep_f64 = 1;
  p->smoother = NDTM_SMOOTH_MR;
  p->sap_mr_iters = 4;
  p->setup_prec = NDTM_PREC_F64;
}

int ndtm_mg_setup(ndtm_ctx* c, const ndtm_mg_params* p, const void* tv, void* stream) {
  if (!c) return NDTM_EINVAL;
  if (!p) return fail(c, NDTM_EINVAL, "mg_setup: null params");
  if (!c->have_gauge || !c->have_params) return fail(c, NDTM_ESTATE, "mg_setup: set_gauge and set_params first");
  const int dims[4] = {c->g.T, c->g.Lz, c->g.Ly, c->g.Lx};
  int nloc = 1;
  for (int i = 0; i < 4; ++i) {
    if (p->block[i] < 1 || dims[i] % p->block[i]) return fail(c, NDTM_EINVAL, "mg_setup: block must divide dims");
    nloc *= p->block[i];
  }
  if (nloc > 256) return fail(c, NDTM_EINVAL, "mg_setup: at most 256 sites per aggregate");
  if (p->n_vec < 2 || p->n_vec > 32 || (p->n_vec & 1))
    return fail(c, NDTM_EINVAL, "mg_setup: n_vec even in [2, 32]");
  if (6 * nloc < p->n_vec) return fail(c, NDTM_EINVAL, "mg_setup: aggregate too small for n_vec vectors");
  if (p->coarse_iters < 1 || p->coarse_iters > 32) return fail(c, NDTM_EINVAL, "mg_setup: coarse_iters in [1, 32]");
  if (!(p->coarse_tol >= 0.0) || (p->coarse_tol > 0.0 && p->coarse_cycles < 1))
    return fail(c, NDTM_EINVAL, "mg_setup: coarse_tol >= 0 and coarse_cycles >= 1");
  if (p->smooth_iters < 0 || p->setup_iters < 0 || p->setup_smooth < 1 || p->setup_refine < 0 || !(p->coarse_mu_factor >= 1.0))
    return fail(c, NDTM_EINVAL, "mg_setup: bad iteration counts or coarse mu factor");
  if (p->precision != NDTM_PREC_F64 && p->precision != NDTM_PREC_F32 && p->precision != NDTM_PREC_F16)
    return fail(c, NDTM_EINVAL, "mg_setup: precision must be F64, F32 or F16");
  if (p->setup_prec != NDTM_PREC_F64 && p->setup_prec != NDTM_PREC_F32)
    return fail(c, NDTM_EINVAL, "mg_setup: setup_prec must be F64 or F32");
  if (p->smoother != NDTM_SMOOTH_MR && p->smoother != NDTM_SMOOTH_SAP)
    return fail(c, NDTM_EINVAL, "mg_setup: smoother must be MR or SAP");
  if (p->smoother == NDTM_SMOOTH_SAP) {
    if (p->sap_mr_iters < 1) return fail(c, NDTM_EINVAL, "mg_setup: sap_mr_iters >= 1");
    if (!sap_block_ok(c->g, p->block))
      return fail(c, NDTM_EINVAL,
                  "mg_setup: SAP needs even aggregate extents, an even number of aggregates per direction "
                  "and 64, 128 or 256 sites per aggregate");
    if (c->op.clover) return fail(c, NDTM_EINVAL, "mg_setup: SAP blocks without the clover term only");
  }
  NDTM_HIP(c, hipSetDevice(c->device));
  const int rc = mg_build(c, p, tv, static_cast<hipStream_t>(stream));
  if (rc != NDTM_OK) ndtm_mg_free(c);
  return rc;
}

long long ndtm_mg_coarse_volume(const ndtm_ctx* c) { return (c && c->mg && c->mg->ready) ? c->mg->g.Vc : 0; }

int ndtm_mg_restrict(ndtm_ctx* c, void* vc, const void* v, void* stream) {
  if (!c) return NDTM_EINVAL;
  if (!c->mg || !c->mg->ready) return fail(c, NDTM_ESTATE, "mg_restrict: no multigrid setup");
  if (!c->mg->P64) return fail(c, NDTM_ESTATE, "mg_restrict: FP64 operators not kept (keep_f64 = 0)");
  if (!vc || !v) return fail(c, NDTM_EINVAL, "mg_restrict: null pointer");
  hipStream_t st = static_cast<hipStream_t>(stream);
  Full F = full_field(c, "ab_f", P64);
  launch_pack_full(c->g, static_cast<const double2*>(v), F.e, F.o, st);
  mg_restrict(P64, c->mg->g, c->mg->P64, nullptr, F.e.v, F.o.v, vc, st);
  NDTM_HIP(c, hipGetLastError());
  return NDTM_OK;
}

int ndtm_mg_prolong(ndtm_ctx* c, void* v, const void* vc, void* stream) {
  if (!c) return NDTM_EINVAL;
  if (!c->mg || !c->mg->ready) return fail(c, NDTM_ESTATE, "mg_prolong: no multigrid setup");
  if (!c->mg->P64) return fail(c, NDTM_ESTATE, "mg_prolong: FP64 operators not kept (keep_f64 = 0)");
  if (!vc || !v) return fail(c, NDTM_EINVAL, "mg_prolong: null pointer");
  hipStream_t st = static_cast<hipStream_t>(stream);
  Full F = full_field(c, "ab_f", P64);
  mg_prolong(P64, c->mg->g, c->mg->P64, nullptr, vc, F.e.v, F.o.v, st);
  launch_unpack_full(c->g, F.e, F.o, static_cast<double2*>(v), st);
  NDTM_HIP(c, hipGetLastError());
  return NDTM_OK;
}

int ndtm_mg_transfer_cycle(ndtm_ctx* c, int dir, void* out, const void* in, void* stream) {
  if (!c) return NDTM_EINVAL;
  if (!c->mg || !c->mg->ready) return fail(c, NDTM_ESTATE, "mg_transfer_cycle: no multigrid setup");
  if (!out || !in || out == in || (dir != 0 && dir != 1))
    return fail(c, NDTM_EINVAL, "mg_transfer_cycle: dir 0 or 1, distinct pointers");
  hipStream_t st = static_cast<hipStream_t>(stream);
  MGData* M = c->mg;
  const int cp = M->cprec;
  Full F64 = full_field(c, "ab_f", P64), Fc = full_field(c, "ab_fc", cp);
  if (!F64.e.v || !Fc.e.v) return fail(c, NDTM_ENOMEM, "mg_transfer_cycle: workspace");
  if (dir == 0) {
    launch_pack_full(c->g, static_cast<const double2*>(in), F64.e, F64.o, st);
    vconvert_field(cp, Fc.base, P64, F64.base, 2, c->g.vh, c->g.stride, st);
    mg_restrict(cp, M->g, M->Pc, M->Psc, Fc.e.v, Fc.o.v, M->cR, st);
    vconvert(P64, out, cp, M->cR, M->ncoarse, st);
  } else {
    vconvert(cp, M->cX, P64, in, M->ncoarse, st);
    mg_prolong(cp, M->g, M->Pc, M->Psc, M->cX, Fc.e.v, Fc.o.v, st);
    vconvert_field(P64, F64.base, cp, Fc.base, 2, c->g.vh, c->g.stride, st);
    launch_unpack_full(c->g, F64.e, F64.o, static_cast<double2*>(out), st);
  }
  NDTM_HIP(c, hipGetLastError());
  return NDTM_OK;
}

int ndtm_mg_cycle(ndtm_ctx* c, void* z, const void* r, double m, void* stream) {
  if (!c) return NDTM_EINVAL;
  if (!c->mg || !c->mg->ready) return fail(c, NDTM_ESTATE, "mg_cycle: no multigrid setup");
  if (!z || !r || z == r) return fail(c, NDTM_EINVAL, "mg_cycle: null or aliased pointer");
  hipStream_t st = static_cast<hipStream_t>(stream);
  MGData* M = c->mg;
  const int cp = M->cprec;
  Full F64 = full_field(c, "ab_f", P64), Rc = full_field(c, "ab_fc", cp), Zc = full_field(c, "ab_fz", cp);
  if (!F64.e.v || !Rc.e.v || !Zc.e.v) return fail(c, NDTM_ENOMEM, "mg_cycle: workspace");
  launch_pack_full(c->g, static_cast<const double2*>(r), F64.e, F64.o, st);
  vconvert_field(cp, Rc.base, P64, F64.base, 2, c->g.vh, c->g.stride, st);
  if (M->eo) (void)einv_for(c, M, m, st);
  mg_vcycle(c, M, Rc, Zc, m, c->epsbar, st);
  vconvert_field(P64, F64.base, cp, Zc.base, 2, c->g.vh, c->g.stride, st);
  launch_unpack_full(c->g, F64.e, F64.o, static_cast<double2*>(z), st);
  NDTM_HIP(c, hipGetLastError());
  return NDTM_OK;
}

int ndtm_mg_smooth(ndtm_ctx* c, void* z, const void* r, double m, void* stream) {
  if (!c) return NDTM_EINVAL;
  if (!c->mg || !c->mg->ready) return fail(c, NDTM_ESTATE, "mg_smooth: no multigrid setup");
  if (!z || !r || z == r) return fail(c, NDTM_EINVAL, "mg_smooth: null or aliased pointer");
  hipStream_t st = static_cast<hipStream_t>(stream);
  MGData* M = c->mg;
  const int cp = M->cprec;
  Full F64 = full_field(c, "ab_f", P64), Rc = full_field(c, "ab_fc", cp), Zc = full_field(c, "ab_fz", cp);
  if (!F64.e.v || !Rc.e.v || !Zc.e.v) return fail(c, NDTM_ENOMEM, "mg_smooth: workspace");
  launch_pack_full(c->g, static_cast<const double2*>(r), F64.e, F64.o, st);
  vconvert_field(cp, Rc.base, P64, F64.base, 2, c->g.vh, c->g.stride, st);
  launch_pack_full(c->g, static_cast<const double2*>(z), F64.e, F64.o, st);
  vconvert_field(cp, Zc.base, P64, F64.base, 2, c->g.vh, c->g.stride, st);
  mg_smooth(c, M, Rc, Zc, m, st);
  vconvert_field(P64, F64.base, cp, Zc.base, 2, c->g.vh, c->g.stride, st);
  launch_unpack_full(c->g, F64.e, F64.o, static_cast<double2*>(z), st);
  NDTM_HIP(c, hipGetLastError());
  return NDTM_OK;
}

int ndtm_mg_coarse_solve(ndtm_ctx* c, void* xc, const void* bc, double m, void* stream) {
  if (!c) return NDTM_EINVAL;
  if (!c->mg || !c->mg->ready) return fail(c, NDTM_ESTATE, "mg_coarse_solve: no multigrid setup");
  if (!xc || !bc || xc == bc) return fail(c, NDTM_EINVAL, "mg_coarse_solve: null or aliased pointer");
  hipStream_t st = static_cast<hipStream_t>(stream);
  MGData* M = c->mg;
  vconvert(M->cprec, M->cR, P64, bc, M->ncoarse, st);
  coarse_solve(c, M, M->cR, M->cX, m, c->epsbar, st);
  vconvert(P64, xc, M->cprec, M->cX, M->ncoarse, st);
  NDTM_HIP(c, hipGetLastError());
  return NDTM_OK;
}

int ndtm_mg_coarse_apply(ndtm_ctx* c, void* yc, const void* xc, double m, void* stream) {
  if (!c) return NDTM_EINVAL;
  if (!c->mg || !c->mg->ready) return fail(c, NDTM_ESTATE, "mg_coarse_apply: no multigrid setup");
  if (!c->mg->P64) return fail(c, NDTM_ESTATE, "mg_coarse_apply: FP64 operators not kept (keep_f64 = 0)");
  if (!yc || !xc || yc == xc) return fail(c, NDTM_EINVAL, "mg_coarse_apply: null or aliased pointer");
  hipStream_t st = static_cast<hipStream_t>(stream);
  mg_coarse_apply(P64, c->mg->g, c->mg->D64, c->mg->Bo64, xc, yc, c->mg->prm.coarse_mu_factor * c->mubar,
                  c->epsbar, m, st);
  NDTM_HIP(c, hipGetLastError());
  return NDTM_OK;
}

int ndtm_mg_coarse_apply_multi(ndtm_ctx* c, void* yc, const void* xc, int k, const double* m, void* stream) {
  if (!c) return NDTM_EINVAL;
  if (!c->mg || !c->mg->ready) return fail(c, NDTM_ESTATE, "mg_coarse_apply_multi: no multigrid setup");
  if (!c->mg->P64) return fail(c, NDTM_ESTATE, "mg_coarse_apply_multi: FP64 operators not kept (keep_f64 = 0)");
  if (!yc || !xc || !m || yc == xc) return fail(c, NDTM_EINVAL, "mg_coarse_apply_multi: null or aliased pointer");
  if (k < 1 || k > kMultiMax) return fail(c, NDTM_EINVAL, "mg_coarse_apply_multi: 1 <= k <= 8");
  hipStream_t st = static_cast<hipStream_t>(stream);
  mg_coarse_apply_multi(c->mg->g, c->mg->D64, c->mg->Bo64, static_cast<const double2*>(xc), static_cast<double2*>(yc),
                        k, m, c->mg->prm.coarse_mu_factor * c->mubar, c->epsbar, st);
  NDTM_HIP(c, hipGetLastError());
  return NDTM_OK;
}


// k coarse systems D'_c(m_r) x_r = b_r at once, FP64 (section 3.2: the coarse
// systems of several shifts and signs share the coarse blocks).  Per system the
// algorithm is the single-system coarse solve's: GMRES(coarse_iters) from zero,
// restarted on the true coarse residual while it is above coarse_tol (at most
// coarse_cycles cycles; one cycle when coarse_tol = 0).  Each Arnoldi step applies
// the coarse operator to the k current basis vectors in one matrix-core launch and
// takes the Gram-Schmidt passes of all k systems in one launch each; the least
// squares and the solution update stay per system.  A system whose
// residual has converged (or turned non-finite) takes no further cycles.
int ndtm_mg_coarse_solve_multi(ndtm_ctx* c, void* xc, const void* bc, int k, const double* m, void* stream) {
  if (!c) return NDTM_EINVAL;
  if (!c->mg || !c->mg->ready) return fail(c, NDTM_ESTATE, "mg_coarse_solve_multi: no multigrid setup");
  if (!c->mg->P64) return fail(c, NDTM_ESTATE, "mg_coarse_solve_multi: FP64 operators not kept (keep_f64 = 0)");
  if (!xc || !bc || !m || xc == bc) return fail(c, NDTM_EINVAL, "mg_coarse_solve_multi: null or aliased pointer");
  if (k < 1 || k > kMultiMax) return fail(c, NDTM_EINVAL, "mg_coarse_solve_multi: 1 <= k <= 8");
  return coarse_solve_multi(c, c->mg, xc, bc, k, m, static_cast<hipStream_t>(stream));
}

}  // extern "C"

namespace ndtm {

int coarse_solve_multi(ndtm_ctx* c, MGData* M, void* xc, const void* bc, int k, const double* m, hipStream_t st) {
  const size_t n = M->ncoarse;
  const int kc = M->prm.coarse_iters;
  const double mubar_c = M->prm.coarse_mu_factor * c->mubar;
  // basis blocks V_j = [k][n] (j = 0..kc), work block W, residual block R; per system
  // scalars: H, H2 (Hessenberg passes), sub, y, beta = {||b||^2, ||r||^2}
  const size_t hsz = 2 * (size_t)(kc + 1) * (kc + 1), per = 2 * hsz + (kc + 1) + 2 * (kc + 1) + 2;
  double2* V = static_cast<double2*>(ws_get(c, "cm_V", (size_t)(kc + 1) * k * n * sizeof(double2)));
  double2* W = static_cast<double2*>(ws_get(c, "cm_W", (size_t)k * n * sizeof(double2)));
  double2* R = static_cast<double2*>(ws_get(c, "cm_R", (size_t)k * n * sizeof(double2)));
  double* sc = static_cast<double*>(ws_get(c, "cm_s", (size_t)k * per * sizeof(double)));
  // per system reduction workspace: counter and the partials of up to kc + 1 complex sums
  const size_t wss = 8 + 2 * (size_t)(kc + 1) * 256;
  double* red = static_cast<double*>(ws_get(c, "cm_red", (size_t)k * wss * sizeof(double)));
  if (!V || !W || !R || !sc || !red) return fail(c, NDTM_ENOMEM, "mg_coarse_solve_multi: workspace");
  const double2* B = static_cast<const double2*>(bc);
  double2* X = static_cast<double2*>(xc);
  auto Hs = [&](int s) { return sc + (size_t)s * per; };
  auto H2s = [&](int s) { return Hs(s) + hsz; };
  auto subs = [&](int s) { return Hs(s) + 2 * hsz; };
  auto ys = [&](int s) { return subs(s) + (kc + 1); };
  auto betas = [&](int s) { return ys(s) + 2 * (kc + 1); };
  auto Vj = [&](int j, int s) { return V + ((size_t)j * k + s) * n; };
  for (int s = 0; s < k; ++s) vnorm2(P64, B + s * n, n, c->vred, betas(s), st);
  std::vector<char> active(k, 1);
  std::vector<double> tol2(k, 0.0);
  const bool restart = M->prm.coarse_tol > 0.0;
  const int cycles = restart ? std::max(1, M->prm.coarse_cycles) : 1;
  for (int cyc = 0; cyc < cycles; ++cyc) {
    for (int s = 0; s < k; ++s)
      if (active[s])
        vscale_inv_sqrt(P64, Vj(0, s), cyc == 0 ? (const void*)(B + s * n) : (const void*)(R + s * n),
                        betas(s) + (cyc == 0 ? 0 : 1), n, st);
    for (int j = 0; j < kc; ++j) {
      mg_coarse_apply_multi(M->g, M->D64, M->Bo64, Vj(j, 0), W, k, m, mubar_c, c->epsbar, st);
      // Gram-Schmidt of all k systems per launch (a finished system's results go unused)
      double* hcol = Hs(0) + 2 * (size_t)j * (kc + 1);
      double* hcol2 = H2s(0) + 2 * (size_t)j * (kc + 1);
      vmultidot_sys(V, (size_t)k * n, j + 1, W, n, k, red, wss, hcol, per, st);
      vmulti_axpy_multidot_sys(W, V, (size_t)k * n, j + 1, hcol, per, n, k, red, wss, hcol2, per, st);
      vmulti_axpy_norm_sys(W, V, (size_t)k * n, j + 1, hcol2, per, n, k, red, wss, subs(0) + j, per, st);
      vscale_inv_sqrt_sys(Vj(j + 1, 0), W, subs(0) + j, per, n, k, st);
    }
    for (int s = 0; s < k; ++s) {
      if (!active[s]) continue;
      std::vector<const void*> Vp(kc);
      for (int i = 0; i < kc; ++i) Vp[i] = Vj(i, s);
      hess_lsq(Hs(s), H2s(s), kc + 1, kc, betas(s) + (cyc == 0 ? 0 : 1), subs(s), ys(s), st);
      vlincomb_dev(P64, X + s * n, Vp.data(), kc, ys(s), cyc > 0, n, st);
    }
    if (!restart || cyc + 1 == cycles) break;
    // true residuals r = b - D' x of all systems (one launch), their norms on the host
    mg_coarse_apply_multi(M->g, M->D64, M->Bo64, X, R, k, m, mubar_c, c->epsbar, st);
    for (int s = 0; s < k; ++s) {
      vaxpby(P64, R + s * n, make_double2(1, 0), B + s * n, make_double2(-1, 0), n, st);  // R = B - D'X
      vnorm2(P64, R + s * n, n, c->vred, betas(s) + 1, st);
    }
    for (int s = 0; s < k; ++s)
      NDTM_HIP(c, hipMemcpyAsync(c->hscal + 2 * s, betas(s), 2 * sizeof(double), hipMemcpyDeviceToHost, st));
    NDTM_HIP(c, hipStreamSynchronize(st));
    int any = 0;
    for (int s = 0; s < k; ++s) {
      const double b2 = c->hscal[2 * s], r2 = c->hscal[2 * s + 1];
      tol2[s] = M->prm.coarse_tol * M->prm.coarse_tol * b2;
      if (active[s] && (!(b2 > 0.0) || !(r2 > tol2[s]) || !std::isfinite(r2))) active[s] = 0;
      any |= active[s];
    }
    if (!any) break;
  }
  NDTM_HIP(c, hipGetLastError());
  return NDTM_OK;
}

}  // namespace ndtm
