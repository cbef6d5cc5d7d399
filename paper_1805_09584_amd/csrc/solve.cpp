// Solve drivers: multi-shift CG (MMS-CG) with device-side recurrences, the
// FP64 true-residual check with single-shift CG polish, and ndtm_solve.
//
// MMS-CG follows the multi-mass-shift scheme the paper takes as its standard
// solver (sections 1 and 4.2): one CG Krylov space built for the smallest shift
// of the set iterates all shifted systems (Q^2 + sigma_s) x_s = b through
// r_s = zeta_s r.  Each iteration is
//   w = (Q^2 + sigma_base) p        two Q applications, Re<p,w> fused in the last epilogue
//   scalars (alpha, zeta_s, alpha_s) one-block kernel
//   r -= alpha w, ||r||^2            fused
//   scalars (beta, beta_s, freeze)   one-block kernel
//   x_s += alpha_s p_s, p_s = zeta_s r + beta_s p_s, p = r + beta p   fused over active shifts
// with a host poll of the done flag every poll_every iterations.  (Taking the
// scalar steps in the last block of the vector kernels instead was slower: the
// device-scope release of every block before the election writes back the
// XCD's L2, which the stencil and the residual update have just filled.)
//
// Deferred form (defer = m >= 2): the last step reads and writes x_s and p_s of
// every active shift each iteration, 4 vectors per shift, more than the stencil
// itself moves.  Over a block of m iterations all shifted vectors stay linear
// combinations of their values at the block start and of the block's residuals
// r_{k+1}, with real coefficients.  The residuals go to m ring slots
// (r_{k+1} -> slot k mod m), the scalar kernel records alpha_s, beta_s, zeta_s of
// each iteration, the base direction p is updated on its own, and once per block
// the coefficients are formed from that record (a backward recurrence) and one
// pass forms x_s (and p_s if more blocks follow) of all shifts from the slots.
// The iterates are those of the direct form up to rounding; the vector traffic
// per iteration drops from (1 + 4 N_active) to about 6 + (m + 3 N_active) / m.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <numeric>

#include "ctx.h"
#include "vec.h"

namespace ndtm {

// unit roundoffs of the mixed form's stencil storages (FP32 mantissa; FP16 relative to
// the per-site scale) and the safety factor of its precision schedule
constexpr double kUnitRoundoff32 = 0x1p-24, kUnitRoundoff16 = 0x1p-11, kRampSafety = 100.0;

static_assert(MS_SIZE + 32 <= kScalN && MS_DONE < 16, "scalar block and poll slots fit the pinned mirror");

namespace {

// Host poll of a solver's done flag without draining the stream: poll j copies
// the flag to pinned memory behind an event and reads the flag of poll j-1,
// whose event has normally completed while the iterations after it were being
// queued.  While it is installed, stencil launches return at once once the flag
// is set, so the iterations queued past convergence cost only their launches.
// With kernel timing on, every poll waits for its own flag instead, so that no
// skipped launch enters the per-class statistics.
// Each poll copies the scalar header S[MS_RR .. MS_DONE], so that the relative
// residual of the base system at the last completed poll is known as well.
struct LaggedPoll {
  static constexpr int kSpan = MS_DONE + 1;
  ndtm_ctx* c;
  hipStream_t st;
  hipEvent_t ev[2] = {nullptr, nullptr};
  double* slot;
  int n = 0;
  const double* S;
  bool lag;
  double rel = INFINITY;  // sqrt(rr / bb) of the base system at the last completed poll
  LaggedPoll(ndtm_ctx* cc, const double* scal, hipStream_t s) : c(cc), st(s), S(scal) {
    const double* done_flag = S + MS_DONE;
    slot = c->hscal + kScalN - 2 * 16;
    for (auto& e : ev) (void)hipEventCreateWithFlags(&e, hipEventDisableTiming);
    lag = c->prof_mask == 0;
    if (lag) c->hop_skip = done_flag;
  }
  ~LaggedPoll() {
    c->hop_skip = nullptr;
    for (auto& e : ev)
      if (e) (void)hipEventDestroy(e);
  }
  // true once a completed poll has seen the flag set
  bool seen(int k) {
    const double* h = slot + 16 * k;
    if (h[MS_BB] > 0) rel = std::sqrt(h[MS_RR] / h[MS_BB]);
    return h[MS_DONE] != 0.0;
  }
  bool done() {
    const int k = n & 1;
    (void)hipMemcpyAsync(slot + 16 * k, S, kSpan * sizeof(double), hipMemcpyDeviceToHost, st);
    (void)hipEventRecord(ev[k], st);
    ++n;
    if (!lag) {
      (void)hipEventSynchronize(ev[k]);
      return seen(k);
    }
    if (n < 2) return false;
    (void)hipEventSynchronize(ev[1 - k]);
    return seen(1 - k);
  }
};

// installs the solve's phase region on the context for the scope of a phase
struct RegionScope {
  ndtm_ctx* c;
  RegionScope(ndtm_ctx* cc, void* region, size_t fields) : c(cc) {
    c->region = region;
    c->region_fields = fields;
  }
  ~RegionScope() {
    c->region = nullptr;
    c->region_fields = 0;
  }
};

}  // namespace

int run_mmscg(ndtm_ctx* c, const std::vector<double>& sigmas, const std::vector<HalfField>& xs,
              const HalfField& b, double tol, int maxiter, int poll_every, int defer, MmsResult* res,
              hipStream_t st, int npass, void* region, const MmsRamp* ramp) {
  const int nsh = (int)sigmas.size();
  const size_t n = half_elems(c);
  const double sig_base = *std::min_element(sigmas.begin(), sigmas.end());
  const int sb = (int)(std::min_element(sigmas.begin(), sigmas.end()) - sigmas.begin());
  HalfField r = half_field(c, "cg_r", P64), p = half_field(c, "cg_p", P64), w = half_field(c, "cg_w", P64);
  HalfField u = half_field(c, "cg_u", P64), te = half_field(c, "cg_te", P64);
  std::vector<double2*> ps(nsh), xv(nsh);
  for (int s = 0; s < nsh; ++s) {
    if (region && s > 0) {
      ps[s] = static_cast<double2*>(region) + (size_t)(s - 1) * n;
    } else {
      HalfField f = half_field(c, "cg_ps" + std::to_string(s), P64);
      if (!f.v) return fail(c, NDTM_ENOMEM, "mmscg: workspace");
      ps[s] = static_cast<double2*>(f.v);
    }
    xv[s] = static_cast<double2*>(xs[s].v);
  }
  if (!r.v || !p.v || !w.v || !u.v || !te.v) return fail(c, NDTM_ENOMEM, "mmscg: workspace");
  if (defer > kMaxDefer) defer = kMaxDefer;
  if (defer >= 2 && !region) {
    // the ring takes at most half of the device memory that is free (or already its own)
    size_t fr = 0, tot = 0;
    (void)hipMemGetInfo(&fr, &tot);
    auto have = c->bufs.find("cg_ring");
    const size_t own = have == c->bufs.end() ? 0 : have->second.bytes;
    const size_t cap = (fr + own) / 2 / (n * sizeof(double2));
    if ((size_t)defer > cap) defer = (int)cap;
  }
  const bool deferred = defer >= 2;
  double2* ring = nullptr;  // defer residual slots, n elements apart
  if (deferred && region) {
    ring = static_cast<double2*>(region) + (size_t)(nsh - 1) * n;
  } else if (deferred) {
    ring = static_cast<double2*>(ws_get(c, "cg_ring", (size_t)defer * n * sizeof(double2)));
    if (!ring) return fail(c, NDTM_ENOMEM, "mmscg: residual slots");
  }
  // mixed form: the stencil's operands in FP32 and FP16 storage
  const bool ramped = ramp && deferred && (ramp->rel32 > 0 || ramp->rel16 > 0);
  HalfField lq[2][4];  // [FP32, FP16][p, w, u, te]
  if (ramped) {
    const char* nm[4] = {"mx_p", "mx_w", "mx_u", "mx_te"};
    for (int q = 0; q < 2; ++q) {
      if ((q == 0 ? ramp->rel32 : ramp->rel16) <= 0) continue;
      for (int k = 0; k < 4; ++k) {
        lq[q][k] = half_field(c, std::string(nm[k]) + (q == 0 ? "32" : "16"), q == 0 ? P32 : P16);
        if (!lq[q][k].v || (q == 1 && !lq[q][k].sc)) return fail(c, NDTM_ENOMEM, "mmscg: workspace");
      }
    }
  }
  int sprec = P64;
  res->it32 = res->it16 = -1;
  const double2* bv = static_cast<const double2*>(b.v);
  blas_copy((double2*)r.v, bv, n, st);
  blas_copy((double2*)p.v, bv, n, st);
  for (int s = 0; s < nsh; ++s) {
    blas_copy(ps[s], bv, n, st);
    blas_zero(xv[s], n * sizeof(double2), st);
  }
  std::vector<double> S(MS_SIZE, 0.0);
  S[MS_ALPHA_PREV] = 1.0;
  S[MS_BETA] = 0.0;
  S[MS_TOL2] = tol * tol;
  S[MS_NSH] = nsh;
  for (int s = 0; s < nsh; ++s) {
    S[MS_ZETA + s] = S[MS_ZETA_PREV + s] = 1.0;
    S[MS_DELTA + s] = sigmas[s] - sig_base;
    S[MS_ACT_NEXT + s] = 1.0;
    S[MS_PASS + s] = s >= nsh - npass ? 1.0 : 0.0;
  }
  NDTM_HIP(c, hipMemcpyAsync(c->mms_S, S.data(), MS_SIZE * sizeof(double), hipMemcpyHostToDevice, st));
  {
    const int g = blas_norm2_partials(bv, n, c->partials, st);
    blas_finalize(c->partials, g, 1, c->dscal, st);
    mms_seed(c->mms_S, c->dscal, st);
  }
  int it = 0;
  if (poll_every < 1) poll_every = 1;
  LaggedPoll poll(c, c->mms_S, st);
  struct Flush {
    int first, nr;
    bool with_p;
  };
  std::vector<Flush> flushes;
  // a flush inside the loop also forms the block-end directions, which the next
  // block starts from; the last one forms the solutions only
  auto flush = [&](int nr, bool with_p) {
    ProfScope pf(c, NDTM_PROF_MMS_UPDATE, 0.0, st);
    mms_flush(xv.data(), ps.data(), nsh, ring, nr, it - nr, with_p, c->mms_S, c->mms_H, c->mms_C, n, st);
    flushes.push_back({it - nr, nr, with_p});
    // the record of the first iterations stays for the spectrum estimate
    const int k0 = it - nr, keep = std::min(nr, kLanczosIters - k0);
    const size_t per = (size_t)kMaxShifts * kHistStride;
    if (keep > 0)
      (void)hipMemcpyAsync(c->mms_L + (size_t)k0 * per, c->mms_H, keep * per * sizeof(double),
                           hipMemcpyDeviceToDevice, st);
  };
  const int hg = hop_grid(c->g);
  const int rg = red_grid(n);
  while (it < maxiter) {
    if (ramped) {
      // the schedule follows the base residual seen by the last completed poll; the
      // direction's copy in the new storage is formed from its FP64 value
      int want = sprec;
      if (ramp->rel16 > 0 && poll.rel <= ramp->rel16)
        want = P16;
      else if (ramp->rel32 > 0 && poll.rel <= ramp->rel32 && sprec == P64)
        want = P32;
      if (want != sprec) {
        const HalfField& pq = lq[want == P16 ? 1 : 0][0];
        launch_convert_half(c->g, p, pq, st);
        (want == P16 ? res->it16 : res->it32) = it;
        sprec = want;
      }
    }
    const HalfField* q = sprec == P64 ? nullptr : lq[sprec == P16 ? 1 : 0];
    // past the done flag the stencil passes and the residual update return at once, and
    // the update kernels of an iteration run only if its scalar step was taken
    if (q)
      apply_qhat2(c, sprec, q[1], q[0], q[2], q[3], sig_base, c->partials, st);
    else
      apply_qhat2(c, P64, w, p, u, te, sig_base, c->partials, st);
    // deferred: r_k is in slot (k-1) mod m (b for k = 0), r_{k+1} goes to slot k mod m
    const int slot = deferred ? it % defer : -1;
    const double2* rin = !deferred ? (const double2*)r.v : it == 0 ? bv : ring + (size_t)((it - 1) % defer) * n;
    double2* rout = deferred ? ring + (size_t)slot * n : (double2*)r.v;
    if (deferred) {
      // the scalar steps ride in the two vector passes; the residual norms go behind
      // the stencil's partials, which the first pass still reads
      double* pr_r = c->partials + hg;
      if (q) {
        // rin, rout FP64 and w in the stencil's storage; p FP64 read and written, its copy written
        const double wb = sprec == P16 ? 100.0 : 192.0;
        {
          ProfScope pr(c, NDTM_PROF_MMS_RESID, (2.0 * 384.0 + wb) * c->g.vh, st);
          mms_update_r_fused_mx(sprec, rin, rout, q[1].v, q[1].sc, c->mms_S, c->g.vh, c->g.stride, c->partials, hg,
                                pr_r, rg, c->hop_skip, it, st);
        }
        ProfScope pu(c, NDTM_PROF_MMS_UPDATE, wb * c->g.vh, st);
        mms_update_pbase_fused_mx(sprec, rout, (double2*)p.v, q[0].v, q[0].sc, c->mms_S, c->g.vh, c->g.stride, pr_r,
                                  rg, slot, c->mms_H, it, st);
      } else {
        {
          ProfScope pr(c, NDTM_PROF_MMS_RESID, 3.0 * 384.0 * c->g.vh, st);
          mms_update_r_fused(rin, rout, (const double2*)w.v, c->mms_S, n, c->partials, hg, pr_r, c->hop_skip, it,
                             st);
        }
        ProfScope pu(c, NDTM_PROF_MMS_UPDATE, 0.0, st);
        mms_update_pbase_fused(rout, (double2*)p.v, c->mms_S, n, pr_r, rg, slot, c->mms_H, it, st);
      }
    } else {
      mms_scal1(c->mms_S, c->partials, hg, st);
      {
        ProfScope pr(c, NDTM_PROF_MMS_RESID, 3.0 * 384.0 * c->g.vh, st);
        mms_update_r(rin, rout, (const double2*)w.v, c->mms_S, n, c->partials, st, c->hop_skip);
      }
      mms_scal2(c->mms_S, c->partials, rg, slot, c->mms_H, st);
      // bytes of this class are added after the loop, once the active counts are known
      ProfScope pu(c, NDTM_PROF_MMS_UPDATE, 0.0, st);
      mms_update_p((double2*)r.v, (double2*)p.v, xv.data(), ps.data(), nsh, sb, c->mms_S, n, st, it);
    }
    ++it;
    if (deferred && it % defer == 0) flush(defer, true);
    if (it % poll_every == 0 && poll.done()) break;
  }
  if (deferred && it % defer != 0) flush(it % defer, false);
  NDTM_HIP(c, hipGetLastError());
  NDTM_HIP(c, hipMemcpyAsync(c->hscal, c->mms_S, MS_SIZE * sizeof(double), hipMemcpyDeviceToHost, st));
  NDTM_HIP(c, hipStreamSynchronize(st));
  res->iterations = (int)c->hscal[MS_IT];
  res->breakdown = c->hscal[MS_BREAK] != 0.0;
  res->iters.resize(nsh);
  for (int s = 0; s < nsh; ++s) res->iters[s] = (int)c->hscal[MS_ITERS + s];
  bool done = c->hscal[MS_DONE] != 0.0;
  if (deferred && res->iterations >= 2 && !res->breakdown) {
    // the base system's alpha_k, beta_k of the first iterations (Lanczos coefficients)
    const int nk = std::min(res->iterations, kLanczosIters);
    std::vector<double> h((size_t)nk * kMaxShifts * kHistStride);
    NDTM_HIP(c, hipMemcpy(h.data(), c->mms_L, h.size() * sizeof(double), hipMemcpyDeviceToHost));
    std::vector<double> al, be;
    for (int k = 0; k < nk; ++k) {
      const double* hk = &h[((size_t)k * kMaxShifts + sb) * kHistStride];
      if (hk[3] == 0.0) break;
      al.push_back(hk[0]);
      be.push_back(hk[1]);
    }
    double lo = 0, hi = 0;
    if (lanczos_extremes(al, be, &lo, &hi) && lo - sig_base > 0) {
      res->lam_lo = lo - sig_base;
      res->lam_hi = hi - sig_base;
    }
  }
  if (deferred && ((c->prof_mask >> NDTM_PROF_MMS_UPDATE) & 1)) {
    // base direction: r read, p read and written per iteration that moves (the launches
    // queued after the done flag return at once); each flush reads its residuals and
    // x_s, p_s of every shift active in its block (shift s is active in iterations
    // 0..iters[s]-1), writes x_s and, inside the loop and while the shift stays
    // active, p_s
    double vecs = 3.0 * res->iterations;
    for (const auto& f : flushes) {
      vecs += f.nr;
      for (int s = 0; s < nsh; ++s) {
        if (res->iters[s] > f.first) vecs += 3.0;
        if (f.with_p && res->iters[s] > f.first + f.nr) vecs += 1.0;
      }
    }
    c->prof_bytes[NDTM_PROF_MMS_UPDATE] += vecs * 384.0 * c->g.vh;
  } else if ((c->prof_mask >> NDTM_PROF_MMS_UPDATE) & 1) {
    // every launch moves r, p (read, p written) and x_s, p_s (read and written) of each active shift;
    // a shift is active in exactly iters[s] launches, and all `it` launches ran
    double active_launches = 0;
    for (int s = 0; s < nsh; ++s) active_launches += res->iters[s];
    // r, p read and p written, 4 vectors per active shift except the base shift (x_s only)
    c->prof_bytes[NDTM_PROF_MMS_UPDATE] += (1.0 * it + 4.0 * active_launches) * 384.0 * c->g.vh;
  }
  if (res->breakdown) return fail(c, NDTM_EBREAKDOWN, "mmscg: breakdown (non-finite or p.Ap <= 0)");
  return done ? NDTM_OK : NDTM_ENOCONV;
}

double true_residual(ndtm_ctx* c, const HalfField& x, const HalfField& b, double sigma, const HalfField& r,
                     hipStream_t st) {
  const size_t n = half_elems(c);
  HalfField u = half_field(c, "tr_u", P64), te = half_field(c, "tr_te", P64);
  // ndtm_solve takes these fields before any work; a caller outside it that runs out of
  // storage gets a non-finite residual (no kernel sees a missing buffer)
  if (!u.v || !te.v || !r.v || !x.v || !b.v) {
    c->err = "true residual: workspace";
    return INFINITY;
  }
  apply_qhat2(c, P64, r, x, u, te, sigma, nullptr, st);
  // r = b - (Q^2 + sigma) x
  blas_axpby((double2*)r.v, make_double2(1, 0), (const double2*)b.v, make_double2(-1, 0), n, st);
  const double rr = norm2_host(c, (const double2*)r.v, n, st);
  const double bb = norm2_host(c, (const double2*)b.v, n, st);
  return std::sqrt(rr / bb);
}

// x += CG((Q^2 + sigma) e = r) until the true residual of x meets tol (up to `rounds` restarts).
static int polish_cg(ndtm_ctx* c, const HalfField& x, const HalfField& b, double sigma, double tol, int maxiter,
                     double* res_out, int* iters_out, hipStream_t st) {
  const size_t n = half_elems(c);
  HalfField r = half_field(c, "pol_r", P64), e = half_field(c, "pol_e", P64);
  if (!r.v || !e.v) return fail(c, NDTM_ENOMEM, "polish: workspace");
  double res = true_residual(c, x, b, sigma, r, st);
  int total = 0;
  for (int round = 0; round < 4 && res > tol; ++round) {
    MmsResult mr;
    std::vector<HalfField> es{e};
    const double inner = std::min(0.5, 0.5 * tol / res);
    int rc = run_mmscg(c, {sigma}, es, r, inner, maxiter, 8, 0, &mr, st);
    total += mr.iterations;
    if (rc != NDTM_OK && rc != NDTM_ENOCONV) return rc;
    blas_axpy((double2*)x.v, make_double2(1, 0), (const double2*)e.v, n, st);
    res = true_residual(c, x, b, sigma, r, st);
  }
  *res_out = res;
  *iters_out = total;
  return res <= tol ? NDTM_OK : NDTM_ENOCONV;
}

int cg_shift(ndtm_ctx* c, const HalfField& x, const HalfField& b, double sigma, double tol, int maxiter,
             double* res_out, int* iters_out, hipStream_t st) {
  HalfField r = half_field(c, "pol_r", P64);
  if (!r.v) return fail(c, NDTM_ENOMEM, "cg shift: workspace");
  if (!std::isfinite(true_residual(c, x, b, sigma, r, st))) blas_zero(x.v, half_elems(c) * sizeof(double2), st);
  return polish_cg(c, x, b, sigma, tol, maxiter, res_out, iters_out, st);
}

// The hybrid part (multigrid shifts) lives in mg.cpp; xs[n_mms .. n_mms+n_pred)
// hold the multi-shift iterates of the passenger shifts.
int solve_mg_shifts(ndtm_ctx* c, const std::vector<double>& sig_desc, int n_mms, int n_pred,
                    std::vector<HalfField>& xs, const HalfField& b, const ndtm_solve_params* p,
                    ndtm_solve_report* rep, hipStream_t st);

}  // namespace ndtm

using namespace ndtm;

extern "C" {

void ndtm_solve_default_params(ndtm_solve_params* p) {
  if (!p) return;
  p->tol = 1e-10;
  p->maxiter = 20000;
  p->n_mmscg = NDTM_MAX_SHIFTS;
  p->guess = NDTM_GUESS_LAGRANGE;
  p->precision = NDTM_PREC_F64;
  p->poll_every = 8;
  p->mg_tol = 0.1;
  p->fgmres_restart = 16;
  p->fgmres_maxiter = 400;
  p->max_rounds = 6;
  p->use_graphs = 1;
  p->mms_defer = 256;
  p->mms_predict = 2;
}

int ndtm_solve(ndtm_ctx* c, void* const* x_dev, const void* b_dev, const ndtm_solve_params* p,
               ndtm_solve_report* rep, void* stream) {
  if (!c) return NDTM_EINVAL;
  if (!x_dev || !b_dev || !p || !rep) return fail(c, NDTM_EINVAL, "solve: null argument");
  if (!c->have_gauge || !c->have_params || c->shifts.empty())
    return fail(c, NDTM_ESTATE, "solve: set_gauge, set_params and set_shifts first");
  if (!(p->tol > 0) || p->maxiter < 1) return fail(c, NDTM_EINVAL, "solve: tol > 0 and maxiter >= 1");
  const int nsh = (int)c->shifts.size();
  for (int i = 0; i < nsh; ++i)
    if (!x_dev[i]) return fail(c, NDTM_EINVAL, "solve: null solution pointer");
  NDTM_HIP(c, hipSetDevice(c->device));
  hipStream_t st = static_cast<hipStream_t>(stream);
  auto t0 = std::chrono::steady_clock::now();
  std::memset(rep, 0, sizeof(*rep));
  rep->n_shifts = nsh;
  rep->mms_it32 = rep->mms_it16 = -1;
  // descending order (section 4.2: solve sigma_1 > sigma_2 > ...)
  std::vector<int> order(nsh);
  std::iota(order.begin(), order.end(), 0);
  std::sort(order.begin(), order.end(), [&](int a, int b) { return c->shifts[a] > c->shifts[b]; });
  std::vector<double> sig(nsh);
  for (int i = 0; i < nsh; ++i) {
    sig[i] = c->shifts[order[i]];
    rep->sigma[i] = sig[i];
    rep->input_index[i] = order[i];
    rep->mlp_res[i] = -1.0;
  }
  const size_t n = half_elems(c);
  HalfField B = half_field(c, "sv_b", P64);
  if (!B.v) return fail(c, NDTM_ENOMEM, "solve: workspace");
  launch_pack_half(c->g, static_cast<const double2*>(b_dev), B, st);
  const double bb = norm2_host(c, (const double2*)B.v, n, st);
  if (!std::isfinite(bb)) {
    rep->status = NDTM_EBREAKDOWN;
    return fail(c, NDTM_EBREAKDOWN, "solve: b is not finite");
  }
  std::vector<HalfField> xs(nsh);
  for (int i = 0; i < nsh; ++i) {
    xs[i] = half_field(c, "sv_x" + std::to_string(i), P64);
    if (!xs[i].v) return fail(c, NDTM_ENOMEM, "solve: workspace");
  }
  // the fixed fields of the later steps (true residuals, CG polish and fallback, the base
  // Krylov vectors) are taken now, so that no step runs out of storage half way
  for (const char* name : {"sv_r", "tr_u", "tr_te", "pol_r", "pol_e", "cg_r", "cg_p", "cg_w", "cg_u", "cg_te", "cg_ps0"})
    if (!half_field(c, name, P64).v) return fail(c, NDTM_ENOMEM, "solve: workspace");
  if (bb == 0.0) {
    for (int i = 0; i < nsh; ++i) blas_zero(xs[i].v, n * sizeof(double2), st);
    for (int i = 0; i < nsh; ++i) launch_unpack_half(c->g, xs[i], static_cast<double2*>(x_dev[order[i]]), st);
    NDTM_HIP(c, hipStreamSynchronize(st));
    return NDTM_OK;
  }
  int n_req = p->n_mmscg;
  if (n_req == NDTM_NMMS_AUTO) {
    // section 4.4: n minimising c_HY(n) = t_CG(m_n^2) + sum_{i>n} t_MG(m_i^2) (eq:costwo)
    n_req = nsh;
    const bool mg = c->mg != nullptr && mg_ready(c);
    if (mg && c->cost_mg_n == 0 && nsh > 1) {
      n_req = nsh - 1;  // measure one multigrid shift first
    } else if (mg && c->est_lmin > 0 && c->cost_iter_n > 0) {
      int n = nsh;
      if (hybrid_choose(nsh, sig.data(), c->est_lmin, c->est_lmax, p->tol, c->cost_iter_ms, c->cost_mg_ms, &n,
                        nullptr) == NDTM_OK)
        n_req = n;
    }
  }
  const int n_mms = std::max(1, std::min(n_req, nsh));
  rep->n_mmscg = n_mms;
  int status = NDTM_OK;
  // ---- MMS-CG for the n_mms largest shifts ----
  // mixed form: the stencil's storage precision follows the base residual (an error of
  // relative size u in the stencil of an iteration whose residual is rho moves the
  // solutions' residuals by about u rho, so the storage with unit roundoff u serves
  // once K u rho <= tol)
  MmsRamp ramp;
  const bool mixed = p->precision == NDTM_PREC_F16;
  if (mixed) {
    ramp.rel32 = p->tol / (kRampSafety * kUnitRoundoff32);
    ramp.rel16 = p->tol / (kRampSafety * kUnitRoundoff16);
  }
  {
    // the first n_pred multigrid shifts ride along as passengers (predicted guesses)
    const int n_pred = std::max(0, std::min(p->mms_predict, nsh - n_mms));
    std::vector<double> s_mms(sig.begin(), sig.begin() + n_mms + n_pred);
    std::vector<HalfField> x_mms(xs.begin(), xs.begin() + n_mms + n_pred);
    // one region serves both phases: shifted directions 1.. and the residual ring, then
    // the multigrid phase's vectors; the ring gets what the region can hold beyond them
    const int n_ps = n_mms + n_pred;
    const size_t fb = n * sizeof(double2);
    const size_t mg_fields = n_mms < nsh ? (size_t)mg_region_fields(p->fgmres_restart, mg_pairs_signs(c)) : 0;
    int defer = std::min(p->mms_defer, kMaxDefer);
    if (defer < 2) defer = 0;
    {
      // the region keeps its size from solve to solve: managed storage gives the ring at
      // most half of the device memory that is free or already the region's; in a caller
      // region it takes the larger of its current block and the largest free one
      const size_t own = ws_bytes(c, "sv_region");
      size_t avail = (c->arena ? std::max(own, dev_largest_free(c)) : (own + dev_largest_free(c)) / 2) / fb;
      // the fields the region holds anyway (its current size, the multigrid phase's) are the ring's too
      avail = std::max(avail, std::max(own / fb, mg_fields));
      const size_t fixed = (size_t)(n_ps - 1);
      if (defer && fixed + defer > avail) defer = avail > fixed + 2 ? (int)(avail - fixed) : 0;
    }
    const size_t fields = std::max(mg_fields, (size_t)(n_ps - 1 + defer));
    void* region = fields ? ws_get(c, "sv_region", fields * fb) : nullptr;
    if (fields && !region) return fail(c, NDTM_ENOMEM, "solve: phase region");
    RegionScope rs(c, region, fields);
    MmsResult mr;
    int rc = run_mmscg(c, s_mms, x_mms, B, 0.5 * p->tol, p->maxiter, p->poll_every, defer, &mr, st, n_pred,
                       region, mixed ? &ramp : nullptr);
    rep->mms_iterations = mr.iterations;
    rep->mms_it32 = mr.it32;
    rep->mms_it16 = mr.it16;
    if (rc != NDTM_OK && rc != NDTM_ENOCONV) {
      rep->status = rc;
      return rc;
    }
    if (mr.lam_lo > 0) {
      c->est_lmin = mr.lam_lo;
      c->est_lmax = mr.lam_hi;
    }
    if (mr.iterations > 0 && !mixed) {
      const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
      c->cost_iter_ms = (c->cost_iter_ms * c->cost_iter_n + ms / mr.iterations) / (c->cost_iter_n + 1);
      ++c->cost_iter_n;
    }
    HalfField R = half_field(c, "sv_r", P64);
    for (int i = 0; i < n_mms; ++i) {
      rep->method[i] = 0;
      rep->iterations[i] = mr.iters[i];
      double res = true_residual(c, xs[i], B, sig[i], R, st);
      if (res > p->tol) {
        int extra = 0;
        int prc = polish_cg(c, xs[i], B, sig[i], p->tol, p->maxiter, &res, &extra, st);
        rep->iterations[i] += extra;
        if (prc != NDTM_OK) status = prc;
      }
      rep->true_res[i] = res;
    }
  }
  auto t1 = std::chrono::steady_clock::now();
  rep->t_mms_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();

  // ---- multigrid (case C) for the remaining shifts ----
  if (n_mms < nsh) {
    const int n_pred = std::max(0, std::min(p->mms_predict, nsh - n_mms));
    const size_t fields = (size_t)mg_region_fields(p->fgmres_restart, mg_pairs_signs(c));
    void* region = ws_get(c, "sv_region", std::max(ws_bytes(c, "sv_region"), fields * n * sizeof(double2)));
    if (!region) return fail(c, NDTM_ENOMEM, "solve: phase region");
    RegionScope rs(c, region, fields);
    const double g0 = rep->t_guess_ms, m0 = rep->t_mg_ms;
    int rc = solve_mg_shifts(c, sig, n_mms, n_pred, xs, B, p, rep, st);
    // multigrid cost per shift, guesses included (a shift whose predicted guess already
    // meets tol costs only its residual check)
    if (rc == NDTM_OK && !mixed) {
      const double ms = (rep->t_guess_ms - g0 + rep->t_mg_ms - m0) / (nsh - n_mms);
      c->cost_mg_ms = (c->cost_mg_ms * c->cost_mg_n + ms) / (c->cost_mg_n + 1);
      ++c->cost_mg_n;
    }
    if (rc != NDTM_OK && status == NDTM_OK) status = rc;

  }
  for (int i = 0; i < nsh; ++i) launch_unpack_half(c->g, xs[i], static_cast<double2*>(x_dev[order[i]]), st);
  NDTM_HIP(c, hipStreamSynchronize(st));
  NDTM_HIP(c, hipGetLastError());
  auto t2 = std::chrono::steady_clock::now();
  rep->t_total_ms = std::chrono::duration<double, std::milli>(t2 - t0).count();
  if ((c->prof_mask >> NDTM_PROF_HOP_F64) & 1) {
    double ms = 0;
    long long nl = 0;
    ndtm_profile_read(c, NDTM_PROF_HOP_F64, &ms, &nl, nullptr, 0);
    rep->hop_ms = ms;
    rep->hop_launches = nl;
  }
  rep->status = status;
  if (status == NDTM_ENOCONV) c->err = "solve: a shift missed the tolerance";
  return status;
}

}  // extern "C"
