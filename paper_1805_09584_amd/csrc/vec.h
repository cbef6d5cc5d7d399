// Vector kernels for FP64/FP32 complex storage (kern_vec.hip) and the
// multigrid kernels (kern_mg.hip).  Internal to the library.
#pragma once

#include "ndtm_internal.h"

namespace ndtm {

// ---- vectors: prec P64 -> double2 storage, P32 -> float2; n complex elements ----
// Reductions (vnorm2, vdot, vmultidot) are single launches: `ws` is a reduction
// workspace [counter (8 doubles, zero between calls)][partials], of at least
// 8 + 2*k*1024 doubles; dst receives the sums (device).  Calls sharing a ws must
// be ordered on one stream.
void vzero(int prec, void* y, size_t n, hipStream_t st);
void vconvert(int prec_dst, void* y, int prec_src, const void* x, size_t n, hipStream_t st);  // flat arrays
// half fields (nhalves consecutive [24][stride] fields) between FP64 and FP32 element orders
void vconvert_field(int prec_dst, void* y, int prec_src, const void* x, int nhalves, int vh, int stride,
                    hipStream_t st);
void vaxpby(int prec, void* y, double2 a, const void* x, double2 b, size_t n, hipStream_t st);   // y = a x + b y
void vaxpy_dev(int prec, void* y, const double* adev, double asgn, const void* x, size_t n,
               hipStream_t st);                                                                  // y += asgn*a x
void vscale_inv_sqrt(int prec, void* y, const void* x, const double* nrm2, size_t n, hipStream_t st);
void vnorm2(int prec, const void* x, size_t n, double* part, double* dst, hipStream_t st);        // dst[0]
void vdot(int prec, const void* x, const void* y, size_t n, double* part, double* dst, hipStream_t st);  // dst[0..1]
void vmultidot(int prec, const void* const* V, int k, const void* w, size_t n, double* part, double* dst,
               hipStream_t st);                                                                  // dst[2j..]
void vlincomb_dev(int prec, void* y, const void* const* V, int k, const double* coef, int accumulate, size_t n,
                  hipStream_t st);
// w -= sum_j coef[j] V_j, then <V_j, w> into dst[2j..2j+1] for j < k (one launch; dst
// must not overlap coef)
void vmulti_axpy_multidot(int prec, void* w, const void* const* V, int k, const double* coef, size_t n, double* part,
                          double* dst, hipStream_t st);
// The Gram-Schmidt steps for k systems in one launch each (FP64; system s = 0..k-1): basis
// vector i of system s at V + i ldv + s n, its vector w + s n, its coefficients coef + s cs,
// its reduction workspace ws + s wss (its own counter and partials: wss >= 8 + 2 cnt * 256),
// its outputs dst + s ds.  Per system the same arithmetic, in the same order, as the
// one-system calls.
void vmultidot_sys(const double2* V, size_t ldv, int cnt, const double2* w, size_t n, int k, double* ws, size_t wss,
                   double* dst, size_t ds, hipStream_t st);
void vmulti_axpy_multidot_sys(double2* w, const double2* V, size_t ldv, int cnt, const double* coef, size_t cs,
                              size_t n, int k, double* ws, size_t wss, double* dst, size_t ds, hipStream_t st);
void vmulti_axpy_norm_sys(double2* w, const double2* V, size_t ldv, int cnt, const double* coef, size_t cs, size_t n,
                          int k, double* ws, size_t wss, double* dst, size_t ds, hipStream_t st);
void vscale_inv_sqrt_sys(double2* y, const double2* x, const double* nrm2, size_t ds, size_t n, int k,
                         hipStream_t st);
// w -= sum_j coef[j] V_j, then ||w||^2 into dst[0] (one launch)
void vmulti_axpy_norm_dev(int prec, void* w, const void* const* V, int k, const double* coef, size_t n, double* ws,
                          double* dst, hipStream_t st);
// minimal-residual step: z += omega s, and s -= omega t if update_s, with omega = <t,s>/<t,t>
// summed from stencil partials part[q * np + i] (q = re, im, norm) by every block
void vmr_update_part(int prec, void* z, void* s, const void* t, const double* part, int np, int update_s, size_t n,
                     hipStream_t st);
void vfinalize(const double* part, int nparts, int width, double* dst, int dst_stride, hipStream_t st);
// least squares min || beta e_1 - H y || for the (m+1) x m Hessenberg matrix with upper part
// H (+ H2 when not null: the two Gram-Schmidt passes; column-major, ldh, complex) and
// subdiagonal sqrt(sub2[j])
void hess_lsq(const double* H, const double* H2, int ldh, int m, const double* beta2, const double* sub2, double* y,
              hipStream_t st);

// ---- multigrid ----
struct MGGeom {
  int T, Lz, Ly, Lx;        // fine dims
  int bt, bz, by, bx;       // aggregate extents
  int CT, CZ, CY, CX;       // coarse dims
  int Vc, nloc, Nv;         // coarse sites, fine sites per aggregate, test vectors
  int stride;               // fine half-field stride
};

// test vectors (canonical complex128 [Nv][V][4][3]) -> P (FP64, [X][l][row][k])
void mg_tv_to_P(const MGGeom& m, const double2* tv, double2* P, hipStream_t st);
// doublet full fields (even half + odd half, FP64; flavour f of field i is test vector 2i+f) -> P
void mg_fields_to_P(const MGGeom& m, const double2* const* fields, int nfields, double2* P, hipStream_t st);
// per aggregate and chirality Gram-Schmidt (classical, applied twice) of P's columns, FP64
void mg_orthonormalize(const MGGeom& m, double2* P, hipStream_t st);
// Galerkin coarse Wilson blocks D[X][b][j][i] (b: 0 self, 1+2mu fwd, 2+2mu bwd), FP64; scratch of
// 8*Vc*(2Nv)^2 complex for the partial self blocks; B_o[X][chi][k][k'] = sum over odd sites P^+ P
void mg_galerkin(const MGGeom& m, const double2* U64e, const double2* U64o, int antiperiodic, double a,
                 const double2* P, double2* D, double2* scratch, double2* Bo, hipStream_t st);
// clover part of the Galerkin self blocks from the fine site blocks M = a + C of both parities
void mg_galerkin_clover(const MGGeom& m, const double2* P, const double* Me, const double* Mo, double a, double2* D,
                        hipStream_t st);
// restrict / prolong between fine full fields (even half at fe, odd half at fo) and coarse [X][2][2Nv];
// Psc (FP32 fields only): P is FP16 with one FP32 scale per fine site (mg_p_to_half)
void mg_restrict(int prec, const MGGeom& m, const void* P, const float* Psc, const void* fe, const void* fo, void* vc,
                 hipStream_t st);
void mg_prolong(int prec, const MGGeom& m, const void* P, const float* Psc, const void* vc, void* fe, void* fo,
                hipStream_t st);
void mg_p_to_half(const MGGeom& m, const void* P64, void* P16, float* Psc, hipStream_t st);
// coarse doublet operator y = D'_c(m) x
// k <= kMultiMax FP64 coarse systems y_r = D'_c(m_r) x_r at once on MFMA; x, y: [k][Vc][2][2Nv]
constexpr int kMultiMax = 8;
void mg_coarse_apply_multi(const MGGeom& g, const double2* D, const double2* Bo, const double2* x, double2* y, int k,
                           const double* m, double mubar_c, double epsbar, hipStream_t st);
// y = D'_c(m) x; with xnorm2 the input is x / sqrt(*xnorm2), and xout (if given) receives that
// scaled input (every coarse site written once)
// par_out >= 0: only the output sites of that coarse parity are written
void mg_coarse_apply(int prec, const MGGeom& g, const void* D, const void* Bo, const void* x, void* y,
                     double mubar_c, double epsbar, double m, hipStream_t st, const double* xnorm2 = nullptr,
                     void* xout = nullptr, int par_out = -1);
// even-odd coarsest level: -A_ee^-1 of the coarse site terms of D'_c(m) for the even sites
// X0 .. X0+count-1 (X0 even; FP64 scratch of count/2 x 4n2 x 8n2 complex), stored at X/2
void mg_einv_build(int prec, const MGGeom& g, int X0, int count, const void* D, const void* Bo, double mubar_c,
                   double epsbar, double m, double2* scratch, void* Einv, unsigned* bad, hipStream_t st);
// out = -A_ee^-1 u on even coarse sites, v (zero when null) on odd ones
void mg_einv_apply(int prec, const MGGeom& g, const void* Einv, const void* u, const void* v, void* out,
                   hipStream_t st);
void mg_coarse_zero_parity(int prec, const MGGeom& g, void* x, int par, hipStream_t st);
// fill a full doublet field (both halves) with complex Gaussian numbers from a counter-based hash
void mg_random_fill(const MGGeom& m, int vh, double2* fe, double2* fo, unsigned long long seed, hipStream_t st);

}  // namespace ndtm
