// Internal declarations of the ndtm library (not part of the C-ABI).
//
// Internal storage layouts (all per parity, structure of arrays so that a
// wavefront reads 64 consecutive sites of one component):
//   half spinor field: component c = f*12 + spin*3 + colour, site h:
//       element [c * stride + h], 24 components; FP16 fields carry one FP32
//       scale per site, sc[h].
//   links of parity p: element [(mu*9 + row*3 + col) * stride + h] is U_mu(x)
//       of the site x with half index h and parity p.
//   full-lattice vector: even half field followed by the odd half field.
//   stride = vh rounded up to a multiple of 256, plus 256; padding stays zero.
//   FP32 and FP16 fields and links group G = 2 (FP32) or 4 (FP16) components
//   per 16-byte word, so that the stencil loads a flavour's spinor in 6 or 3
//   and a link in 5 or 3 instructions: spinor element (c, h) at
//   ((c/G)*stride + h)*G + c%G (idx32, idx16); link component k < 8 of
//   direction mu at (((8/G)*mu + k/G)*stride + h)*G + k%G and component 8 at
//   (32 + mu)*stride + h (lidx32, lidx16).  FP64 keeps one component per array.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>

#include <cstddef>
#include <cstdint>

namespace ndtm {

constexpr int kBlock = 256;         // threads per block of the lattice kernels
constexpr int kSitesPerBlock = 128; // two threads (one per flavour) per site
constexpr int kMaxShifts = 16;
constexpr int kMaxPartials = 8192;  // reduction partials per scalar

struct Geom {
  int T, Lz, Ly, Lx;
  int vh;      // V/2
  int stride;  // padded vh
  int antiperiodic;
};

// P32H: a stencil precision only, FP32 fields with the FP16 links (the multigrid cycle's
// FP16-storage form); fields and buffers are P64, P32 or P16
enum Prec { P64 = 0, P32 = 1, P16 = 2, P32H = 3 };

__host__ __device__ inline long idx32(int c, int stride, long h) {
  return ((long)(c >> 1) * stride + h) * 2 + (c & 1);
}
__host__ __device__ inline long lidx32(int mu, int k, int stride, long h) {
  return k < 8 ? ((long)(4 * mu + (k >> 1)) * stride + h) * 2 + (k & 1) : (long)(32 + mu) * stride + h;
}
__host__ __device__ inline long idx16(int c, int stride, long h) {
  return ((long)(c >> 2) * stride + h) * 4 + (c & 3);
}
__host__ __device__ inline long lidx16(int mu, int k, int stride, long h) {
  return k < 8 ? ((long)(2 * mu + (k >> 2)) * stride + h) * 4 + (k & 3) : (long)(32 + mu) * stride + h;
}
// element of component c (0..23) at half-site h in a half field of precision prec
__host__ __device__ inline long fidx(int prec, int c, int stride, long h) {
  return prec == P64 ? (long)c * stride + h : prec == P32 ? idx32(c, stride, h) : idx16(c, stride, h);
}

// Epilogues of the hopping kernel.
enum Epi {
  EPI_PLAIN = 0,   // out = H in
  EPI_AINV = 1,    // out = A^-1 H in
  EPI_QHAT = 2,    // out = Gamma5 tau1 (A xs - 1/4 H in)
  EPI_QHAT_SIG = 3,// out = Gamma5 tau1 (A xs - 1/4 H in) + sigma zs
  EPI_SITE = 4,    // out = (A + i ms Gamma5 tau1) xs + hop_coef H in
  EPI_SITE_Q = 5   // out = Gamma5 tau1 [(A + i ms Gamma5 tau1) xs + hop_coef H in]
};
// RED_MR (site epilogue): per block, <out, x> (complex) and ||out||^2 over the block's
// sites, with x the site vector the epilogue reads; stored at partials[q * 2 nblk + b]
// for q = re, im, norm, so that the two parity passes of one full-lattice operator
// (partials offset by nblk for the second) fill one [3][2 nblk] table
enum Red { RED_NONE = 0, RED_NORM = 1, RED_REDOT = 2, RED_MR = 3 };

struct OpParams {
  double a, mubar, epsbar, inv_den;
  int recon12;  // links are SU(3): the stencils rebuild the third row (see u8 for FP64)
  // FP64 SU(3) links in eight parameters per link, per parity (null: the FP64 stencil
  // reads two rows, or nine components)
  const double2* u8[2] = {nullptr, nullptr};
  // optional device flag: a stencil launch returns at once while *skip != 0 (the
  // iterations a solver runs past its done flag before the host sees it)
  const double* skip = nullptr;
  int chunk = 0;    // z extent of the stencil's traversal tile (divides Lz); 0: from the L2 size
  int chunk_y = 0;  // y extent (divides Ly); 0: whole planes
  // clover term of eq:Wilson (0: off).  Site blocks per parity in FP64 ([0]) and FP32 ([1],
  // used by the FP32 and FP16 stencils): M = a + C, 72 component arrays of `stride`
  // entries; the even parity's N and M N, 144 arrays
  int clover = 0;
  const void* clv_m[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
  const void* clv_inv[2] = {nullptr, nullptr};
};

// A precision-tagged half field (device pointers).
struct HalfField {
  void* v = nullptr;    // double2 / float2 / __half2
  float* sc = nullptr;  // per-site scale (FP16 only)
  int prec = P64;
};

// Launch the hopping kernel: out (parity `parity`) from in (parity 1-parity).
// Uo: links of the output parity, Ui: links of the input parity (same precision
// as the fields: FP64 links for P64, FP32 for P32, FP16 for P16).
void launch_hop(int prec, int epi, int red, const Geom& g, int parity, const OpParams& op,
                const void* Uo, const void* Ui, const HalfField& in, const HalfField& out,
                const HalfField* xs, const HalfField* zs, double ms, double hop_coef,
                double sigma, double* partials, hipStream_t st);
int hop_grid(const Geom& g);

// Schwarz alternating procedure: the block solves of one colour (section 3's smoother).
// Blocks of block[] sites tile the lattice with an even number per direction and hold a
// multiple of 32 sites, at most 256 (sap_block_ok).  For every block B of colour `colour`
// (parity of the sum of its block coordinates): mr_iters minimal-residual steps on
// D'_B e = s_B from e = 0, D' = a + i mubar g5 tau3 - epsbar tau1 + hop_coef H (+ i ms g5 tau1
// on odd sites) restricted to B, then z += e.  prec: P64, P32 or P32H (FP32 fields on FP16
// links); U0, U1 the links of the even and odd sites in that stencil's storage.
bool sap_block_ok(const Geom& g, const int block[4]);
void launch_sap_block(int prec, const Geom& g, const int block[4], int colour, int mr_iters, const OpParams& op,
                      const void* U0, const void* U1, const HalfField& s_e, const HalfField& s_o,
                      const HalfField& z_e, const HalfField& z_o, double ms, double hop_coef, hipStream_t st);

// Clover site blocks of one parity from the FP64 links (kern_clover.hip); Ninv only for the
// even parity.  bad counts blocks M^2 + mubar^2 - epsbar^2 that could not be inverted.
void launch_clover_build(const Geom& g, const double2* Ue, const double2* Uo, int parity, double a, double csw,
                         double mubar, double epsbar, double* Mout, double* Ninv, unsigned* bad, hipStream_t st);
void launch_to_f32(const double* src, float* dst, long n, hipStream_t st);

// ---- layout conversion -------------------------------------------------
void launch_pack_gauge(const Geom& g, const double2* U, double2* U64e, double2* U64o, float2* U32e,
                       float2* U32o, __half2* U16e, __half2* U16o, hipStream_t st);
// canonical [V/2][24] (complex128) <-> internal half field (any precision)
// max over all links of |row 2 - conj(row 0 x row 1)| of canonical links (V sites x 4),
// per-block maxima written to part[0..nblk) (nblk = 1024); returns nblk
// FP64 links of one parity in eight parameters (the FP64 stencil's SU(3) form); part:
// per-block minimum of |U01|^2 + |U02|^2 (returns the block count)
int launch_pack_r8(const Geom& g, const double2* U64, double2* U8, double* part, hipStream_t st);
int launch_su3_check(long V, const double2* U, double* part, hipStream_t st);
// streaming reference kernels: kind 0 copy a -> b, 1 read a, 2 write b (bytes multiple of 16)
void launch_stream(int kind, const void* a, void* b, size_t bytes, unsigned* sink, hipStream_t st);
void launch_pack_half(const Geom& g, const double2* canon, const HalfField& f, hipStream_t st);
void launch_unpack_half(const Geom& g, const HalfField& f, double2* canon, hipStream_t st);
// canonical full lattice [V][24] <-> even + odd half fields
void launch_pack_full(const Geom& g, const double2* canon, const HalfField& fe, const HalfField& fo,
                      hipStream_t st);
void launch_unpack_full(const Geom& g, const HalfField& fe, const HalfField& fo, double2* canon,
                        hipStream_t st);
// out = (Gamma5 x tau1) in on FP64 half fields (out must not alias in)
void launch_g5t1(const Geom& g, const double2* in, double2* out, hipStream_t st);
// precision conversion between internal half fields of the same geometry
void launch_convert_half(const Geom& g, const HalfField& src, const HalfField& dst, hipStream_t st);

// ---- BLAS on FP64 complex arrays of n elements ------------------------------
void blas_zero(void* p, size_t bytes, hipStream_t st);
void blas_copy(double2* y, const double2* x, size_t n, hipStream_t st);
void blas_axpy(double2* y, double2 a, const double2* x, size_t n, hipStream_t st);      // y += a x
void blas_xpay(double2* y, const double2* x, double2 a, size_t n, hipStream_t st);      // y = x + a y
void blas_axpby(double2* y, double2 a, const double2* x, double2 b, size_t n, hipStream_t st); // y = a x + b y
void blas_scale(double2* y, double2 a, size_t n, hipStream_t st);
// partial sums, then finalize into dst (device) in a fixed order
int blas_norm2_partials(const double2* x, size_t n, double* partials, hipStream_t st);
int blas_dot_partials(const double2* x, const double2* y, size_t n, double* partials, hipStream_t st);  // <x,y>, 2 doubles
void blas_finalize(const double* partials, int nparts, int width, double* dst, hipStream_t st);
// multi-dot: dst[2i..2i+1] = <V_i, w> for i < k (V_i = base + i*ld)
void blas_multidot(const double2* const* V, int k, const double2* w, size_t n, double* partials,
                   double* dst, hipStream_t st);
// w -= sum_i coef[i] V_i, coef read from device memory (complex, 2 doubles each), scaled by sgn
void blas_multi_axpy_dev(double2* w, const double2* const* V, int k, const double* coef, double sgn,
                         size_t n, hipStream_t st);
// y = sum_i c_i V_i (host coefficients)
void blas_lincomb(double2* y, const double2* const* V, const double2* c, int k, size_t n,
                  hipStream_t st);
// Gram matrix M_ij = <V_i, V_j> (upper triangle incl. diagonal) into dst[(i*k+j)*2]
void blas_gram(const double2* const* V, int k, size_t n, double* partials, double* dst, hipStream_t st);

// ---- MMS-CG -----------------------------------------------------------------
// Device-side scalars in S (layout below).
void mms_scal1(double* S, const double* partials, int nparts, hipStream_t st);
// r_out = r_in - alpha w (r_out may equal r_in), ||r_out||^2 partials; a set *skip
// returns at once
void mms_update_r(const double2* rin, double2* rout, const double2* w, const double* S, size_t n,
                  double* partials, hipStream_t st, const double* skip = nullptr);
// beta, zeta_s, beta_s, freezing; slot >= 0 also records the iteration in slot
// `slot` of the history H (deferred form)
void mms_scal2(double* S, const double* partials, int nparts, int slot, double* H, hipStream_t st);
// p_s, x_s of every active shift in one pass; sb = the base shift (delta 0), whose
// direction is p itself and whose ps[sb] is not used
// it >= 0: returns at once unless iteration it took its scalar step
void mms_update_p(double2* r, double2* p, double2* const* xs, double2* const* ps, int nsh, int sb,
                  const double* S, size_t n, hipStream_t st, int it = -1);
// deferred form: base direction p = r + beta p of iteration it (returns at once unless
// that iteration took its scalar step); the flush of a block of nr iterations that
// began at iteration k0: coefficients from the history (H -> C), then x_s (and, with
// with_p, the block-end p_s) of every shift touched in the block from the residuals
// in slots 0..nr-1 of the ring R (slot j at R + j n)
void mms_update_pbase(const double2* r, double2* p, const double* S, size_t n, int it, hipStream_t st);
// deferred form with the scalar steps of iteration `it` fused: the residual update
// takes step 1 from the stencil partials pst[0..nst) (block 0), writing its own
// partials (not over pst); the base direction update takes step 2 from those (npr of
// them) and records slot `slot` of H (block 0).  The first returns at once while
// *skip is set, and the second whenever the first did.
void mms_update_r_fused(const double2* rin, double2* rout, const double2* w, double* S, size_t n, const double* pst,
                        int nst, double* partials, const double* skip, int it, hipStream_t st);
void mms_update_pbase_fused(const double2* r, double2* p, double* S, size_t n, const double* pr, int npr, int slot,
                            double* H, int it, hipStream_t st);
// mixed form of the two fused passes: FP64 vectors; the stencil's output wq (FP32 or FP16
// words of precision prec, FP16 with the per-site scale wsc) read by the residual pass,
// p's copy in that precision (psc: its FP16 scales) written by the direction pass; nblk:
// blocks of the residual pass (its partial count)
void mms_update_r_fused_mx(int prec, const double2* rin, double2* rout, const void* wq, const float* wsc, double* S,
                           int vh, int stride, const double* pst, int nst, double* partials, int nblk,
                           const double* skip, int it, hipStream_t st);
void mms_update_pbase_fused_mx(int prec, const double2* r, double2* p, void* pq, float* psc, double* S, int vh,
                               int stride, const double* pr, int npr, int slot, double* H, int it, hipStream_t st);
void mms_flush(double2* const* xs, double2* const* ps, int nsh, const double2* R, int nr, int k0, bool with_p,
               const double* S, const double* H, double* C, size_t n, hipStream_t st);
// Deferred multi-shift update: the shifted x_s, p_s are formed once per block of
// at most kMaxDefer iterations from the residuals of that block.  Each iteration
// records per shift (alpha_s or 0, beta_s, zeta_{k+1}, active) in slot k mod m of
// the history H [slot][shift][kHistStride]; the flush turns the block's history
// into the coefficients C [shift][kCoefStride] = [a, e, touched, -, c[m], d[m]].
constexpr int kMaxDefer = 256;
constexpr int kHistStride = 4;
enum MmsCoefIdx { MC_A = 0, MC_E = 1, MC_TOUCHED = 2, MC_C = 4, MC_D = MC_C + kMaxDefer };
constexpr int kCoefStride = MC_D + kMaxDefer;
// Layout of the scalar block S (doubles).
enum MmsIdx {
  MS_RR = 0, MS_PW, MS_ALPHA, MS_ALPHA_PREV, MS_BETA, MS_BB, MS_TOL2, MS_IT, MS_NSH, MS_DONE,
  MS_BREAK, MS_RR_OLD /* ||r_k||^2 of the iteration in progress (step 1 copies it) */,
  MS_GO /* fused deferred form: k + 1 once step 1 of iteration k has run */, MS_HDR = 16,
  // per-shift arrays of length kMaxShifts follow
  MS_ZETA = MS_HDR, MS_ZETA_PREV = MS_ZETA + kMaxShifts, MS_ZETA_NEXT = MS_ZETA_PREV + kMaxShifts,
  MS_ALPHA_S = MS_ZETA_NEXT + kMaxShifts, MS_BETA_S = MS_ALPHA_S + kMaxShifts,
  MS_DELTA = MS_BETA_S + kMaxShifts, MS_ACT = MS_DELTA + kMaxShifts,
  MS_ACT_NEXT = MS_ACT + kMaxShifts, MS_ITERS = MS_ACT_NEXT + kMaxShifts,
  // passenger shifts: iterated along but not waited for (their iterates become
  // initial guesses); the solve is done once every other shift is frozen
  MS_PASS = MS_ITERS + kMaxShifts,
  MS_SIZE = MS_PASS + kMaxShifts
};

}  // namespace ndtm
