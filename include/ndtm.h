/*
 * ndtm -- multi-shift solver for the non-degenerate (N_f = 1+1) twisted-mass
 * Wilson operator on one MI355X (gfx950).
 *
 * Problem statement (paper: eq:shifted_linear with the operator of
 * eq:non-degenerate, section 2): for a gauge field U, parameters
 * (kappa, mubar, epsbar) and shifts sigma_i = m_i^2 > 0, compute for one right-hand
 * side b all solutions x_i of
 *
 *     (Q^2 + sigma_i) x_i = b,      Q = (Gamma5 x tau1) S,
 *     S = A - 1/4 H_oe A^-1 H_eo    (even-odd Schur complement on the odd sites),
 *     A = a + i mubar Gamma5 x tau3 - epsbar tau1,   a = 1/(2 kappa),
 *
 * H the Wilson hopping sum of eq:Wilson (clover term off).  The solve uses
 * multi-shift CG for the larger shifts and, for the smallest ones, a two-level
 * aggregation multigrid (section 3) applied through the difference of single
 * solves (eq:lindif) started from interpolated guesses (section 4.2).
 *
 * Conventions shared by every call:
 *  - dims = {T, Lz, Ly, Lx}, all even and >= 2; site s = ((t*Lz+z)*Ly+y)*Lx+x;
 *    parity (t+z+y+x) mod 2; direction mu = 0 time, 1 x, 2 y, 3 z.
 *  - Gauge field: complex128 U[V][4][3][3] (row-major colour matrix, U_mu(x)
 *    connects x to x+mu).  Boundaries periodic; bc_flags bit 0 makes time
 *    antiperiodic for the fermion field.
 *  - Odd-site doublet spinor (the space Q acts on): complex128
 *    [V/2][2 flavour][4 spin][3 colour], half index h = s >> 1 over the odd
 *    sites.  Full-lattice doublet spinor: complex128 [V][2][4][3].
 *  - Gamma matrices in the chiral basis, gamma5 = diag(1,1,-1,-1).
 *
 * Ownership: every pointer argument is owned by the caller; device pointers
 * must be device memory of the context's GPU, 16-byte aligned, and are only
 * used during the call (asynchronously on `stream`, a hipStream_t, NULL for
 * the default stream).  The library never keeps a caller pointer, with one
 * exception: the workspace region of ndtm_set_workspace.  Lattice-sized
 * storage (repacked links, Krylov vectors, multigrid data, network buffers)
 * lives either in that caller-owned region, carved up by the library (no
 * hipMalloc or hipFree after ndtm_set_workspace), or, without a region, in
 * hipMalloc allocations made on demand and freed by ndtm_destroy.  ndtm_create
 * itself allocates a fixed few MB of reduction and scalar buffers and a pinned
 * host mirror.  Call order: create -> (workspace_bytes -> set_workspace) ->
 * set_gauge -> set_params -> set_shifts -> (mg_setup) -> solve / apply.
 *
 * Errors: every call returns an ndtm_status; ndtm_last_error gives a
 * per-context message.  No exception crosses the boundary.  A call made
 * before its prerequisite (apply before set_gauge/set_params) returns
 * NDTM_ESTATE.  Calls are asynchronous on `stream` unless stated otherwise.
 */
#ifndef NDTM_H
#define NDTM_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ndtm_ctx ndtm_ctx;

typedef enum {
  NDTM_OK = 0,
  NDTM_EINVAL = -1,      /* bad argument (dims, sizes, null pointers, op codes) */
  NDTM_ENOMEM = -2,      /* device allocation failed */
  NDTM_ENOCONV = -3,     /* a shift missed the tolerance within the iteration caps */
  NDTM_EBREAKDOWN = -4,  /* non-finite values or a Krylov breakdown */
  NDTM_ESTATE = -5,      /* prerequisite call missing */
  NDTM_EHIP = -6         /* HIP runtime error */
} ndtm_status;

#define NDTM_MAX_SHIFTS 16
#define NDTM_NMMS_AUTO (-1)

/* Precision of the stencil / multigrid inner work. */
enum { NDTM_PREC_F64 = 0, NDTM_PREC_F32 = 1, NDTM_PREC_F16 = 2, NDTM_PREC_F32_H16 = 3 };
/* NDTM_PREC_F32_H16 (ndtm_apply only): FP32 fields and arithmetic on the FP16 links, the
 * stencil of the multigrid cycle in its FP16-storage form */

/* Operators of ndtm_apply. */
enum {
  NDTM_OP_QHAT = 0,       /* y_o = Q x_o                                          */
  NDTM_OP_QHAT2 = 1,      /* y_o = (Q^2 + param) x_o                              */
  NDTM_OP_SHAT_SHIFT = 2, /* y_o = (S + i param Gamma5 tau1) x_o                  */
  NDTM_OP_DFULL = 3,      /* y = (D_ND + i param (Gamma5 x tau1) P_odd) x, full lattice */
  NDTM_OP_HOP_EO = 4,     /* y_e = H_eo x_o (even sites, same half layout)         */
  NDTM_OP_HOP_OE = 5      /* y_o = H_oe x_e                                        */
};

/* Initial-guess modes for the multigrid shifts.  LAGRANGE: interpolation over
 * the converged solutions (section 4.2); MLP: the learned proposer with Lagrange
 * as fallback; PROJECTION: the combination of all converged solutions with the
 * smallest residual, from the Gram matrix of [b, x_1..x_K] and the identity of
 * appendix B, refined on the true residual (a generalisation of section 4.2). */
enum { NDTM_GUESS_ZERO = 0, NDTM_GUESS_LAGRANGE = 1, NDTM_GUESS_MLP = 2, NDTM_GUESS_PROJECTION = 3,
       NDTM_GUESS_MMS = 4 /* report only: the shift's own multi-shift CG iterate (mms_predict) */ };

/* Creates a context on HIP device `device` for the T x L^3 lattice of section 2
 * (dims {T,Lz,Ly,Lx}; the fields of eq:Wilson live on its sites, the even-odd
 * reduction of section 2 splits it by parity).  EINVAL if a dim is odd or < 2, or
 * if V/2 exceeds about 20.6 million sites (the stencil's 32-bit per-field byte
 * offsets; 128 x 64^3 fits); EHIP for a bad device; ENOMEM if its fixed buffers
 * cannot be allocated.  *out receives the context, owned by the caller until
 * ndtm_destroy. */
int ndtm_create(const int dims[4], int bc_flags, int device, ndtm_ctx** out);
void ndtm_destroy(ndtm_ctx* ctx);
const char* ndtm_last_error(const ndtm_ctx* ctx);
/* V/2 (the number of odd sites) and V. */
long long ndtm_half_volume(const ndtm_ctx* ctx);

/* Copies and repacks the gauge field (eq:Wilson's U_mu(x)) from U_dev
 * (complex128 [V][4][3][3], device).  FP32 and FP16 copies for the mixed form
 * are made at the same time.  If every link's third row equals
 * conj(row 0 x row 1) to 1e-14 (SU(3) links), the stencil rebuilds the third
 * row: the FP32 and FP16 stencils load two rows per link, the FP64 stencil loads
 * eight parameters per link (two entries of row 0, one of the first column, two
 * phases) and rebuilds the rest, unless some |U_00|^2 + |U_0j|^2 falls below
 * 1e-20, when it loads two rows as well.  Otherwise all three rows are loaded.
 * Any complex 3x3 links are accepted.  Synchronises the stream; invalidates any multigrid
 * setup. */
int ndtm_set_gauge(ndtm_ctx* ctx, const void* U_dev, void* stream);

/* kappa > 0, a = 1/(2 kappa); requires a^2 + mubar^2 - epsbar^2 != 0 (the
 * closed-form inverse of the site block A).  Invalidates the coarse operator. */
int ndtm_set_params(ndtm_ctx* ctx, double kappa, double mubar, double epsbar);

/* The clover term of eq:Wilson, -c_sw/32 sum_{mu,nu} (gamma_mu gamma_nu) x (Q_mu_nu - Q_nu_mu),
 * with Q_mu_nu(x) the sum of the four plaquettes of the mu-nu plane at x (clover leaf), added
 * to the site term a; c_sw = 0 (the default) switches it off.  The site blocks (a + C per
 * site and chirality, and on the even sites the inverse of the doublet's site block through
 * N = ((a + C)^2 + mubar^2 - epsbar^2)^-1) are built on the device when the gauge field and
 * the parameters are set, and rebuilt by set_gauge / set_params; every operator, solve and
 * multigrid setup then uses them (the Galerkin coarse operator gets P^+ C P).  Invalidates
 * any multigrid setup.  EINVAL for non-finite c_sw or site blocks that cannot be inverted;
 * ENOMEM if the storage (about 3 x 72 x V/2 doubles and as many floats) is not there.
 * Synchronises the device. */
int ndtm_set_clover(ndtm_ctx* ctx, double csw);

/* n in [1, NDTM_MAX_SHIFTS] shifts sigma_i = m_i^2 > 0, any order, distinct
 * (eq:shifted_linear).  The solve orders them descending internally
 * (section 4.2: sigma_1 > sigma_2 > ...). */
int ndtm_set_shifts(ndtm_ctx* ctx, int n, const double* sigma);

/* Applies an operator (NDTM_OP_*) in precision prec (NDTM_PREC_*): Q = Gamma5 tau1 S
 * and Q^2 + sigma on the odd sites (section 2, even-odd reduction, with
 * eq:g5tau1-hermiticity), S + i m Gamma5 tau1 (its shifted Schur form, section 3.1),
 * D_ND + i m (Gamma5 x tau1) P_odd on the full lattice (eq:non-degenerate), or one
 * hopping term H_eo / H_oe of eq:Wilson.  x_dev and y_dev are canonical complex128
 * device arrays (odd-site, even-site or full lattice as the op states), owned by the
 * caller; y_dev must not alias x_dev.  Lower precisions convert x to the internal
 * storage format, apply, and convert back.  EINVAL for null or aliased pointers, an
 * unknown op or precision; ESTATE before set_gauge and set_params; ENOMEM if the
 * workspace cannot hold its five temporary fields.  Asynchronous on stream. */
int ndtm_apply(ndtm_ctx* ctx, int op, int prec, void* y_dev, const void* x_dev,
               double param, void* stream);

/* ndtm_apply without device allocation, for callers that cannot allocate (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).  FP64 only,
 * same operators and layouts as ndtm_apply, same results bit for bit.  Its four
 * internal half fields live in a fixed device array of ndtm_apply_noalloc_max_bytes()
 * bytes (128 MiB) that each GPU the library runs on holds until the process ends; a
 * lattice needing more (4 x 24 x (V/2 rounded up to 256, + 256) x 16 bytes, about
 * V/2 <= 87,000 sites) is refused with NDTM_EINVAL.  The array is shared by all calls
 * on one GPU and keeps the last call's contents: calls that overlap on one GPU (other
 * streams or threads) race and must be serialised by the caller.  No hipMalloc, hipFree
 * or other allocating call is made.  Errors as ndtm_apply; NDTM_EHIP if the array's
 * device address could not be resolved when the context was created. */
int ndtm_apply_noalloc(ndtm_ctx* ctx, int op, void* y_dev, const void* x_dev, double param, void* stream);
size_t ndtm_apply_noalloc_max_bytes(void);

/* ---- multigrid (section 3, section 3.2) -------------------------------- */
typedef struct {
  int block[4];        /* aggregate extents {bt,bz,by,bx}; each divides the dim */
  int n_vec;           /* test vectors N_v (<= 32); coarse dof per flavour = 2 N_v */
  int setup_iters;     /* inverse-iteration sweeps building the test vectors */
  int setup_smooth;    /* CG steps on the normal equations D^+ D x = v per
                          inverse-iteration sweep (D^+ = Gamma5 tau1 D Gamma5 tau1) */
  int setup_refine;    /* refinement sweeps: each replaces every test vector by one
                          two-level cycle applied to it, then rebuilds P and D_c */
  int setup_nd;        /* 0: iterate the one-flavour operators D_W +- i mubar Gamma5
                          (section 3.2's reuse of the twisted-mass setup); 1: iterate the
                          doublet operator D_ND itself and use both flavour components */
  int smooth_iters;    /* post-smoothing iterations per cycle (0 pre; default 8): minimal-residual
                          steps, or SAP sweeps (see smoother) */
  int coarse_iters;    /* GMRES iterations of the coarse solve per cycle (default 12) */
  double coarse_mu_factor; /* d >= 1 scaling mubar on the coarse grid (d = 1 default) */
  unsigned long long seed; /* seed of the random initial test vectors */
  int precision;       /* the cycle's precision: NDTM_PREC_F64; NDTM_PREC_F32 (FP32 P, coarse
                          operator, fields and stencil); NDTM_PREC_F16 (FP16 storage: P in FP16
                          with one FP32 scale per fine site and the smoother's stencil on the
                          FP16 links, FP32 fields, coarse operator and arithmetic) */
  double coarse_tol;   /* 0: the coarse solve is coarse_iters GMRES iterations from zero (a fixed
                          sequence, which the cycle graphs capture).  > 0: GMRES(coarse_iters)
                          restarted on the true coarse residual until it is below coarse_tol
                          relative (section 3: the coarse system solved to a loose tolerance);
                          the host reads the residual after each cycle, so no graphs */
  int coarse_cycles;   /* restart cap of the coarse solve when coarse_tol > 0 (>= 1) */
  int coarse_eo;       /* 1 (default): the coarse solve runs GMRES on the odd Schur complement of
                          the coarse operator (section 3: even-odd reduction on the coarsest
                          level), with the even site terms inverted per value of m (cached);
                          needs even coarse extents, else (or 0) GMRES on the full coarse system */
  int keep_f64;        /* 1 (default): keep the FP64 P and coarse blocks, which the FP64 calls
                          ndtm_mg_restrict/prolong/coarse_apply(_multi)/coarse_solve_multi
                          use; 0 with an FP32 cycle: free them after the setup (those
                          calls then return NDTM_ESTATE), about 2/3 of the multigrid storage */
  int pair_signs;      /* 1 (default): case C runs the FGMRES solves of +m and -m in lock-step, and
                          each of their cycles solves the two coarse systems D'_c(+m), D'_c(-m)
                          together by the batched coarse solve on the matrix cores (section 3.2:
                          several coarse systems share the coarse blocks; FP64 coarse GMRES on the
                          full coarse system).  Needs the FP64 coarse blocks (keep_f64 = 1); without
                          them, or with 0, one sign after the other */
  int smoother;        /* NDTM_SMOOTH_MR (default): smooth_iters minimal-residual steps on the whole
                          lattice.  NDTM_SMOOTH_SAP: smooth_iters sweeps of the Schwarz alternating
                          procedure (section 3, eq:error_propagation's smoother M): the aggregates
                          as blocks in two colours, each block system D'_B e = s_B solved by
                          sap_mr_iters minimal-residual steps, the residual formed again after
                          each colour.  SAP needs even aggregate extents, an even number of
                          aggregates per direction, 64, 128 or 256 sites per aggregate, and no
                          clover term */
  int sap_mr_iters;    /* minimal-residual steps per block solve of SAP (default 4, >= 1) */
  int setup_prec;      /* NDTM_PREC_F64 (default): the inverse iteration's CG in FP64;
                          NDTM_PREC_F32: in FP32 fields and links (about half the setup time;
                          the test vectors, P and the coarse operator are still formed in FP64) */
} ndtm_mg_params;

#define NDTM_SMOOTH_MR 0
#define NDTM_SMOOTH_SAP 1

/* Fills *p with the defaults (4^4 aggregates, 24 vectors, ...). */
void ndtm_mg_default_params(ndtm_mg_params* p);

/* Builds P and the coarse operator.  If test_vectors_dev is not NULL it
 * supplies the N_v test vectors (complex128 [N_v][V][4][3], device) and the
 * inverse iteration is skipped; otherwise they come from inverse iteration on
 * the single-flavour twisted-mass operator D_W + i mubar Gamma5 (section 3.2:
 * the setup of the one-flavour operator is reused for the doublet).  Per
 * aggregate and chirality the vectors are orthonormalised (Gram-Schmidt in
 * vector order).  Synchronises the stream. */
int ndtm_mg_setup(ndtm_ctx* ctx, const ndtm_mg_params* p, const void* test_vectors_dev, void* stream);

/* z = one two-level cycle for D'(m) z = r, the preconditioner of case C's FGMRES
 * (section 3, eq:error_propagation with no pre-smoothing): the coarse correction
 * (P x I2) D'_c(m)^-1 (P x I2)^dag r, the coarse system solved as the setup chose
 * (coarse_iters GMRES iterations, or restarted to coarse_tol), then the post-smoother,
 * in the cycle's precision.  D'(m) = D_ND + i m (Gamma5 x tau1) on odd sites.  z_dev,
 * r_dev: full-lattice doublets, complex128 [V][2 flavour][4 spin][3 colour] canonical
 * order, device, distinct; z_dev is written.  ESTATE without a multigrid setup. */
int ndtm_mg_cycle(ndtm_ctx* ctx, void* z_dev, const void* r_dev, double m, void* stream);

/* z <- the cycle's post-smoother applied to D'(m) z = r (section 3: the smoother M of
 * eq:error_propagation, started from z as the cycle starts it from the coarse correction),
 * with D'(m) = D_ND + i m (Gamma5 x tau1) on odd sites: smooth_iters minimal-residual steps
 * or SAP sweeps as the setup chose, in the cycle's precision.  z_dev, r_dev: full-lattice
 * doublets, complex128 [V][2 flavour][4 spin][3 colour] canonical order, device, distinct;
 * z_dev is read and overwritten.  ESTATE without a multigrid setup. */
int ndtm_mg_smooth(ndtm_ctx* ctx, void* z_dev, const void* r_dev, double m, void* stream);

/* Coarse vector layout: complex128 [Vc][2 flavour][2 N_v], dof = chi*N_v + k. */
long long ndtm_mg_coarse_volume(const ndtm_ctx* ctx);
/* vc = (P x I2)^dag v; v full-lattice canonical doublet. */
int ndtm_mg_restrict(ndtm_ctx* ctx, void* vc_dev, const void* v_dev, void* stream);
/* v = (P x I2) vc. */
int ndtm_mg_prolong(ndtm_ctx* ctx, void* v_dev, const void* vc_dev, void* stream);
/* The restriction (dir 0: out = (P x I2)^dag in, in full-lattice canonical, out coarse) or
 * prolongation (dir 1: out = (P x I2) in) as the cycle runs it: the input is rounded to
 * the cycle's field precision, P read in the cycle's storage (FP64, FP32, or FP16 with
 * per-site scales), the output returned in complex128.  Works without the FP64 copies
 * (keep_f64 = 0).  ESTATE without a setup; EINVAL for another dir or equal pointers. */
int ndtm_mg_transfer_cycle(ndtm_ctx* ctx, int dir, void* out_dev, const void* in_dev, void* stream);
/* yc = D'_c(m) xc = (D_W,c x I2 + i d mubar Gamma5_c x tau3 - epsbar tau1
 *                     + i m C_o x tau1) xc   (eq:non-degenerate_coarse). */
int ndtm_mg_coarse_apply(ndtm_ctx* ctx, void* yc_dev, const void* xc_dev, double m, void* stream);

/* y_r = D'_c(m_r) x_r for k systems at once (1 <= k <= 8), FP64: xc, yc hold the k
 * coarse vectors back to back, complex128 [k][Vc][2][2 N_v], not aliased; m: k host
 * doubles.  The coarse blocks are shared by the systems and both flavours, so the
 * products form one dense complex matrix product per coarse site, taken on the
 * matrix cores (v_mfma_f64_16x16x4f64): the blocks are read once for all k systems
 * (section 3.2, eq:non-degenerate_coarse; batching the coarse systems of the shifts
 * and signs).  Same result as k calls of ndtm_mg_coarse_apply up to rounding. */
int ndtm_mg_coarse_apply_multi(ndtm_ctx* ctx, void* yc_dev, const void* xc_dev, int k, const double* m,
                               void* stream);

/* xc ~ D'_c(m)^-1 bc by the coarse solver the cycle uses, in the cycle precision:
 * coarse_iters GMRES iterations from zero, restarted while the relative residual
 * is above coarse_tol (when that is > 0, at most coarse_cycles cycles). */
int ndtm_mg_coarse_solve(ndtm_ctx* ctx, void* xc_dev, const void* bc_dev, double m, void* stream);

/* x_r ~ D'_c(m_r)^-1 b_r for k systems at once (1 <= k <= 8), FP64, by the same
 * algorithm as ndtm_mg_coarse_solve per system: coarse_iters GMRES iterations from
 * zero, restarted on the true coarse residual while it is above coarse_tol (when
 * that is > 0, at most coarse_cycles cycles; a converged system stops).  Each
 * Arnoldi step applies the coarse operator to the k basis vectors in one
 * matrix-core launch (as ndtm_mg_coarse_apply_multi): the coarse blocks are read
 * once for all systems (section 3.2; the coarse systems of the shifts and signs).
 * xc, bc: the k coarse vectors back to back, complex128 [k][Vc][2][2 N_v], device,
 * not aliased; m: k host doubles.  The library keeps its workspace (about
 * (coarse_iters + 3) k coarse vectors).  Same result as k calls of
 * ndtm_mg_coarse_solve with an FP64 cycle (precision NDTM_PREC_F64) up to rounding.
 * Errors: NDTM_ESTATE without a multigrid setup, NDTM_EINVAL for k out of range or
 * null or aliased pointers, NDTM_ENOMEM if the workspace cannot be allocated. */
int ndtm_mg_coarse_solve_multi(ndtm_ctx* ctx, void* xc_dev, const void* bc_dev, int k, const double* m,
                               void* stream);

/* ---- solve ------------------------------------------------------------- */
typedef struct {
  double tol;          /* target true relative residual per shift (1e-10) */
  int maxiter;         /* MMS-CG iteration cap */
  int n_mmscg;         /* shifts solved by MMS-CG (the largest ones); the
                          rest go to the multigrid; >= number of shifts means
                          plain MMS-CG for all.  NDTM_NMMS_AUTO: chosen by the
                          cost model of section 4.4 (eq:costwo, as ndtm_hybrid_split)
                          from this context's spectrum estimate of Q^2 and its measured
                          costs of one multi-shift iteration and of one multigrid shift
                          (the mean over earlier solves); while no multigrid shift has
                          been timed on a context with a multigrid setup, one shift goes
                          to the multigrid so that its cost is measured; without a
                          setup or a spectrum estimate, all shifts go to MMS-CG */
  int guess;           /* NDTM_GUESS_* for the multigrid shifts */
  int precision;       /* NDTM_PREC_F64: FP64 throughout.  NDTM_PREC_F16: mixed form, the
                          multi-shift CG keeps its FP64 vectors, residual slots, solutions
                          and scalar recurrences, but its stencil moves to lower-precision
                          operand storage as the base residual falls: FP32 once
                          ||r||/||b|| <= tol / (K u32) and FP16 (one FP32 scale per site,
                          FP32 arithmetic) once ||r||/||b|| <= tol / (K u16), with u32, u16
                          the storages' unit roundoffs and K a safety factor; each stencil
                          error then enters the solutions scaled by the residual of its
                          iteration, below tol.  Every shift is checked by its FP64 true
                          residual and finished by FP64 CG if it misses.  Needs the
                          deferred recurrences (mms_defer >= 2; otherwise FP64).  Other
                          values select the FP64 form. */
  int poll_every;      /* MMS-CG iterations between host convergence polls */
  double mg_tol;       /* cap on the relative residual of each single (Q +- i m) solve; each
                          round tightens it so that the squared system meets tol */
  int fgmres_restart;  /* outer FGMRES restart length */
  int fgmres_maxiter;  /* outer FGMRES iteration cap per single solve */
  int max_rounds;      /* FP64 defect-correction rounds per multigrid shift */
  int use_graphs;      /* 1: replay the multigrid cycle from a captured HIP graph (one per
                          shift sign, cached until the next setup); 0: launch eagerly */
  int mms_defer;       /* FP64 MMS-CG: 2..256 forms the shifted solutions (and, between
                          blocks, directions) once per block of this many iterations from
                          the block's residuals, kept in as many extra half fields (same
                          iterates up to rounding, far fewer vector passes); 0 or 1 updates
                          them every iteration.  Clamped to 256 and so that the residual
                          slots take at most half of the free device memory */
  int mms_predict;     /* FP64 hybrid: the first this many multigrid shifts ride along in the
                          multi-shift CG without being waited for (section 4.2, initial guesses
                          via MMS-CG); each starts from its multi-shift iterate when that has
                          the smaller true residual than the `guess` proposal (report
                          guess_kind NDTM_GUESS_MMS), and needs no multigrid work when the
                          iterate already meets tol.  0 disables */
} ndtm_solve_params;

void ndtm_solve_default_params(ndtm_solve_params* p);

typedef struct {
  int status;
  int n_shifts;
  int mms_iterations;               /* iterations of the shared Krylov space */
  double sigma[NDTM_MAX_SHIFTS];    /* in solve order (descending) */
  int input_index[NDTM_MAX_SHIFTS]; /* position of this shift in set_shifts */
  int method[NDTM_MAX_SHIFTS];      /* 0 = MMS-CG, 1 = multigrid case C, 2 = multigrid
                                       did not converge, finished by FP64 CG */
  int iterations[NDTM_MAX_SHIFTS];  /* MMS-CG: iteration when frozen; MG: outer iterations */
  int rounds[NDTM_MAX_SHIFTS];      /* MG: defect-correction rounds */
  double true_res[NDTM_MAX_SHIFTS]; /* ||b - (Q^2+sigma) x|| / ||b||, FP64 */
  double guess_res[NDTM_MAX_SHIFTS];/* relative residual of the chosen initial guess */
  double lagrange_res[NDTM_MAX_SHIFTS]; /* predicted residual of the Lagrange guess */
  double mlp_res[NDTM_MAX_SHIFTS];  /* predicted residual of the network's guess (or -1) */
  int guess_kind[NDTM_MAX_SHIFTS];  /* NDTM_GUESS_* actually used */
  double t_mms_ms, t_guess_ms, t_mg_ms, t_total_ms;
  double hop_ms;                    /* summed duration of FP64 stencil launches (if profiling) */
  long long hop_launches;
  int n_mmscg;                      /* shifts the multi-shift CG solved (the choice of NDTM_NMMS_AUTO) */
  int mms_it32, mms_it16;           /* mixed form: first multi-shift iteration whose stencil ran on
                                       FP32 / FP16 storage (-1: none) */
} ndtm_solve_report;

/* Solves all shifts for one b.  x_dev[i] receives the solution of the i-th
 * shift as given to ndtm_set_shifts (odd-site canonical, device); b_dev is
 * odd-site canonical.  Synchronises the stream at the end to fill the report.
 * Returns ENOCONV (solutions and report still written) if a shift misses tol,
 * EBREAKDOWN on non-finite input or a Krylov breakdown. */
int ndtm_solve(ndtm_ctx* ctx, void* const* x_dev, const void* b_dev,
               const ndtm_solve_params* p, ndtm_solve_report* report, void* stream);

/* ---- device storage ----------------------------------------------------------
 * Not an operation of the paper: storage for the fields the solve of
 * eq:shifted_linear works on (links, the Krylov vectors of section 4.2, the
 * multigrid data of section 3).
 *
 * ndtm_workspace_bytes: an upper bound, in *bytes, on the lattice storage that
 * set_gauge (with the clover term if c_sw is already set), apply (any op and
 * precision), mg_setup with *mg and the multigrid
 * calls, and solve / solve_rational with *sp for n_shifts shifts need together
 * (mg or sp NULL: that part left out; the learned-guess training calls with batch B
 * need about B x 35 KB more).  EINVAL for a null ctx or bytes, n_shifts outside
 * [1, NDTM_MAX_SHIFTS] with sp, or mg parameters that do not fit the lattice.
 *
 * ndtm_set_workspace: hands the context a device region of `bytes` (256-byte
 * aligned) that the caller owns and keeps alive until ndtm_destroy or a later
 * ndtm_set_workspace(ctx, NULL, 0).  From then on every lattice-sized buffer is
 * carved out of it (first fit, 256-byte blocks) and no call allocates device
 * memory; a call whose storage does not fit returns NDTM_ENOMEM.  With a region
 * smaller than the bound for the solve's mms_defer, the multi-shift CG keeps fewer
 * residual slots (same iterates).  dev NULL returns to hipMalloc storage.  ESTATE
 * once the context holds lattice storage (call it before set_gauge); EINVAL for a
 * misaligned or tiny region.
 *
 * ndtm_workspace_stats: live and peak bytes of lattice storage and the number of
 * hipMalloc calls the context has made for it (0 in a caller region). */
int ndtm_workspace_bytes(const ndtm_ctx* ctx, int n_shifts, const ndtm_mg_params* mg, const ndtm_solve_params* sp,
                         size_t* bytes);
int ndtm_set_workspace(ndtm_ctx* ctx, void* dev, size_t bytes);
int ndtm_workspace_stats(const ndtm_ctx* ctx, size_t* live, size_t* peak, long long* device_allocs);
/* Gives back the temporary fields that earlier solve, apply, guess and multigrid calls
 * keep for reuse (to hipFree, or to the caller region); the links, the multigrid setup
 * and the network weights stay.  Later calls take them again.  Synchronises the
 * device. */
int ndtm_trim(ndtm_ctx* ctx);

/* ---- hybrid split (section 4.4) ------------------------------------------ */
/* The n minimising c_HY(n) = t_CG(m_n^2) + sum_{i>n} t_MG(m_i^2) (eq:costwo) for the
 * shifts sigma_desc[0..n_shifts) (strictly descending, > 0): t_CG(sigma) is the CG
 * iteration bound 0.5 sqrt(kappa) ln(2/tol), kappa = (lambda_max + sigma) /
 * (lambda_min + sigma), times ms_per_iteration; t_MG = ms_per_mg_shift, a cost the
 * caller measures for its multigrid and initial guesses (the paper fits both costs
 * to measurements).  The spectrum may come from ndtm_spectrum_estimate.  Host
 * computation, no context or device.  EINVAL on inconsistent arguments. */
int ndtm_hybrid_split(int n_shifts, const double* sigma_desc, double lambda_min, double lambda_max, double tol,
                      double ms_per_iteration, double ms_per_mg_shift, int* n_out);

/* Extreme eigenvalues of Q^2 estimated from the Lanczos matrix of the base system
 * (its CG coefficients over the first 512 iterations) of the last multi-shift solve on
 * this context that used the deferred form (Ritz values: inside the spectrum, the
 * largest close to lambda_max after a few dozen iterations).  They bound the spectrum
 * for ndtm_hybrid_split, the automatic split, case C's tolerance and the interval of
 * ndtm_solve_rational.  ESTATE before one. */
int ndtm_spectrum_estimate(const ndtm_ctx* ctx, double* lambda_min, double* lambda_max);

/* ---- rational approximation (section "Rational approximation") ---------- */
/* Zolotarev's optimal rational approximation R(y) = a prod_j (y + c_{2j-1})/(y + c_{2j})
 * of 1/sqrt(y) on eps < y < 1, order n (eq:rational, eq:zolotarev_shifts): writes
 * c[0..2n-1] = c_1..c_2n (descending), *a and *delta = max |1 - sqrt(y) R(y)|
 * (eq:deviation; delta = d^2 / (1 + sqrt(1 - d^2))^2).  Host computation, no
 * context or device; 0 <= n <= 16, 0 < eps < 1, else EINVAL. */
int ndtm_zolotarev(int n, double eps, double* c, double* a, double* delta);

/* y ~ (Q^2)^{-1/2} b by eq:ratapp, for a spectrum of Q^2 inside [eps lambda, lambda]:
 * the order-n coefficients on [eps, 1] give the shifts sigma_i = lambda c_{2i}, which
 * become the context's shifts (as ndtm_set_shifts would set them), all shifts are
 * solved by ndtm_solve with *p (report in *report), and
 * y = lambda^{-1/2} a (b + sum_i q_i lambda x_i).  b, y: odd-site canonical complex128
 * on the device, not aliased.  The relative error of y is at most delta plus the solve
 * tolerance amplified by the weights.  Returns ndtm_solve's status (y is written for
 * ENOCONV too); EINVAL for 1 <= n <= 16, 0 < eps < 1, lambda > 0 violated.
 * Synchronises the stream. */
int ndtm_solve_rational(ndtm_ctx* ctx, void* y_dev, const void* b_dev, int n, double eps, double lambda,
                        const ndtm_solve_params* p, ndtm_solve_report* report, void* stream);

/* ---- learned initial-guess proposer ------------------------------------ */
/* A 3-layer tanh network (59 -> 64 -> 64 -> 11) proposes the correction y to the
 * Lagrange coefficients over the converged solutions, c = l + tau y with
 * tau = ||r_L|| / ||b|| (r_L the Lagrange guess's residual), a generalisation of
 * the interpolated guesses of section 4.2.  Its relative loss
 * L = 1 + 2 h.y + y.G.y is exact from the Gram form of appendix B (see
 * ndtm_mlp_sample).  Weights: NDTM_MLP_NPARAM floats, W1 (64x59), b1, W2 (64x64),
 * b2, W3 (11x64), b3, row-major; FP32 for training, a BF16 copy for inference.
 * All arrays of these calls are host memory; the calls synchronise the device. */
#define NDTM_MLP_NFEAT 59
#define NDTM_MLP_KMAX 11
#define NDTM_MLP_NPARAM 8715
/* Loads weights and resets the Adam state (initial or trained weights). */
int ndtm_mlp_set_weights(ndtm_ctx* ctx, const float* w, size_t n);
int ndtm_mlp_get_weights(ndtm_ctx* ctx, float* w, size_t n);
/* Outputs y (B x 11) for features (B x 59); bf16 != 0 uses the BF16 inference
 * kernel, else the FP32 one, which also returns the per-sample loss when mask,
 * G (B x 11 x 11) and h (B x 11) are given (NULL = zeros). */
int ndtm_mlp_forward(ndtm_ctx* ctx, int B, const float* feat, const float* mask, const float* G, const float* h,
                     int bf16, float* y, float* loss);
/* Gradient of the batch-mean loss w.r.t. the flat parameters, and the mean loss. */
int ndtm_mlp_grad(ndtm_ctx* ctx, int B, const float* feat, const float* mask, const float* G, const float* h,
                  float* grad, float* mean_loss);
/* `steps` full-batch Adam steps (beta1 0.9, beta2 0.999, eps 1e-8) on the device;
 * loss_hist (optional, steps floats) receives the mean loss before each step. */
int ndtm_mlp_train(ndtm_ctx* ctx, int B, const float* feat, const float* mask, const float* G, const float* h,
                   int steps, float lr, float* loss_hist);
/* One training sample from solved vectors: x_dev[0..K) are the converged
 * solutions (odd-site canonical, device) of the shifts nodes[0..K), descending
 * and all above sig_t; b_dev the right-hand side (same layout).  Computes x_L, r_L = b - (Q^2 + sig_t) x_L, the Gram
 * matrix of [b, x_1..x_K] and the overlaps with r_L on the GPU, then the
 * features (59), mask (11), G (11 x 11) and h (11) in slot order (slot 0 = the
 * nearest node).  The solver's node selection applies first: the farthest
 * nodes are dropped while the Lebesgue constant of the Lagrange coefficients
 * exceeds 4, and the sample covers nodes[first..K).  info (optional, 4 doubles):
 * [tau, ||r_L||^2, ||b||^2, first]. */
int ndtm_mlp_sample(ndtm_ctx* ctx, int K, void* const* x_dev, const double* nodes, double sig_t, const void* b_dev,
                    float* feat, float* mask, float* G, float* h, double* info, void* stream);

/* Kernel timing.  When enabled, every launch of the kernel classes below made
 * by later calls is bracketed by HIP events on its stream, and its algorithmic
 * byte count (the bytes the operation must move, see NDTM_PROF_*) is added to
 * the class.  ndtm_profile_read returns, for one class, the summed kernel
 * milliseconds, the launch count and the algorithmic bytes since the last
 * reset (it synchronises the recorded events). */
enum {
  NDTM_PROF_HOP_F64 = 0,  /* stencil pass, per output site 1920 B: 8 links of 18 reals, one
                             input and one output doublet spinor; the fused site epilogues
                             also move 384 B per site vector they read (ndtm_profile_moved) */
  NDTM_PROF_HOP_F32 = 1,  /* 960 B (moved: +192 per epilogue vector) */
  NDTM_PROF_HOP_F16 = 2,  /* 488 B (moved: +100 per epilogue vector) */
  NDTM_PROF_MMS_UPDATE = 3, /* shifted updates.  Deferred form: p = r + beta p, 3 x 384 B
                               per odd site and iteration, and each flush of m residuals,
                               (m + 3 N_touched + N_still_active) x 384 B per odd site.
                               Per-iteration form: (1 + 4 N_active) x 384 B per odd site
                               (r, p in, p out; x_s, p_s in and out; the base shift's
                               direction is p itself) */
  NDTM_PROF_MMS_RESID = 4,  /* r -= alpha w with ||r||^2, 3 x 384 B per odd site */
  NDTM_PROF_RESTRICT = 5,   /* restriction, V x (12 Nv + 24) complex of the cycle precision */
  NDTM_PROF_PROLONG = 6,    /* prolongation, same bytes as the restriction */
  NDTM_PROF_COARSE = 7,     /* coarse stencil, Vc x 5.5 (2 Nv)^2 complex (self and forward blocks,
                               the odd-projector block) + 2 coarse vectors */
  NDTM_PROF_NCLASS = 8
};
/* Streaming reference on the context's device: a copy (read + write), a read
 * and a write of `bytes` (>= 1 MiB, multiple of 16) with 16-byte non-temporal
 * accesses per lane, each repeated `reps` times and timed with HIP events; the
 * bandwidths in GB/s are written to the three host doubles.  Allocates and
 * frees two device buffers of `bytes`; synchronises the device.  It gives the
 * measured ceiling that the library's bandwidth-bound kernels are compared with. */
int ndtm_stream_bandwidth(ndtm_ctx* ctx, size_t bytes, int reps, double* copy_gbs, double* read_gbs,
                          double* write_gbs);

/* Traversal of the hopping stencil (eq:Wilson's H on one parity).  A tuning knob: the
 * result is bit for bit the same, as every output site sums its eight hops in the same
 * order.  Output sites are visited in (z, y) tiles of bz x by sites with whole x rows,
 * each tile marched through t, so that a site's t-neighbours are still in the L2 when
 * they are read again.  bz = 0: chosen from the L2 size; by = 0: whole y planes.
 * EINVAL unless bz and by are 0 or divide Lz and Ly. */
int ndtm_set_stencil_tile(ndtm_ctx* ctx, int bz, int by);

/* mask: bit k enables timing of kernel class k (NDTM_PROF_*); 0 disables. */
int ndtm_profile_enable(ndtm_ctx* ctx, int mask);
int ndtm_profile_read(ndtm_ctx* ctx, int kernel_class, double* total_ms, long long* launches,
                      double* alg_bytes, int reset);
/* Bytes the class's timed launches moved since the last reset: the algorithmic bytes
 * plus, for the stencil, the site vectors its fused epilogues read.  Call after
 * ndtm_profile_read (which collects the events) and before its reset. */
int ndtm_profile_moved(const ndtm_ctx* ctx, int kernel_class, double* moved_bytes);

#ifdef __cplusplus
}
#endif

#endif /* NDTM_H */
