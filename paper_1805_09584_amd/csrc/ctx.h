// The library context and the internal operator helpers shared by the
// drivers (MMS-CG, multigrid, hybrid).  Not part of the C-ABI.
#pragma once

#include <map>
#include <string>
#include <complex>
#include <vector>

#include "../../include/ndtm.h"
#include "ndtm_internal.h"

namespace ndtm {

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

struct MGData;  // multigrid state (mg.cpp)
struct MLPData; // learned proposer state (mlp.cpp)
struct Arena;   // caller-provided device region (memory.cpp)

}  // namespace ndtm

struct ndtm_ctx {
  int device = 0;
  ndtm::Geom g{};
  long long V = 0;
  std::string err;
  bool have_gauge = false, have_params = false;
  double kappa = 0, mubar = 0, epsbar = 0;
  ndtm::OpParams op{};
  double su3_dev = 0;  // max deviation of the stored links from SU(3) row structure
  std::vector<double> shifts;
  void* U[3][2] = {{nullptr, nullptr}, {nullptr, nullptr}, {nullptr, nullptr}};  // [prec][parity]
  void* U8[2] = {nullptr, nullptr};  // FP64 links in eight parameters (SU(3) fields), [parity]
  // clover term (eq:Wilson): c_sw and the site blocks [FP64, FP32][parity], even inverse
  double csw = 0;
  void* clv_m[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
  void* clv_inv[2] = {nullptr, nullptr};
  unsigned* clv_bad = nullptr;
  double* partials = nullptr;
  double* vred = nullptr;  // single-launch reduction workspace: [counter][partials]
  size_t partials_n = 0;
  double* dscal = nullptr;  // device scalar scratch (kScalN doubles)
  double* hscal = nullptr;  // pinned host mirror
  double* mms_S = nullptr;
  double* mms_H = nullptr;  // MMS-CG history of the deferred form [kMaxDefer][kMaxShifts][kHistStride]
  double* mms_L = nullptr;  // the history of the first kLanczosIters iterations, kept for the spectrum estimate
  double* mms_C = nullptr;  // its flush coefficients [kMaxShifts][kCoefStride]
  std::map<std::string, ndtm::DevBuf> bufs;
  int prof_mask = 0;  // bit k: time kernel class k
  const double* hop_skip = nullptr;  // device flag handed to stencil launches (see OpParams::skip)
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_used[NDTM_PROF_NCLASS];
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_free;
  double prof_ms[NDTM_PROF_NCLASS] = {};
  long long prof_n[NDTM_PROF_NCLASS] = {};
  double prof_bytes[NDTM_PROF_NCLASS] = {};  // algorithmic bytes
  double prof_moved[NDTM_PROF_NCLASS] = {};  // bytes the launches move (fused epilogue vectors too)
  ndtm::MGData* mg = nullptr;
  // extreme eigenvalues of Q^2 from the base system's Lanczos coefficients of the last
  // FP64 multi-shift solve (<= 0 while unknown)
  double est_lmin = -1, est_lmax = -1;
  // measured costs for the section 4.4 cost model: mean milliseconds per FP64 multi-shift
  // iteration and per multigrid shift (guess and case C), with their sample counts
  double cost_iter_ms = 0, cost_mg_ms = 0;
  long long cost_iter_n = 0, cost_mg_n = 0;
  ndtm::MLPData* mlp = nullptr;
  // device storage (memory.cpp): caller region or hipMalloc per buffer
  ndtm::Arena* arena = nullptr;
  std::map<void*, size_t> mem_sizes;  // every live buffer from dev_alloc
  size_t mem_live = 0, mem_peak = 0;
  long long mem_device_allocs = 0;    // hipMalloc calls made for lattice storage
  // the running solve's phase region (ndtm_solve): the multi-shift phase's shifted
  // directions and residual ring, then the multigrid phase's case-C and FGMRES vectors
  void* region = nullptr;
  size_t region_fields = 0;  // FP64 half fields it holds
};

namespace ndtm {

constexpr int kScalN = 8192;
constexpr int kLanczosIters = 512;
constexpr size_t kVredN = 8 + 96 * 1024;  // counter + partials of up to 48 complex sums over 1024 blocks

// status helpers
int fail(ndtm_ctx* c, int code, const std::string& msg);
int hip_check(ndtm_ctx* c, hipError_t e, const char* what);
#define NDTM_HIP(ctx, call)                                   \
  do {                                                        \
    hipError_t _e = (call);                                   \
    if (_e != hipSuccess) return ndtm::hip_check(ctx, _e, #call); \
  } while (0)

// device storage: every lattice-sized buffer comes from dev_alloc (caller region
// after ndtm_set_workspace, else hipMalloc); nullptr when it cannot be had
void* dev_alloc(ndtm_ctx* c, size_t bytes);
void dev_free(ndtm_ctx* c, void* p);
size_t dev_largest_free(const ndtm_ctx* c);  // largest block dev_alloc could still return
int arena_set(ndtm_ctx* c, void* dev, size_t bytes);
void arena_release(ndtm_ctx* c);
// (re)builds the clover site blocks from the links and parameters (no-op when c_sw = 0)
int clover_build(ndtm_ctx* c, hipStream_t st);
// resolves this device's address of the fixed scratch array of ndtm_apply_noalloc
void noalloc_setup(int device);
// bytes of the named buffer (0 if absent)
size_t ws_bytes(const ndtm_ctx* c, const std::string& name);

// named workspace (grown on demand, zero-filled when (re)allocated)
void* ws_get(ndtm_ctx* c, const std::string& name, size_t bytes);
HalfField half_field(ndtm_ctx* c, const std::string& name, int prec);
size_t half_elems(const ndtm_ctx* c);  // complex elements of a half field (24*stride)

// event timing of one launch of a kernel class (no-ops when profiling is off)
struct ProfScope {
  ndtm_ctx* c;
  int cls;
  hipStream_t st;
  std::pair<hipEvent_t, hipEvent_t> ev{};
  // bytes: algorithmic bytes of the launch; moved: bytes it moves (default: the same)
  ProfScope(ndtm_ctx* c_, int cls_, double bytes, hipStream_t st_, double moved = -1.0);
  ~ProfScope();
};

// stencil launch with optional event timing
void hop(ndtm_ctx* c, int prec, int epi, int red, int parity, const HalfField& in, const HalfField& out,
         const HalfField* xs, const HalfField* zs, double ms, double hop_coef, double sigma,
         double* partials, hipStream_t st);

// y = Q x (odd), using tmp_e (even)
void apply_qhat(ndtm_ctx* c, int prec, const HalfField& y, const HalfField& x, const HalfField& tmp_e,
                hipStream_t st);
// w = (Q^2 + sigma) p using u (odd) and tmp_e; partials receive Re<p, w> per block
void apply_qhat2(ndtm_ctx* c, int prec, const HalfField& w, const HalfField& p, const HalfField& u,
                 const HalfField& tmp_e, double sigma, double* partials, hipStream_t st);
// y = (S + i m Gamma5 tau1) x (odd)
void apply_sshift(ndtm_ctx* c, int prec, const HalfField& y, const HalfField& x, const HalfField& tmp_e,
                  double m, hipStream_t st);
// full lattice: (ye, yo) = D'(m) (xe, xo)
void apply_dfull(ndtm_ctx* c, int prec, const HalfField& ye, const HalfField& yo, const HalfField& xe,
                 const HalfField& xo, double m, hipStream_t st);

// reductions returning host values (synchronise the stream)
double norm2_host(ndtm_ctx* c, const double2* x, size_t n, hipStream_t st);
double2 dot_host(ndtm_ctx* c, const double2* x, const double2* y, size_t n, hipStream_t st);

int red_grid(size_t n);
void mms_seed(double* S, const double* src, hipStream_t st);

// drivers
// Stencil precision schedule of the mixed form (deferred recurrences only): the
// stencil moves to FP32 storage once ||r|| / ||b|| of the base system is at most
// rel32 and to FP16 once it is at most rel16 (0: never).  Vectors, ring, solutions
// and scalars stay FP64.
struct MmsRamp {
  double rel32 = 0, rel16 = 0;
};
struct MmsResult {
  int iterations = 0;
  int it32 = -1, it16 = -1;  // first iteration on FP32 / FP16 stencil storage (-1: none)
  std::vector<int> iters;
  bool breakdown = false;
  double lam_lo = -1, lam_hi = -1;  // extreme eigenvalues of Q^2 from the Lanczos coefficients (deferred form)
};
bool lanczos_extremes(const std::vector<double>& alpha, const std::vector<double>& beta, double* lo, double* hi);
int hybrid_choose(int N, const double* sig, double lmin, double lmax, double tol, double ms_iter, double ms_mg,
                  int* n_out, double* cost_out);
// MMS-CG for (Q^2 + sigma_s) x_s = b on internal FP64 fields; sigmas any order.
// defer >= 2: shifted vectors formed once per block of `defer` iterations (at most
// kMaxDefer); 0 or 1: updated every iteration.
// The last npass shifts of sigmas are passengers: iterated along but not waited
// for, so that their iterates can serve as initial guesses (section 4.2).
// region (optional): holds the shifted directions of shifts 1.. and the `defer`
// residual slots, (nsh - 1 + defer) FP64 half fields; without it they are named
// workspace buffers and defer is clamped to half of the free device memory.
// ramp (optional, deferred form): the mixed form's stencil precision schedule.
int run_mmscg(ndtm_ctx* c, const std::vector<double>& sigmas, const std::vector<HalfField>& xs,
              const HalfField& b, double tol, int maxiter, int poll_every, int defer, MmsResult* res,
              hipStream_t st, int npass = 0, void* region = nullptr, const MmsRamp* ramp = nullptr);
// FP64 half fields the multigrid phase takes from the solve's region (case C and FGMRES)
int mg_region_fields(int fgmres_restart, bool pair = false);
bool mg_pairs_signs(const ndtm_ctx* c);  // the setup runs case C's two signs in lock-step
// true relative residual ||b - (Q^2+sigma) x|| / ||b|| (FP64); r receives the residual
// Gram matrix <B_i, B_j> of B = [b, x_1, x_2, ...] (row-major 17 x 17), filled
// for the first `count` vectors; kept across the multigrid targets of one solve
struct GramCache {
  std::vector<std::complex<double>> M;
  int count = 0;
};
// x += CG corrections on (Q^2 + sigma) until the true residual of x meets tol
int cg_shift(ndtm_ctx* c, const HalfField& x, const HalfField& b, double sigma, double tol, int maxiter,
             double* res_out, int* iters_out, hipStream_t st);
int guess_first_node(const std::vector<double>& nodes, double sig_t);
bool mg_ready(const ndtm_ctx* c);  // a multigrid setup is in place
double true_residual(ndtm_ctx* c, const HalfField& x, const HalfField& b, double sigma,
                     const HalfField& r, hipStream_t st);

}  // namespace ndtm

extern "C" {
void ndtm_mg_free(ndtm_ctx* c);
void ndtm_mlp_free(ndtm_ctx* c);
}

namespace ndtm {
// frees every workspace buffer whose name starts with prefix
void ws_free_prefix(ndtm_ctx* c, const std::string& prefix);
}  // namespace ndtm
