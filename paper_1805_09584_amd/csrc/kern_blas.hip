// Vector kernels on FP64 complex arrays, deterministic two-pass reductions and
// the device-side multi-shift CG recurrences.
//
// Reductions: every block writes one partial per scalar; blas_finalize sums
// the partials of each scalar in a fixed order, so results are bitwise
// reproducible run to run.  Grids are capped (grid-stride loops) so the number
// of partials per scalar never exceeds kRedBlocks.
//
// Multi-shift CG (MMS-CG, the standard solver of section 1 and section 4.2):
// one Krylov space for the smallest shift; the shifted systems follow from
// r_s = zeta_s r.  All recurrences (alpha, beta, zeta_s, alpha_s, beta_s,
// freezing) run on the device in FP64; the host only polls the done flag.
#include "mms_scalars.h"
#include "ndtm_internal.h"

namespace ndtm {
namespace {

constexpr int kRedBlocks = 1024;
constexpr int kMaxVec = 40;

struct VecList {
  const double2* v[kMaxVec];
};
struct MutVecList {
  double2* v[kMaxVec];
};

inline unsigned grid_for(size_t n) {
  size_t g = (n + 255) / 256;
  if (g > (size_t)kRedBlocks) g = kRedBlocks;
  if (g == 0) g = 1;
  return (unsigned)g;
}

__device__ __forceinline__ double block_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off);
  __shared__ double ws[4];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) ws[w] = v;
  __syncthreads();
  double s = 0;
  if (threadIdx.x == 0) s = ws[0] + ws[1] + ws[2] + ws[3];
  return s;  // valid in thread 0
}

__global__ void zero_k(double* p, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

__global__ void copy_k(double2* y, const double2* x, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    y[i] = x[i];
}

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__global__ void axpby_k(double2* y, double2 a, const double2* x, double2 b, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const double2 xa = cmul(a, x[i]);
    const double2 yb = cmul(b, y[i]);
    y[i] = make_double2(xa.x + yb.x, xa.y + yb.y);
  }
}

__global__ void axpy_k(double2* y, double2 a, const double2* x, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const double2 xa = cmul(a, x[i]);
    y[i] = make_double2(y[i].x + xa.x, y[i].y + xa.y);
  }
}

__global__ void scale_k(double2* y, double2 a, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    y[i] = cmul(a, y[i]);
}

__global__ void norm2_k(const double2* x, size_t n, double* partials) {
  double s = 0;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    s += x[i].x * x[i].x + x[i].y * x[i].y;
  s = block_sum(s);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

__global__ void dot_k(const double2* x, const double2* y, size_t n, double* partials) {
  double re = 0, im = 0;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    re += x[i].x * y[i].x + x[i].y * y[i].y;
    im += x[i].x * y[i].y - x[i].y * y[i].x;
  }
  re = block_sum(re);
  im = block_sum(im);
  if (threadIdx.x == 0) {
    partials[blockIdx.x] = re;
    partials[gridDim.x + blockIdx.x] = im;
  }
}

// partials laid out [width][nparts]; block j sums column j in a fixed order.
__global__ void finalize_k(const double* partials, int nparts, double* dst) {
  const double* p = partials + (size_t)blockIdx.x * nparts;
  double s = strided_sum(p, nparts);
  s = block_sum(s);
  if (threadIdx.x == 0) dst[blockIdx.x] = s;
}

// <V_i, w> for i < k: each thread accumulates k complex sums.
template <int KMAX>
__global__ void multidot_k(VecList V, int k, const double2* w, size_t n, double* partials) {
  double re[KMAX], im[KMAX];
#pragma unroll
  for (int j = 0; j < KMAX; ++j) re[j] = im[j] = 0;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const double2 wi = w[i];
#pragma unroll
    for (int j = 0; j < KMAX; ++j) {
      if (j < k) {
        const double2 v = V.v[j][i];
        re[j] += v.x * wi.x + v.y * wi.y;
        im[j] += v.x * wi.y - v.y * wi.x;
      }
    }
  }
  for (int j = 0; j < k; ++j) {
    const double a = block_sum(re[j]);
    const double b = block_sum(im[j]);
    if (threadIdx.x == 0) {
      partials[(size_t)(2 * j) * gridDim.x + blockIdx.x] = a;
      partials[(size_t)(2 * j + 1) * gridDim.x + blockIdx.x] = b;
    }
  }
}

__global__ void multi_axpy_dev_k(double2* w, VecList V, int k, const double* coef, double sgn, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    double2 acc = w[i];
    for (int j = 0; j < k; ++j) {
      const double2 c = make_double2(sgn * coef[2 * j], sgn * coef[2 * j + 1]);
      const double2 t = cmul(c, V.v[j][i]);
      acc.x -= t.x;
      acc.y -= t.y;
    }
    w[i] = acc;
  }
}

struct CoefList {
  double2 c[kMaxVec];
};

__global__ void lincomb_k(double2* y, VecList V, CoefList C, int k, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    double2 acc = make_double2(0, 0);
    for (int j = 0; j < k; ++j) {
      const double2 t = cmul(C.c[j], V.v[j][i]);
      acc.x += t.x;
      acc.y += t.y;
    }
    y[i] = acc;
  }
}

// ---------------- MMS-CG ----------------
constexpr int kFusedPrefetch = 4;  // elements per thread loaded before the scalar is known

// Deferred form, fused: the two vector passes of iteration `it` also carry its two
// scalar steps.  Every block takes alpha (beta) from the partials itself, in the
// same order as the stand-alone steps, and block 0 also takes the step on S, before
// its share of the vector (so that the serial step does not end the launch).  No
// block reads a value that the step of the same launch changes (beta takes
// ||r_k||^2 from MS_RR_OLD, written by step 1 in the previous launch; the step
// writes the rest of the header back unchanged).  A set *skip (the done flag)
// makes the residual pass return at once, before step 1; the direction pass then
// sees no MS_GO mark for this iteration and returns too (it cannot read the done
// flag itself: its own step 2 may set it).
__global__ void __launch_bounds__(256) mms_update_r_fused_k(const double2* rin, double2* rout, const double2* w,
                                                            double* S, size_t n, const double* pst, int nst,
                                                            double* partials, const double* skip, int it) {
  if (skip && *skip != 0.0) return;
  const size_t i0 = blockIdx.x * (size_t)blockDim.x + threadIdx.x, stride = (size_t)gridDim.x * blockDim.x;
  // the first elements are on their way while alpha is formed
  double2 rp[kFusedPrefetch], wp[kFusedPrefetch];
#pragma unroll
  for (int j = 0; j < kFusedPrefetch; ++j) {
    const size_t i = i0 + j * stride;
    if (i < n) {
      rp[j] = rin[i];
      wp[j] = w[i];
    }
  }
  const double pw = mms::sum_partials(pst, nst);
  const double alpha = mms::alpha_of(S, pw);
  // block 0 takes the step first, while the other blocks stream
  if (blockIdx.x == 0) mms::step1_pw(S, pw, (double)(it + 1));
  double acc = 0;
#pragma unroll
  for (int j = 0; j < kFusedPrefetch; ++j) {
    const size_t i = i0 + j * stride;
    if (i < n) {
      double2 v = rp[j];
      v.x -= alpha * wp[j].x;
      v.y -= alpha * wp[j].y;
      rout[i] = v;
      acc += v.x * v.x + v.y * v.y;
    }
  }
  for (size_t i = i0 + kFusedPrefetch * stride; i < n; i += stride) {
    double2 v = rin[i];
    const double2 wi = w[i];
    v.x -= alpha * wi.x;
    v.y -= alpha * wi.y;
    rout[i] = v;
    acc += v.x * v.x + v.y * v.y;
  }
  acc = block_sum(acc);
  if (threadIdx.x == 0) partials[blockIdx.x] = acc;
}

__global__ void __launch_bounds__(256) mms_update_pbase_fused_k(const double2* r, double2* p, double* S, size_t n,
                                                                const double* pr, int npr, int slot, double* H,
                                                                int it) {
  if (S[MS_GO] != (double)(it + 1)) return;
  const bool stepped = S[MS_ALPHA] != 0.0;
  const size_t i0 = blockIdx.x * (size_t)blockDim.x + threadIdx.x, stride = (size_t)gridDim.x * blockDim.x;
  double2 rp[kFusedPrefetch], pp[kFusedPrefetch];
  if (stepped) {
#pragma unroll
    for (int j = 0; j < kFusedPrefetch; ++j) {
      const size_t i = i0 + j * stride;
      if (i < n) {
        rp[j] = r[i];
        pp[j] = p[i];
      }
    }
  }
  const double rr = mms::sum_partials(pr, npr);
  // block 0 takes the step first, while the other blocks stream
  if (blockIdx.x == 0) mms::step2_rr(S, rr, slot, H);
  if (stepped) {
    if (isfinite(rr)) {
      const double beta = rr / S[MS_RR_OLD];
#pragma unroll
      for (int j = 0; j < kFusedPrefetch; ++j) {
        const size_t i = i0 + j * stride;
        if (i < n) p[i] = make_double2(rp[j].x + beta * pp[j].x, rp[j].y + beta * pp[j].y);
      }
      for (size_t i = i0 + kFusedPrefetch * stride; i < n; i += stride) {
        const double2 ri = r[i], pi = p[i];
        p[i] = make_double2(ri.x + beta * pi.x, ri.y + beta * pi.y);
      }
    }
  }
}

// Scalar steps of an iteration (one block each).
__global__ void mms_scal1_k(double* S, const double* partials, int nparts) { mms::step1(S, partials, nparts); }

__global__ void mms_scal2_k(double* S, const double* partials, int nparts, int slot, double* H) {
  mms::step2(S, partials, nparts, slot, H);
}

// r_out = r_in - alpha w (in place when r_out == r_in), with ||r_out||^2 partials.
// A set *skip (the solve's done flag) makes the launch return at once.
__global__ void __launch_bounds__(256) mms_update_r_k(const double2* rin, double2* rout, const double2* w,
                                                      const double* S, size_t n, double* partials,
                                                      const double* skip) {
  if (skip && *skip != 0.0) return;
  const double alpha = S[MS_ALPHA];
  double acc = 0;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    double2 v = rin[i];
    const double2 wi = w[i];
    v.x -= alpha * wi.x;
    v.y -= alpha * wi.y;
    rout[i] = v;
    acc += v.x * v.x + v.y * v.y;
  }
  acc = block_sum(acc);
  if (threadIdx.x == 0) partials[blockIdx.x] = acc;
}


struct ShiftPtrs {
  double2* x[kMaxShifts];
  double2* p[kMaxShifts];
};

// sb: the base shift (delta = 0).  Its zeta stays 1, so its direction equals the
// base direction p and is not stored separately: x_sb += alpha p before p moves.
// it >= 0: the launch belongs to iteration it and returns at once unless that
// iteration took its scalar step (the iterations queued past convergence).
__global__ void mms_update_p_k(const double2* r, double2* p, ShiftPtrs P, int nsh, int sb, const double* S,
                               size_t n, int it) {
  if (it >= 0 && S[MS_IT] != (double)(it + 1)) return;
  const double beta = S[MS_BETA];
  const bool any_before = S[MS_ALPHA] != 0.0;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const double2 ri = r[i];
    const double2 pold = p[i];
    for (int s = 0; s < nsh; ++s) {
      if (S[MS_ACT + s] == 0.0) continue;
      if (s == sb) {
        const double as = S[MS_ALPHA_S + s];
        double2 xs = P.x[s][i];
        xs.x += as * pold.x;
        xs.y += as * pold.y;
        P.x[s][i] = xs;
        continue;
      }
      const double as = S[MS_ALPHA_S + s], bs = S[MS_BETA_S + s], z = S[MS_ZETA + s];
      double2 ps = P.p[s][i];
      double2 xs = P.x[s][i];
      xs.x += as * ps.x;
      xs.y += as * ps.y;
      ps.x = z * ri.x + bs * ps.x;
      ps.y = z * ri.y + bs * ps.y;
      P.x[s][i] = xs;
      P.p[s][i] = ps;
    }
    if (any_before) p[i] = make_double2(ri.x + beta * pold.x, ri.y + beta * pold.y);
  }
}

typedef double v2d_nt __attribute__((ext_vector_type(2)));
__device__ __forceinline__ double2 ld_stream(const double2* p) {
  const v2d_nt v = __builtin_nontemporal_load(reinterpret_cast<const v2d_nt*>(p));
  return make_double2(v.x, v.y);
}

// Base direction of the deferred form: p = r + beta p (r is r_{k+1}) for
// iteration it; skipped unless that iteration took its scalar step.
__global__ void __launch_bounds__(256) mms_update_pbase_k(const double2* r, double2* p, const double* S,
                                                           size_t n, int it) {
  if (S[MS_IT] != (double)(it + 1) || S[MS_ALPHA] == 0.0) return;
  const double beta = S[MS_BETA];
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const double2 ri = r[i], pi = p[i];
    p[i] = make_double2(ri.x + beta * pi.x, ri.y + beta * pi.y);
  }
}

struct DeferPtrs {
  double2* x[kMaxShifts];
  double2* p[kMaxShifts];
};

// Coefficients of a block of nr iterations that began at iteration k0 (one thread
// per shift).  Only the iterations that took their step count (S[MS_IT] of them in
// total): K = min(nr, S[MS_IT] - k0).  With x_{k+1} = x_k + alpha_k p_k and
// p_{k+1} = zeta_{k+1} r_{k+1} + beta_k p_k, unrolled from the block start P, X:
//   x_end = X + S_{k0} P + sum_j zeta_{k0+j+1} S_{k0+j+1} r_{k0+j+1},
//   p_end = T_{k0} P + sum_j zeta_{k0+j+1} T_{k0+j+1} r_{k0+j+1},
// with S_k = alpha_k + beta_k S_{k+1}, T_k = beta_k T_{k+1}, S_end = 0, T_end = 1.
// A frozen shift records alpha = 0, so its S stays exact; its T is not used.
__global__ void mms_flush_prep_k(const double* S, const double* H, double* C, int nr, int k0) {
  // the history is staged through LDS in chunks of kPrepChunk slots (loaded by the
  // whole block), so that the per-shift recurrence does not wait on global memory
  constexpr int kPrepChunk = 64;
  __shared__ double hs[kPrepChunk][kMaxShifts][kHistStride];
  const int nsh = (int)S[MS_NSH];
  const int K = max(0, min(nr, (int)S[MS_IT] - k0));
  const int s = threadIdx.x;
  double* c = C + (size_t)(s < kMaxShifts ? s : 0) * kCoefStride;
  double sa = 0.0, t = 1.0;
  bool touched = false;
  if (s < nsh)
    for (int j = K; j < nr; ++j) c[MC_C + j] = c[MC_D + j] = 0.0;
  for (int top = K; top > 0; top -= kPrepChunk) {
    const int lo = max(0, top - kPrepChunk);
    __syncthreads();
    for (int e = threadIdx.x; e < (top - lo) * kMaxShifts * kHistStride; e += blockDim.x)
      (&hs[0][0][0])[e] = H[(size_t)lo * kMaxShifts * kHistStride + e];
    __syncthreads();
    if (s < nsh) {
      for (int j = top - 1; j >= lo; --j) {
        const double* h = hs[j - lo][s];
        const double al = h[0], be = h[1], ze = h[2];
        c[MC_D + j] = ze * sa;
        c[MC_C + j] = ze * t;
        sa = al + be * sa;
        t = be * t;
        touched |= h[3] != 0.0;
      }
    }
  }
  if (s < nsh) {
    c[MC_A] = t;
    c[MC_E] = sa;
    c[MC_TOUCHED] = touched ? 1.0 : 0.0;
  }
}

// The flush: for every shift touched in the block,
//   x_s = x_s + e P_s + sum_j d_j R_j,   P_s = a P_s + sum_j c_j R_j (WITH_P),
// with the shifts' sums kept in registers while the residuals stream by in chunks
// of kFlushChunk, so each residual and each x_s, P_s moves once.  A chunk's
// coefficients are staged in LDS (the loop over elements is block-uniform so that
// every thread reaches the barriers).  The direction of a shift that has frozen is
// not written back (it is never used again).
constexpr int kFlushChunk = 8;
template <bool WITH_P>
__global__ void __launch_bounds__(256) mms_flush_k(DeferPtrs P, const double2* R, int nr, const double* S,
                                                   const double* C, size_t n) {
  __shared__ double cd[kMaxShifts][2][kFlushChunk];  // [k][0: c, 1: d][j] of the current chunk
  __shared__ double ae[kMaxShifts][2];
  __shared__ int keep[kMaxShifts], list[kMaxShifts], nlist;
  const int nsh = (int)S[MS_NSH];
  if (threadIdx.x == 0) {
    int k = 0;
    for (int s = 0; s < nsh; ++s)
      if (C[(size_t)s * kCoefStride + MC_TOUCHED] != 0.0) list[k++] = s;
    nlist = k;
  }
  __syncthreads();
  const int nl = nlist;
  if (nl == 0) return;
  if (threadIdx.x < nl) {
    const int s = list[threadIdx.x];
    const double* c = C + (size_t)s * kCoefStride;
    ae[threadIdx.x][0] = c[MC_A];
    ae[threadIdx.x][1] = c[MC_E];
    keep[threadIdx.x] = S[MS_ACT_NEXT + s] != 0.0;
  }
  __syncthreads();
  for (size_t base = blockIdx.x * (size_t)blockDim.x; base < n; base += (size_t)gridDim.x * blockDim.x) {
    const size_t i = base + threadIdx.x;
    const bool valid = i < n;
    double2 ax[kMaxShifts], ap[kMaxShifts];
#pragma unroll
    for (int k = 0; k < kMaxShifts; ++k) {
      if (k < nl && valid) {
        const double2 p0 = P.p[list[k]][i], x0 = P.x[list[k]][i];
        const double a = ae[k][0], e = ae[k][1];
        ax[k] = make_double2(x0.x + e * p0.x, x0.y + e * p0.y);
        if (WITH_P) ap[k] = make_double2(a * p0.x, a * p0.y);
      }
    }
    for (int c0 = 0; c0 < nr; c0 += kFlushChunk) {
      __syncthreads();  // the previous chunk's coefficients are no longer read
      if (threadIdx.x < nl * 2 * kFlushChunk) {
        const int k = threadIdx.x / (2 * kFlushChunk), w = (threadIdx.x / kFlushChunk) & 1;
        const int j = threadIdx.x % kFlushChunk;
        cd[k][w][j] = c0 + j < nr ? C[(size_t)list[k] * kCoefStride + (w ? MC_D : MC_C) + c0 + j] : 0.0;
      }
      __syncthreads();
      if (!valid) continue;
      double2 rv[kFlushChunk];
#pragma unroll
      for (int j = 0; j < kFlushChunk; ++j)
        rv[j] = c0 + j < nr ? ld_stream(R + (size_t)(c0 + j) * n + i) : make_double2(0.0, 0.0);
#pragma unroll
      for (int k = 0; k < kMaxShifts; ++k) {
        if (k < nl) {
#pragma unroll
          for (int j = 0; j < kFlushChunk; ++j) {
            const double d = cd[k][1][j];
            ax[k].x += d * rv[j].x;
            ax[k].y += d * rv[j].y;
            if (WITH_P) {
              const double c = cd[k][0][j];
              ap[k].x += c * rv[j].x;
              ap[k].y += c * rv[j].y;
            }
          }
        }
      }
    }
    if (!valid) continue;
#pragma unroll
    for (int k = 0; k < kMaxShifts; ++k) {
      if (k < nl) {
        P.x[list[k]][i] = ax[k];
        if (WITH_P && keep[k]) P.p[list[k]][i] = ap[k];
      }
    }
  }
}

__global__ void mms_seed_k(double* S, const double* src) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    S[MS_RR] = src[0];
    S[MS_BB] = src[0];
  }
}

// ---------------- deferred MMS-CG on low-precision stencil storage ----------------
// The mixed form keeps the FP64 Krylov vectors and residual ring of the deferred form;
// only the stencil runs on FP32 or FP16 copies.  The residual pass reads w as the
// stencil wrote it, the direction pass writes p's copy for the next stencil.  Both
// storages come in 16-byte words per half-site: FP32 holds 2 complex components a word
// (12 words), FP16 4 (6 words, one FP32 scale per site).  Scalar steps as in the FP64
// fused passes.
typedef unsigned mx_v4u __attribute__((ext_vector_type(4)));
union MxWord {
  mx_v4u w;
  __half2 h[4];
  float2 f[2];
};

template <int PREC>
struct MxStore {
  static constexpr int kPer = PREC == P16 ? 4 : 2;  // complex components per word
  static constexpr int kWords = 24 / kPer;
  __device__ static float2 get(const MxWord& u, int j) {
    if constexpr (PREC == P16)
      return __half22float2(u.h[j]);
    else
      return u.f[j];
  }
  __device__ static void put(MxWord& u, int j, double x, double y, double inv) {
    if constexpr (PREC == P16)
      u.h[j] = __floats2half2_rn((float)(x * inv), (float)(y * inv));
    else
      u.f[j] = make_float2((float)x, (float)y);
  }
};

template <int PREC>
__global__ void __launch_bounds__(256) mms_update_r_fused_mx_k(const double2* rin, double2* rout, const mx_v4u* wq,
                                                               const float* wsc, double* S, int vh, int stride,
                                                               const double* pst, int nst, double* partials,
                                                               const double* skip, int it) {
  using M = MxStore<PREC>;
  if (skip && *skip != 0.0) return;
  const double pw = mms::sum_partials(pst, nst);
  const double alpha = mms::alpha_of(S, pw);
  if (blockIdx.x == 0) mms::step1_pw(S, pw, (double)(it + 1));
  double acc = 0;
  // the padding sites past vh carry rin over (the FP64 passes treat them as sites)
  const long nq = (long)M::kWords * stride;
  for (long q = blockIdx.x * (long)blockDim.x + threadIdx.x; q < nq; q += (long)gridDim.x * blockDim.x) {
    const int g = (int)(q / stride), h = (int)(q - (long)g * stride);
    MxWord u;
    double a = 0;
    if (h < vh) {
      u.w = wq[(long)g * stride + h];
      a = PREC == P16 ? alpha * (double)wsc[h] : alpha;
    } else {
      u.w = mx_v4u{0u, 0u, 0u, 0u};
    }
#pragma unroll
    for (int j = 0; j < M::kPer; ++j) {
      const long i = (long)(M::kPer * g + j) * stride + h;
      const float2 wf = M::get(u, j);
      double2 v = rin[i];
      v.x -= a * (double)wf.x;
      v.y -= a * (double)wf.y;
      rout[i] = v;
      acc += v.x * v.x + v.y * v.y;
    }
  }
  acc = block_sum(acc);
  if (threadIdx.x == 0) partials[blockIdx.x] = acc;
}

template <int PREC>
__global__ void __launch_bounds__(256) mms_update_pbase_fused_mx_k(const double2* r, double2* p, mx_v4u* pq,
                                                                   float* psc, double* S, int vh, int stride,
                                                                   const double* pr, int npr, int slot, double* H,
                                                                   int it) {
  using M = MxStore<PREC>;
  if (S[MS_GO] != (double)(it + 1)) return;
  const bool stepped = S[MS_ALPHA] != 0.0;
  const double rr = mms::sum_partials(pr, npr);
  if (blockIdx.x == 0) mms::step2_rr(S, rr, slot, H);
  if (!stepped || !isfinite(rr)) return;
  const double beta = rr / S[MS_RR_OLD];
  for (int h = blockIdx.x * blockDim.x + threadIdx.x; h < vh; h += gridDim.x * blockDim.x) {
    double2 pv[24];
    double mx = 0;
#pragma unroll
    for (int c = 0; c < 24; ++c) {
      const long i = (long)c * stride + h;
      const double2 ri = r[i], pi = p[i];
      pv[c] = make_double2(ri.x + beta * pi.x, ri.y + beta * pi.y);
      p[i] = pv[c];
      mx = fmax(mx, fmax(fabs(pv[c].x), fabs(pv[c].y)));
    }
    double inv = 1.0;
    if constexpr (PREC == P16) {
      const float sc = (float)mx;
      inv = sc > 0.f ? 1.0 / (double)sc : 0.0;
      psc[h] = sc;
    }
#pragma unroll
    for (int g = 0; g < M::kWords; ++g) {
      MxWord u;
#pragma unroll
      for (int j = 0; j < M::kPer; ++j) M::put(u, j, pv[M::kPer * g + j].x, pv[M::kPer * g + j].y, inv);
      pq[(long)g * stride + h] = u.w;
    }
  }
}


}  // namespace

void mms_update_r_fused_mx(int prec, const double2* rin, double2* rout, const void* wq, const float* wsc, double* S,
                           int vh, int stride, const double* pst, int nst, double* partials, int nblk,
                           const double* skip, int it, hipStream_t st) {
  if (prec == P16)
    hipLaunchKernelGGL(mms_update_r_fused_mx_k<P16>, dim3(nblk), dim3(256), 0, st, rin, rout, (const mx_v4u*)wq, wsc,
                       S, vh, stride, pst, nst, partials, skip, it);
  else
    hipLaunchKernelGGL(mms_update_r_fused_mx_k<P32>, dim3(nblk), dim3(256), 0, st, rin, rout, (const mx_v4u*)wq, wsc,
                       S, vh, stride, pst, nst, partials, skip, it);
}
void mms_update_pbase_fused_mx(int prec, const double2* r, double2* p, void* pq, float* psc, double* S, int vh,
                               int stride, const double* pr, int npr, int slot, double* H, int it, hipStream_t st) {
  const dim3 grid((vh + 255) / 256);
  if (prec == P16)
    hipLaunchKernelGGL(mms_update_pbase_fused_mx_k<P16>, grid, dim3(256), 0, st, r, p, (mx_v4u*)pq, psc, S, vh,
                       stride, pr, npr, slot, H, it);
  else
    hipLaunchKernelGGL(mms_update_pbase_fused_mx_k<P32>, grid, dim3(256), 0, st, r, p, (mx_v4u*)pq, psc, S, vh,
                       stride, pr, npr, slot, H, it);
}

void blas_zero(void* p, size_t bytes, hipStream_t st) {
  const size_t n = bytes / sizeof(double);
  hipLaunchKernelGGL(zero_k, dim3(grid_for(n)), dim3(256), 0, st, static_cast<double*>(p), n);
}
void blas_copy(double2* y, const double2* x, size_t n, hipStream_t st) {
  hipLaunchKernelGGL(copy_k, dim3(grid_for(n)), dim3(256), 0, st, y, x, n);
}
void blas_axpy(double2* y, double2 a, const double2* x, size_t n, hipStream_t st) {
  hipLaunchKernelGGL(axpy_k, dim3(grid_for(n)), dim3(256), 0, st, y, a, x, n);
}
void blas_xpay(double2* y, const double2* x, double2 a, size_t n, hipStream_t st) {
  hipLaunchKernelGGL(axpby_k, dim3(grid_for(n)), dim3(256), 0, st, y, make_double2(1, 0), x, a, n);
}
void blas_axpby(double2* y, double2 a, const double2* x, double2 b, size_t n, hipStream_t st) {
  hipLaunchKernelGGL(axpby_k, dim3(grid_for(n)), dim3(256), 0, st, y, a, x, b, n);
}
void blas_scale(double2* y, double2 a, size_t n, hipStream_t st) {
  hipLaunchKernelGGL(scale_k, dim3(grid_for(n)), dim3(256), 0, st, y, a, n);
}
int blas_norm2_partials(const double2* x, size_t n, double* partials, hipStream_t st) {
  const unsigned g = grid_for(n);
  hipLaunchKernelGGL(norm2_k, dim3(g), dim3(256), 0, st, x, n, partials);
  return (int)g;
}
int blas_dot_partials(const double2* x, const double2* y, size_t n, double* partials, hipStream_t st) {
  const unsigned g = grid_for(n);
  hipLaunchKernelGGL(dot_k, dim3(g), dim3(256), 0, st, x, y, n, partials);
  return (int)g;
}
void blas_finalize(const double* partials, int nparts, int width, double* dst, hipStream_t st) {
  hipLaunchKernelGGL(finalize_k, dim3(width), dim3(256), 0, st, partials, nparts, dst);
}
void blas_multidot(const double2* const* V, int k, const double2* w, size_t n, double* partials,
                   double* dst, hipStream_t st) {
  VecList L;
  for (int i = 0; i < k && i < kMaxVec; ++i) L.v[i] = V[i];
  const unsigned g = grid_for(n);
  if (k <= 8)
    hipLaunchKernelGGL(multidot_k<8>, dim3(g), dim3(256), 0, st, L, k, w, n, partials);
  else if (k <= 16)
    hipLaunchKernelGGL(multidot_k<16>, dim3(g), dim3(256), 0, st, L, k, w, n, partials);
  else
    hipLaunchKernelGGL(multidot_k<kMaxVec>, dim3(g), dim3(256), 0, st, L, k, w, n, partials);
  blas_finalize(partials, (int)g, 2 * k, dst, st);
}
void blas_multi_axpy_dev(double2* w, const double2* const* V, int k, const double* coef, double sgn,
                         size_t n, hipStream_t st) {
  VecList L;
  for (int i = 0; i < k && i < kMaxVec; ++i) L.v[i] = V[i];
  hipLaunchKernelGGL(multi_axpy_dev_k, dim3(grid_for(n)), dim3(256), 0, st, w, L, k, coef, sgn, n);
}
void blas_lincomb(double2* y, const double2* const* V, const double2* c, int k, size_t n, hipStream_t st) {
  VecList L;
  CoefList C;
  for (int i = 0; i < k && i < kMaxVec; ++i) {
    L.v[i] = V[i];
    C.c[i] = c[i];
  }
  hipLaunchKernelGGL(lincomb_k, dim3(grid_for(n)), dim3(256), 0, st, y, L, C, k, n);
}
void blas_gram(const double2* const* V, int k, size_t n, double* partials, double* dst, hipStream_t st) {
  // row i: <V_i, V_j> for all j (full matrix, k multidots)
  for (int j = 0; j < k; ++j) blas_multidot(V, k, V[j], n, partials, dst + 2 * k * j, st);
}

void mms_scal1(double* S, const double* partials, int nparts, hipStream_t st) {
  hipLaunchKernelGGL(mms_scal1_k, dim3(1), dim3(256), 0, st, S, partials, nparts);
}
void mms_update_r(const double2* rin, double2* rout, const double2* w, const double* S, size_t n,
                  double* partials, hipStream_t st, const double* skip) {
  hipLaunchKernelGGL(mms_update_r_k, dim3(grid_for(n)), dim3(256), 0, st, rin, rout, w, S, n, partials, skip);
}
void mms_scal2(double* S, const double* partials, int nparts, int slot, double* H, hipStream_t st) {
  hipLaunchKernelGGL(mms_scal2_k, dim3(1), dim3(256), 0, st, S, partials, nparts, slot, H);
}
void mms_update_r_fused(const double2* rin, double2* rout, const double2* w, double* S, size_t n, const double* pst,
                        int nst, double* partials, const double* skip, int it, hipStream_t st) {
  hipLaunchKernelGGL(mms_update_r_fused_k, dim3(grid_for(n)), dim3(256), 0, st, rin, rout, w, S, n, pst, nst, partials,
                     skip, it);
}
void mms_update_pbase_fused(const double2* r, double2* p, double* S, size_t n, const double* pr, int npr, int slot,
                            double* H, int it, hipStream_t st) {
  hipLaunchKernelGGL(mms_update_pbase_fused_k, dim3(grid_for(n)), dim3(256), 0, st, r, p, S, n, pr, npr, slot, H, it);
}
void mms_update_pbase(const double2* r, double2* p, const double* S, size_t n, int it, hipStream_t st) {
  hipLaunchKernelGGL(mms_update_pbase_k, dim3(grid_for(n)), dim3(256), 0, st, r, p, S, n, it);
}
void mms_flush(double2* const* xs, double2* const* ps, int nsh, const double2* R, int nr, int k0, bool with_p,
               const double* S, const double* H, double* C, size_t n, hipStream_t st) {
  DeferPtrs P;
  for (int s = 0; s < nsh; ++s) {
    P.x[s] = xs[s];
    P.p[s] = ps[s];
  }
  hipLaunchKernelGGL(mms_flush_prep_k, dim3(1), dim3(256), 0, st, S, H, C, nr, k0);
  if (with_p)
    hipLaunchKernelGGL(mms_flush_k<true>, dim3(grid_for(n)), dim3(256), 0, st, P, R, nr, S, C, n);
  else
    hipLaunchKernelGGL(mms_flush_k<false>, dim3(grid_for(n)), dim3(256), 0, st, P, R, nr, S, C, n);
}
void mms_update_p(double2* r, double2* p, double2* const* xs, double2* const* ps, int nsh, int sb,
                  const double* S, size_t n, hipStream_t st, int it) {
  ShiftPtrs P;
  for (int s = 0; s < nsh; ++s) {
    P.x[s] = xs[s];
    P.p[s] = ps[s];
  }
  hipLaunchKernelGGL(mms_update_p_k, dim3(grid_for(n)), dim3(256), 0, st, r, p, P, nsh, sb, S, n, it);
}
int red_grid(size_t n) { return (int)grid_for(n); }
void mms_seed(double* S, const double* src, hipStream_t st) {
  hipLaunchKernelGGL(mms_seed_k, dim3(1), dim3(64), 0, st, S, src);
}

}  // namespace ndtm
