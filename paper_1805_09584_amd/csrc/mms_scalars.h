// Device-side scalar recurrences of multi-shift CG (Jegerlehner's scheme, the
// standard solver of sections 1 and 4.2), taken by one block per step.
//
// The recurrences of one iteration are a short serial chain on one thread; it
// runs on a copy of the scalar header in LDS (loaded and stored back by the
// whole block), so that the chain does not wait on global memory at each step.
#pragma once

#include "ndtm_internal.h"
#include "reduce.h"

namespace ndtm {
namespace mms {

// Block sum in a fixed order: thread i adds partials i, i+256, ...; then a
// fixed shuffle tree per wave and the wave sums in order.  Valid in every thread.
__device__ __forceinline__ double sum_partials(const double* part, int n) {
  __shared__ double ws[kBlock / 64];
  __shared__ double tot;
  double v = strided_sum(part, n);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += ws[w];
    tot = s;
  }
  __syncthreads();
  return tot;
}

__device__ __forceinline__ void stage(double* dst, const double* src) {
  for (int i = threadIdx.x; i < MS_SIZE; i += blockDim.x) dst[i] = src[i];
}

// alpha of step 1 from pw, from the values step 1 reads (so that every block of a
// kernel can take it before, and while, block 0 runs the step itself)
__device__ inline double alpha_of(const double* S, double pw) {
  const int nsh = (int)S[MS_NSH];
  int any = 0;
  for (int s = 0; s < nsh; ++s) any |= S[MS_ACT_NEXT + s] != 0.0;
  if (!any || S[MS_BREAK] != 0.0 || !(pw > 0.0) || !isfinite(pw)) return 0.0;
  return S[MS_RR] / pw;
}

// alpha, zeta_{k+1}, alpha_s from pw = <p, (Q^2 + sigma_base) p>
__device__ inline void step1_body(double* S, double pw) {
  const int nsh = (int)S[MS_NSH];
  S[MS_PW] = pw;
  S[MS_RR_OLD] = S[MS_RR];
  int any = 0;
  for (int s = 0; s < nsh; ++s) {
    S[MS_ACT + s] = S[MS_ACT_NEXT + s];
    any |= S[MS_ACT + s] != 0.0;
  }
  if (!any || S[MS_BREAK] != 0.0) {
    S[MS_ALPHA] = 0.0;
    for (int s = 0; s < nsh; ++s) S[MS_ALPHA_S + s] = 0.0;
    return;
  }
  if (!(pw > 0.0) || !isfinite(pw)) {
    S[MS_BREAK] = 1.0;
    S[MS_ALPHA] = 0.0;
    for (int s = 0; s < nsh; ++s) {
      S[MS_ALPHA_S + s] = 0.0;
      S[MS_ACT + s] = 0.0;
    }
    return;
  }
  const double alpha = S[MS_RR] / pw;
  const double ap = S[MS_ALPHA_PREV], bp = S[MS_BETA];
  S[MS_ALPHA] = alpha;
  for (int s = 0; s < nsh; ++s) {
    if (S[MS_ACT + s] == 0.0) {
      S[MS_ALPHA_S + s] = 0.0;
      continue;
    }
    const double z = S[MS_ZETA + s], zp = S[MS_ZETA_PREV + s], d = S[MS_DELTA + s];
    const double den = alpha * bp * (zp - z) + zp * ap * (1.0 + d * alpha);
    const double zn = z * zp * ap / den;
    S[MS_ZETA_NEXT + s] = zn;
    S[MS_ALPHA_S + s] = alpha * zn / z;
  }
}

// beta, beta_s, the zeta roll and freezing from rr = ||r_{k+1}||^2.  Returns 1
// when the shifts active in this iteration took a step.
__device__ inline int step2_body(double* S, double rr) {
  const int nsh = (int)S[MS_NSH];
  int any = 0;
  for (int s = 0; s < nsh; ++s) any |= S[MS_ACT + s] != 0.0;
  if (!any) {
    S[MS_DONE] = 1.0;
    return 0;
  }
  if (!isfinite(rr)) {
    S[MS_BREAK] = 1.0;
    S[MS_DONE] = 1.0;
    for (int s = 0; s < nsh; ++s) S[MS_ACT_NEXT + s] = S[MS_ACT + s] = 0.0;
    return 0;
  }
  const double beta = rr / S[MS_RR];
  const double it = S[MS_IT] + 1.0;
  int still = 0;
  for (int s = 0; s < nsh; ++s) {
    if (S[MS_ACT + s] == 0.0) continue;
    const double z = S[MS_ZETA + s], zn = S[MS_ZETA_NEXT + s];
    const double q = zn / z;
    S[MS_BETA_S + s] = beta * q * q;
    S[MS_ZETA_PREV + s] = z;
    S[MS_ZETA + s] = zn;
    S[MS_ITERS + s] = it;
    // freeze once the shifted residual |zeta_s| ||r|| reaches tol ||b||
    const bool frozen = zn * zn * rr <= S[MS_TOL2] * S[MS_BB];
    S[MS_ACT_NEXT + s] = frozen ? 0.0 : 1.0;
    if (S[MS_PASS + s] == 0.0) still |= !frozen;
  }
  // done: passengers stop with the last shift that is waited for
  if (!still)
    for (int s = 0; s < nsh; ++s) S[MS_ACT_NEXT + s] = 0.0;
  S[MS_BETA] = beta;
  S[MS_ALPHA_PREV] = S[MS_ALPHA];
  S[MS_RR] = rr;
  S[MS_IT] = it;
  S[MS_DONE] = still ? 0.0 : 1.0;
  return 1;
}

// Whole block: step1 on an LDS copy of S, from pw already summed (the same value in
// every thread); go > 0 is stored in MS_GO with it.
__device__ inline void step1_pw(double* S, double pw, double go = 0.0) {
  __shared__ double sh[MS_SIZE];
  stage(sh, S);
  __syncthreads();
  if (threadIdx.x == 0) {
    step1_body(sh, pw);
    if (go > 0.0) sh[MS_GO] = go;
  }
  __syncthreads();
  stage(S, sh);
}

// Whole block: pw from the partials, then step1.
__device__ inline void step1(double* S, const double* partials, int nparts) {
  step1_pw(S, sum_partials(partials, nparts));
}

// Whole block: rr from the partials, step2 on an LDS copy of S, and for slot >= 0
// the iteration's record in slot `slot` of the history H: per shift
// (alpha_s, beta_s, zeta_{k+1}, 1) if it took a step, zeros otherwise.
// step2_rr takes rr already summed (the same value in every thread).
__device__ inline void step2_rr(double* S, double rr, int slot, double* H) {
  __shared__ double sh[MS_SIZE];
  __shared__ int go;
  stage(sh, S);
  __syncthreads();
  if (threadIdx.x == 0) go = step2_body(sh, rr);
  __syncthreads();
  stage(S, sh);
  if (slot < 0) return;
  const int s = threadIdx.x;
  if (s >= (int)sh[MS_NSH]) return;
  double* h = H + ((size_t)slot * kMaxShifts + s) * kHistStride;
  const bool act = go && sh[MS_ACT + s] != 0.0;
  h[0] = act ? sh[MS_ALPHA_S + s] : 0.0;
  h[1] = act ? sh[MS_BETA_S + s] : 0.0;
  h[2] = act ? sh[MS_ZETA + s] : 0.0;
  h[3] = act ? 1.0 : 0.0;
}

__device__ inline void step2(double* S, const double* partials, int nparts, int slot, double* H) {
  step2_rr(S, sum_partials(partials, nparts), slot, H);
}

}  // namespace mms
}  // namespace ndtm
