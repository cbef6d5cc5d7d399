// Even-odd hopping stencil of the non-degenerate twisted-mass doublet with its
// site terms fused into the epilogue.
//
// Operator (section 2, eq:Wilson and eq:non-degenerate): per flavour,
//   (H psi)(x) = sum_mu (1 - gamma_mu) U_mu(x) psi(x+mu) + (1 + gamma_mu) U_mu(x-mu)^+ psi(x-mu),
// one output parity per launch.  Site block A = a + i mubar gamma5 tau3 - epsbar tau1
// and its closed-form inverse (a - i mubar gamma5 tau3 + epsbar tau1)/(a^2+mubar^2-epsbar^2)
// are applied in the epilogue, as is Gamma5 x tau1 for Q = Gamma5 tau1 (A - H_oe A^-1 H_eo/4).
//
// Work decomposition: two threads per output site, one per flavour; both read
// the same link (one cache line), each reads only its flavour of the
// neighbour spinors, and the flavour-mixing site terms exchange values with
// the partner lane (lane ^ 1).  The spin projection (1 -+ gamma_mu) halves the
// colour matrix-vector work (chiral basis, gamma_0 = [[0,-1],[-1,0]],
// gamma_k = [[0,-i s_k],[i s_k,0]]).  Blocks are remapped so that each of the 8
// XCDs (block b runs on XCD b mod 8) sweeps one contiguous slab of the lattice,
// which keeps neighbour re-reads inside that XCD's L2.
#include <type_traits>

#include "ndtm_internal.h"

namespace ndtm {
namespace {

template <class R>
struct cx {
  R x, y;
};
template <class R>
__device__ __forceinline__ cx<R> operator+(cx<R> a, cx<R> b) { return {a.x + b.x, a.y + b.y}; }
template <class R>
__device__ __forceinline__ cx<R> operator-(cx<R> a, cx<R> b) { return {a.x - b.x, a.y - b.y}; }
template <class R>
__device__ __forceinline__ cx<R> operator*(R s, cx<R> a) { return {s * a.x, s * a.y}; }
template <class R>
__device__ __forceinline__ cx<R> mul(cx<R> a, cx<R> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <class R>
__device__ __forceinline__ cx<R> mulc(cx<R> a, cx<R> b) {  // conj(a) * b
  return {a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x};
}
// s + a b and s + conj(a) b with explicit fused multiply-adds
__device__ __forceinline__ double fmad(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fmad(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
template <class R>
__device__ __forceinline__ cx<R> cmac(cx<R> s, cx<R> a, cx<R> b) {
  return {fmad(-a.y, b.y, fmad(a.x, b.x, s.x)), fmad(a.y, b.x, fmad(a.x, b.y, s.y))};
}
template <class R>
__device__ __forceinline__ cx<R> cmacc(cx<R> s, cx<R> a, cx<R> b) {
  return {fmad(a.y, b.y, fmad(a.x, b.x, s.x)), fmad(-a.y, b.x, fmad(a.x, b.y, s.y))};
}
template <class R>
__device__ __forceinline__ cx<R> ipl(cx<R> a) { return {-a.y, a.x}; }  // i a
template <class R>
__device__ __forceinline__ cx<R> imi(cx<R> a) { return {a.y, -a.x}; }  // -i a
template <class R>
__device__ __forceinline__ cx<R> shfl1(cx<R> v) {
  return {__shfl_xor(v.x, 1), __shfl_xor(v.y, 1)};
}

template <class S>
struct RealOf;
template <>
struct RealOf<double2> { using T = double; };
template <>
struct RealOf<float2> { using T = float; };
template <>
struct RealOf<__half2> { using T = float; };
template <class S>
constexpr bool kHalf = std::is_same<S, __half2>::value;

// Streaming accesses (links, the site's own vectors, the output): each element
// is touched once per pass, so they are loaded/stored non-temporally and leave
// the L2 to the neighbour spinors, which are read eight times.
typedef double v2d __attribute__((ext_vector_type(2)));
typedef float v2f __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void stc_nt(double2* p, cx<double> v) {
  v2d w = {v.x, v.y};
  __builtin_nontemporal_store(w, reinterpret_cast<v2d*>(p));
}
__device__ __forceinline__ void stc_nt(float2* p, cx<float> v) {
  v2f w = {v.x, v.y};
  __builtin_nontemporal_store(w, reinterpret_cast<v2f*>(p));
}
__device__ __forceinline__ void stc_nt(__half2* p, cx<float> v) {
  union {
    unsigned u;
    __half2 h;
  } w;
  w.h = __float22half2_rn(make_float2(v.x, v.y));
  __builtin_nontemporal_store(w.u, reinterpret_cast<unsigned*>(p));
}

template <class S, class L>
struct HopArgs {
  const S* in;
  const float* in_sc;
  const L* Uo;
  const L* Ui;
  S* out;
  float* out_sc;
  const S* xs;
  const float* xs_sc;
  const S* zs;
  const float* zs_sc;
  double* partials;
  const double* skip;
  // clover site blocks of the output parity (packed Hermitian 6x6 per chirality, component
  // arrays of `stride` entries in the arithmetic precision): M = a + C (72 arrays) and, for
  // the even parity, N and M N (144 arrays); null without the clover term
  const typename RealOf<S>::T* clm;
  const typename RealOf<S>::T* clinv;
  int T, Lz, Ly, Lx, vh, stride, parity, antiperiodic;
  int bz, by;  // (z, y) tile of the traversal order (divide Lz, Ly); x rows are whole
  double a, mubar, epsbar, inv_den, ms, hop_coef, sigma;
};

__device__ __forceinline__ double2 ld_nt(const double2* p) {
  const v2d v = __builtin_nontemporal_load(reinterpret_cast<const v2d*>(p));
  return make_double2(v.x, v.y);
}
__device__ __forceinline__ float2 ld_nt(const float2* p) {
  const v2f v = __builtin_nontemporal_load(reinterpret_cast<const v2f*>(p));
  return make_float2(v.x, v.y);
}
__device__ __forceinline__ __half2 ld_nt(const __half2* p) {
  union {
    unsigned u;
    __half2 h;
  } w;
  w.u = __builtin_nontemporal_load(reinterpret_cast<const unsigned*>(p));
  return w.h;
}
__device__ __forceinline__ cx<double> cvt(double2 v) { return {v.x, v.y}; }
__device__ __forceinline__ cx<float> cvt(float2 v) { return {v.x, v.y}; }
__device__ __forceinline__ cx<float> cvt(__half2 v) {
  const float2 f = __half22float2(v);
  return {f.x, f.y};
}

// Address of component array k (a uniform base, kept in scalar registers)
// plus a per-lane byte offset below 4 GiB: the loads then take the
// scalar-base + 32-bit-offset form and need no per-load address arithmetic.
template <class T>
__device__ __forceinline__ const T* at(const T* base, long comp_elems, unsigned off_bytes) {
  return reinterpret_cast<const T*>(reinterpret_cast<const char*>(base + comp_elems) + off_bytes);
}
template <class T>
__device__ __forceinline__ T* at(T* base, long comp_elems, unsigned off_bytes) {
  return reinterpret_cast<T*>(reinterpret_cast<char*>(base + comp_elems) + off_bytes);
}
// byte offset of flavour f of half-site h in a [24][stride] field
template <class S>
__device__ __forceinline__ unsigned flav_off(int f, int stride, int h) {
  return (unsigned)(f * 12 * stride + h) * (unsigned)sizeof(S);
}

// FP32 and FP16 fields: G = 16/sizeof(S) components per 16-byte word
// (idx32/idx16, lidx32/lidx16 layouts); group g of flavour f at half-site h is
// word (f*NG + g)*stride + h with NG = 12/G groups per flavour.
template <class S>
constexpr bool kGrouped = !std::is_same<S, double2>::value;
template <class S>
constexpr int kG = 16 / (int)sizeof(S);
typedef unsigned v4u __attribute__((ext_vector_type(4)));
template <class S>
union Grp {
  v4u w;
  S e[16 / sizeof(S)];
};
template <bool NT, class S>
__device__ __forceinline__ Grp<S> ld_group(const S* base, long group, int stride, unsigned off_bytes) {
  const v4u* q =
      reinterpret_cast<const v4u*>(reinterpret_cast<const char*>(base + group * stride * kG<S>) + off_bytes);
  Grp<S> u;
  if constexpr (NT) u.w = __builtin_nontemporal_load(q);
  else u.w = *q;
  return u;
}
template <class S>
__device__ __forceinline__ unsigned group_off(int f, int stride, int h) {
  return (unsigned)(f * (12 / kG<S>)*stride + h) * 16u;
}

// Loads the 12 components (4 spins x 3 colours) of flavour f at site h.
template <class S, class R, bool NT = false>
__device__ __forceinline__ void load_flav(cx<R> (&v)[4][3], const S* p, const float* sc, int f,
                                          int stride, int h) {
  if constexpr (kGrouped<S>) {
    constexpr int G = kG<S>;
    R s = 1;
    if constexpr (kHalf<S>) s = sc[h];
    const unsigned vo = group_off<S>(f, stride, h);
#pragma unroll
    for (int g = 0; g < 12 / G; ++g) {
      const Grp<S> u = ld_group<NT>(p, g, stride, vo);
#pragma unroll
      for (int q = 0; q < G; ++q) {
        cx<R> t = cvt(u.e[q]);
        if constexpr (kHalf<S>) t = s * t;
        v[(G * g + q) / 3][(G * g + q) % 3] = t;
      }
    }
  } else {
    const unsigned vo = flav_off<S>(f, stride, h);
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const S* q = at(p, (long)(sp * 3 + c) * stride, vo);
        if constexpr (NT) v[sp][c] = cvt(ld_nt(q));
        else v[sp][c] = cvt(*q);
      }
  }
}

// y = H u for one chirality chi of v (spins 2 chi, 2 chi + 1), H a packed Hermitian 6x6
// (6 real diagonal entries, then the upper entries row by row as re, im) stored as
// component arrays starting at comp0.
template <class R, class CT>
__device__ __forceinline__ void herm6(const CT* base, int stride, int h, int comp0, const cx<R> (&v)[4][3], int chi,
                                      cx<R> (&y)[6]) {
  cx<R> u[6];
#pragma unroll
  for (int q = 0; q < 2; ++q)
#pragma unroll
    for (int c = 0; c < 3; ++c) u[q * 3 + c] = v[2 * chi + q][c];
  const unsigned off = (unsigned)h * (unsigned)sizeof(CT);
#pragma unroll
  for (int i = 0; i < 6; ++i) y[i] = R(*at(base, (long)(comp0 + i) * stride, off)) * u[i];
  int k = 6;
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int j = i + 1; j < 6; ++j, k += 2) {
      const cx<R> e = {R(*at(base, (long)(comp0 + k) * stride, off)), R(*at(base, (long)(comp0 + k + 1) * stride, off))};
      y[i] = cmac(y[i], e, u[j]);
      y[j] = cmacc(y[j], e, u[i]);
    }
}

// sin and cos of an angle in [-pi, pi] in FP64, for the eight-parameter links: the
// angle is reduced by the nearest multiple k of pi/2 (pi/2 split in two parts, so
// the remainder |r| <= pi/4 is exact to rounding), then the Taylor series of sin r
// (to r^15) and cos r (to r^16), whose truncation errors stay below 1e-16 at pi/4,
// and the quadrant k mod 4 selects and signs them.  Small in registers, unlike a
// general-purpose sincos with its reduction for large arguments.
__device__ __forceinline__ void sincos_pi(double x, double* sn, double* cs) {
  const double k = rint(x * 0.63661977236758134308);
  const double r = fma(-k, 6.123233995736766e-17, fma(-k, 1.5707963267948966, x));
  const double r2 = r * r;
  // coefficients (-1)^n / (2n+1)! and (-1)^n / (2n)!, n >= 1
  const double ps = fma(fma(fma(fma(fma(fma(-7.647163731819816e-13, r2, 1.6059043836821613e-10), r2, -2.505210838544172e-08), r2, 2.7557319223985893e-06), r2, -0.0001984126984126984), r2, 0.008333333333333333), r2, -0.16666666666666666);
  const double pc = fma(fma(fma(fma(fma(fma(fma(4.779477332387385e-14, r2, -1.1470745597729725e-11), r2, 2.08767569878681e-09), r2, -2.755731922398589e-07), r2, 2.48015873015873e-05), r2, -0.001388888888888889), r2, 0.041666666666666664), r2, -0.5);
  const double sr = fma(r * r2, ps, r), cr = fma(r2, pc, 1.0);
  const int q = (int)k & 3;
  *sn = q == 0 ? sr : q == 1 ? cr : q == 2 ? -sr : -cr;
  *cs = q == 0 ? cr : q == 1 ? -sr : q == 2 ? -cr : sr;
}

// sin and cos of the two phases of one eight-parameter link.  Kept out of line: inlined
// into the eight hops, the compiler scheduled all sixteen evaluations together and the
// FP64 stencil spilled to scratch at one wave per SIMD; as a call it runs at three.
struct SinCos2 {
  double s0, c0, s1, c1;
};
__device__ __noinline__ SinCos2 sincos_pair(double x0, double x1) {
  SinCos2 r;
  sincos_pi(x0, &r.s0, &r.c0);
  sincos_pi(x1, &r.s1, &r.c1);
  return r;
}

// Raw operands of one hop in storage precision: the neighbour spinor of the
// lane's flavour (12 complex), its scale (FP16 only) and the link (9 complex).
// Loading them is split from the arithmetic so that the loads of the next
// hop are in flight while the current one is computed (two buffers).
template <class S, class L>
struct Raw {
  S p[12];
  L u[9];
  float sc;
};

// The link of one hop in storage precision at half-site hl of link array U: rows 0-1
// (components 0..5) always, row 2 too without R12 (then rebuilt in hop_compute); R8
// (FP64, SU(3) links): U points at the eight-parameter arrays, four complex words per
// link (see launch_pack_r8).  The links group by their own storage (FP32 links with FP32
// fields, FP16 links with FP16 or FP32 fields).
template <int MU, bool R12, bool R8, class S, class L>
__device__ __forceinline__ void load_link(Raw<S, L>& r, const L* U, int stride, int hl) {
  if constexpr (kGrouped<S>) {
    const unsigned vl = (unsigned)hl * 16u;
    constexpr int GL = kG<L>;
    constexpr int NLG = R12 ? (6 + GL - 1) / GL : 8 / GL;
#pragma unroll
    for (int g = 0; g < NLG; ++g) {
      const Grp<L> u = ld_group<true>(U, (8 / GL) * MU + g, stride, vl);
#pragma unroll
      for (int q = 0; q < GL; ++q)
        if (GL * g + q < 9) r.u[GL * g + q] = u.e[q];
    }
    if constexpr (!R12) r.u[8] = ld_nt(at(U, (long)(32 + MU) * stride, (unsigned)hl * (unsigned)sizeof(L)));
  } else {
    const unsigned vl = (unsigned)hl * (unsigned)sizeof(L);
    if constexpr (R8) {
#pragma unroll
      for (int k = 0; k < 4; ++k) r.u[k] = ld_nt(at(U, (long)(MU * 4 + k) * stride, vl));
    } else {
#pragma unroll
      for (int k = 0; k < (R12 ? 6 : 9); ++k) r.u[k] = ld_nt(at(U, (long)(MU * 9 + k) * stride, vl));
    }
  }
}

template <int MU, bool R12, bool R8, class S, class L>
__device__ __forceinline__ void load_raw(Raw<S, L>& r, const HopArgs<S, L>& A, int f, int hn, const L* U,
                                         int hl) {
  if constexpr (kGrouped<S>) {
    constexpr int G = kG<S>;
    const unsigned vo = group_off<S>(f, A.stride, hn);
#pragma unroll
    for (int g = 0; g < 12 / G; ++g) {
      const Grp<S> u = ld_group<false>(A.in, g, A.stride, vo);
#pragma unroll
      for (int q = 0; q < G; ++q) r.p[G * g + q] = u.e[q];
    }
    if constexpr (kHalf<S>) r.sc = A.in_sc[hn];
  } else {
    const unsigned vo = flav_off<S>(f, A.stride, hn);
#pragma unroll
    for (int k = 0; k < 12; ++k) r.p[k] = *at(A.in, (long)k * A.stride, vo);
  }
  load_link<MU, R12, R8>(r, U, A.stride, hl);
}

// One of the eight hops: project, colour-multiply, reconstruct, accumulate.
// SIGN: the hop carries the sign sg of an antiperiodic time boundary; the
// FP16 spinor scale and sg multiply the colour products once, at the end.
template <int MU, bool FWD, bool SIGN, bool R12, bool R8, class S, class L, class R>
__device__ __forceinline__ void hop_compute(cx<R> (&acc)[4][3], const Raw<S, L>& raw, R sg) {
  cx<R> p[4][3];
#pragma unroll
  for (int sp = 0; sp < 4; ++sp)
#pragma unroll
    for (int c = 0; c < 3; ++c) p[sp][c] = cvt(raw.p[sp * 3 + c]);
  cx<R> h0[3], h1[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    if constexpr (MU == 0) {
      h0[c] = FWD ? p[0][c] + p[2][c] : p[0][c] - p[2][c];
      h1[c] = FWD ? p[1][c] + p[3][c] : p[1][c] - p[3][c];
    } else if constexpr (MU == 1) {
      h0[c] = FWD ? p[0][c] + ipl(p[3][c]) : p[0][c] - ipl(p[3][c]);
      h1[c] = FWD ? p[1][c] + ipl(p[2][c]) : p[1][c] - ipl(p[2][c]);
    } else if constexpr (MU == 2) {
      h0[c] = FWD ? p[0][c] + p[3][c] : p[0][c] - p[3][c];
      h1[c] = FWD ? p[1][c] - p[2][c] : p[1][c] + p[2][c];
    } else {
      h0[c] = FWD ? p[0][c] + ipl(p[2][c]) : p[0][c] - ipl(p[2][c]);
      h1[c] = FWD ? p[1][c] - ipl(p[3][c]) : p[1][c] + ipl(p[3][c]);
    }
  }
  cx<R> u[3][3];
  if constexpr (R8) {
    // eight parameters: a = (U01, U02) and the kept first-column entry exactly, the
    // phases of U00 and of the other first-column entry (+8 marks that U20 was kept);
    // |U00| and the other entry's magnitude from the row and column norms (both equal
    // 1 - |a|^2 off the corner), and with c = (U10, U20)^T, u = U00, n = |a|^2 the
    // unitarity and det U = 1 relations give the lower 2x2 block
    //   B = -(1/n) [ (conj c2, -conj c1)^T (conj a2, -conj a1) + conj(u) c a ]
    auto cj = [](cx<R> z) { return cx<R>{z.x, -z.y}; };
    const cx<R> a1 = cvt(raw.u[0]), a2 = cvt(raw.u[1]), ks = cvt(raw.u[2]), th = cvt(raw.u[3]);
    const bool k20 = th.y > R(4);
    const R tho = k20 ? th.y - R(8) : th.y;
    const R n = a1.x * a1.x + a1.y * a1.y + a2.x * a2.x + a2.y * a2.y;
    const R mu = sqrt(fmax(R(1) - n, R(0)));
    const R mo = sqrt(fmax(n - (ks.x * ks.x + ks.y * ks.y), R(0)));
    const SinCos2 sc = sincos_pair(th.x, tho);
    const cx<R> u0 = {mu * sc.c0, mu * sc.s0}, oth = {mo * sc.c1, mo * sc.s1};
    const cx<R> c1 = k20 ? oth : ks, c2 = k20 ? ks : oth;
    const cx<R> uc = cj(u0);
    const R in = R(1) / n;
    u[0][0] = u0;
    u[0][1] = a1;
    u[0][2] = a2;
    u[1][0] = c1;
    u[2][0] = c2;
    u[1][1] = (-in) * (cj(mul(c2, a2)) + mul(uc, mul(c1, a1)));
    u[1][2] = in * (cj(mul(c2, a1)) - mul(uc, mul(c1, a2)));
    u[2][1] = in * (cj(mul(c1, a2)) - mul(uc, mul(c2, a1)));
    u[2][2] = (-in) * (cj(mul(c1, a1)) + mul(uc, mul(c2, a2)));
  } else {
#pragma unroll
  for (int r = 0; r < (R12 ? 2 : 3); ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) u[r][c] = cvt(raw.u[r * 3 + c]);
  }
  if constexpr (R12 && !R8) {
    // SU(3): row 2 = conj(row 0 x row 1)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int a = (c + 1) % 3, b = (c + 2) % 3;
      const cx<R> x = mul(u[0][a], u[1][b]) - mul(u[0][b], u[1][a]);
      u[2][c] = {x.x, -x.y};
    }
  }
  cx<R> g0[3], g1[3];
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    cx<R> s0, s1;
    if constexpr (FWD) {
      s0 = mul(u[r][0], h0[0]);
      s1 = mul(u[r][0], h1[0]);
#pragma unroll
      for (int c = 1; c < 3; ++c) {
        s0 = cmac(s0, u[r][c], h0[c]);
        s1 = cmac(s1, u[r][c], h1[c]);
      }
    } else {
      s0 = mulc(u[0][r], h0[0]);
      s1 = mulc(u[0][r], h1[0]);
#pragma unroll
      for (int c = 1; c < 3; ++c) {
        s0 = cmacc(s0, u[c][r], h0[c]);
        s1 = cmacc(s1, u[c][r], h1[c]);
      }
    }
    if constexpr (kHalf<S> || SIGN) {
      R fac = 1;
      if constexpr (kHalf<S>) fac = R(raw.sc);
      if constexpr (SIGN) fac *= sg;
      s0 = fac * s0;
      s1 = fac * s1;
    }
    g0[r] = s0;
    g1[r] = s1;
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    acc[0][c] = acc[0][c] + g0[c];
    acc[1][c] = acc[1][c] + g1[c];
    if constexpr (MU == 0) {
      acc[2][c] = FWD ? acc[2][c] + g0[c] : acc[2][c] - g0[c];
      acc[3][c] = FWD ? acc[3][c] + g1[c] : acc[3][c] - g1[c];
    } else if constexpr (MU == 1) {
      acc[2][c] = FWD ? acc[2][c] + imi(g1[c]) : acc[2][c] + ipl(g1[c]);
      acc[3][c] = FWD ? acc[3][c] + imi(g0[c]) : acc[3][c] + ipl(g0[c]);
    } else if constexpr (MU == 2) {
      acc[2][c] = FWD ? acc[2][c] - g1[c] : acc[2][c] + g1[c];
      acc[3][c] = FWD ? acc[3][c] + g0[c] : acc[3][c] - g0[c];
    } else {
      acc[2][c] = FWD ? acc[2][c] + imi(g0[c]) : acc[2][c] + ipl(g0[c]);
      acc[3][c] = FWD ? acc[3][c] + ipl(g1[c]) : acc[3][c] + imi(g1[c]);
    }
  }
}

__device__ __forceinline__ void block_reduce_store(double v, double* partials) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off);
  __shared__ double ws[kBlock / 64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) ws[w] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0;
#pragma unroll
    for (int i = 0; i < kBlock / 64; ++i) s += ws[i];
    partials[blockIdx.x] = s;
  }
}

// the three RED_MR partials of a block, at partials[q * 2 gridDim + blockIdx]
__device__ __forceinline__ void block_reduce_store3(double v0, double v1, double v2, double* partials) {
  double v[3] = {v0, v1, v2};
  __shared__ double ws3[3][kBlock / 64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < 3; ++q) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v[q] += __shfl_down(v[q], off);
    if (lane == 0) ws3[q][w] = v[q];
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    double s = 0;
#pragma unroll
    for (int i = 0; i < kBlock / 64; ++i) s += ws3[threadIdx.x][i];
    partials[(size_t)threadIdx.x * 2 * gridDim.x + blockIdx.x] = s;
  }
}

template <class S, class L, int EPI, int RED, bool R12, bool CLV, bool R8 = false>
__global__ __launch_bounds__(kBlock) void hop_kernel(HopArgs<S, L> A) {
  using R = typename RealOf<S>::T;
  if (A.skip && *A.skip != 0.0) return;
  // XCD-aware block order: XCD k = b % 8 gets one contiguous range of logical blocks.
  const int nb = gridDim.x, b = blockIdx.x;
  const int q = nb >> 3, rem = nb & 7, xcd = b & 7, loc = b >> 3;
  const int lb = xcd * q + min(xcd, rem) + loc;
  const int f = threadIdx.x & 1;
  // traversal order: (z, y) tiles of bz x by whole x rows outermost (y tiles fastest),
  // each marched through t, then z, y, x within the tile.  A site's t-neighbours are
  // read two tile slices apart and its z, y neighbours within one, so the window the
  // L2 must hold is a few tile slices instead of a few 3-d slices of the lattice.
  const int o = lb * kSitesPerBlock + (threadIdx.x >> 1);
  const bool valid = o < A.vh;
  const int Lxh = A.Lx >> 1;
  int h = 0, t = 0, z = 0, y = 0, xh = 0;
  {
    const int row = A.by * Lxh, tslice = A.bz * row, tile = A.T * tslice;
    const int k = o / tile, r0 = o - k * tile;
    t = r0 / tslice;
    const int r1 = r0 - t * tslice;
    const int zin = r1 / row, r2 = r1 - zin * row;
    const int yin = r2 / Lxh;
    xh = r2 - yin * Lxh;
    const int nty = A.Ly / A.by;
    const int kz = k / nty, ky = k - kz * nty;
    z = kz * A.bz + zin;
    y = ky * A.by + yin;
    h = ((t * A.Lz + z) * A.Ly + y) * Lxh + xh;
  }
  double red = 0.0, red_im = 0.0, red_tt = 0.0;

  cx<R> acc[4][3];
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int c = 0; c < 3; ++c) acc[s][c] = {0, 0};

  if (valid) {
    const int row = (t * A.Lz + z) * A.Ly + y;
    const int tz = t * A.Lz + z;
    const int x = 2 * xh + ((A.parity + t + z + y) & 1);
    // neighbour half indices
    const int xp = (x + 1 == A.Lx) ? 0 : x + 1;
    const int xm = (x == 0) ? A.Lx - 1 : x - 1;
    const int yp = (y + 1 == A.Ly) ? 0 : y + 1;
    const int ym = (y == 0) ? A.Ly - 1 : y - 1;
    const int zp = (z + 1 == A.Lz) ? 0 : z + 1;
    const int zm = (z == 0) ? A.Lz - 1 : z - 1;
    const int tp = (t + 1 == A.T) ? 0 : t + 1;
    const int tm = (t == 0) ? A.T - 1 : t - 1;
    const int hx_p = row * Lxh + (xp >> 1);
    const int hx_m = row * Lxh + (xm >> 1);
    const int hy_p = (tz * A.Ly + yp) * Lxh + xh;
    const int hy_m = (tz * A.Ly + ym) * Lxh + xh;
    const int hz_p = ((t * A.Lz + zp) * A.Ly + y) * Lxh + xh;
    const int hz_m = ((t * A.Lz + zm) * A.Ly + y) * Lxh + xh;
    const int ht_p = ((tp * A.Lz + z) * A.Ly + y) * Lxh + xh;
    const int ht_m = ((tm * A.Lz + z) * A.Ly + y) * Lxh + xh;
    const R sg_tp = (A.antiperiodic && t == A.T - 1) ? R(-1) : R(1);
    const R sg_tm = (A.antiperiodic && t == 0) ? R(-1) : R(1);
    if constexpr (std::is_same<S, double2>::value) {
      // FP64: the operands of one hop already take ~90 registers; a second
      // buffer would leave one wave per SIMD, so hops are loaded one at a time
      Raw<S, L> r;
      load_raw<0, R12, R8>(r, A, f, ht_p, A.Uo, h);
      hop_compute<0, true, true, R12, R8>(acc, r, sg_tp);
      load_raw<0, R12, R8>(r, A, f, ht_m, A.Ui, ht_m);
      hop_compute<0, false, true, R12, R8>(acc, r, sg_tm);
      load_raw<1, R12, R8>(r, A, f, hx_p, A.Uo, h);
      hop_compute<1, true, false, R12, R8>(acc, r, R(1));
      load_raw<1, R12, R8>(r, A, f, hx_m, A.Ui, hx_m);
      hop_compute<1, false, false, R12, R8>(acc, r, R(1));
      load_raw<2, R12, R8>(r, A, f, hy_p, A.Uo, h);
      hop_compute<2, true, false, R12, R8>(acc, r, R(1));
      load_raw<2, R12, R8>(r, A, f, hy_m, A.Ui, hy_m);
      hop_compute<2, false, false, R12, R8>(acc, r, R(1));
      load_raw<3, R12, R8>(r, A, f, hz_p, A.Uo, h);
      hop_compute<3, true, false, R12, R8>(acc, r, R(1));
      load_raw<3, R12, R8>(r, A, f, hz_m, A.Ui, hz_m);
      hop_compute<3, false, false, R12, R8>(acc, r, R(1));
    } else {
    Raw<S, L> ra, rb;
    load_raw<0, R12, R8>(ra, A, f, ht_p, A.Uo, h);
    load_raw<0, R12, R8>(rb, A, f, ht_m, A.Ui, ht_m);
    hop_compute<0, true, true, R12, R8>(acc, ra, sg_tp);
    load_raw<1, R12, R8>(ra, A, f, hx_p, A.Uo, h);
    hop_compute<0, false, true, R12, R8>(acc, rb, sg_tm);
    load_raw<1, R12, R8>(rb, A, f, hx_m, A.Ui, hx_m);
    hop_compute<1, true, false, R12, R8>(acc, ra, R(1));
    load_raw<2, R12, R8>(ra, A, f, hy_p, A.Uo, h);
    hop_compute<1, false, false, R12, R8>(acc, rb, R(1));
    load_raw<2, R12, R8>(rb, A, f, hy_m, A.Ui, hy_m);
    hop_compute<2, true, false, R12, R8>(acc, ra, R(1));
    load_raw<3, R12, R8>(ra, A, f, hz_p, A.Uo, h);
    hop_compute<2, false, false, R12, R8>(acc, rb, R(1));
    load_raw<3, R12, R8>(rb, A, f, hz_m, A.Ui, hz_m);
    hop_compute<3, true, false, R12, R8>(acc, ra, R(1));
    hop_compute<3, false, false, R12, R8>(acc, rb, R(1));
    }
  }

  // ---- epilogue (both lanes of a site are valid or invalid together) ----
  const R a = R(A.a), mub = R(A.mubar), eps = R(A.epsbar);
  const R t3 = f == 0 ? R(1) : R(-1);
  cx<R> out[4][3];
  if constexpr (EPI == EPI_PLAIN) {
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int c = 0; c < 3; ++c) out[s][c] = acc[s][c];
  } else if constexpr (EPI == EPI_AINV && CLV) {
    // A^-1 acc with the clover term: M N acc_f - i mubar g5 tau3 N acc_f + epsbar N acc_{1-f}
#pragma unroll
    for (int chi = 0; chi < 2; ++chi) {
      cx<R> nu[6], mnu[6];
      if (valid) {
        herm6(A.clinv, A.stride, h, 36 * chi, acc, chi, nu);
        herm6(A.clinv, A.stride, h, 72 + 36 * chi, acc, chi, mnu);
      } else {
#pragma unroll
        for (int i = 0; i < 6; ++i) nu[i] = mnu[i] = {0, 0};
      }
      const R g5 = chi == 0 ? R(1) : R(-1);
#pragma unroll
      for (int i = 0; i < 6; ++i) {
        const cx<R> o = shfl1(nu[i]);
        out[2 * chi + i / 3][i % 3] = mnu[i] - (mub * g5 * t3) * ipl(nu[i]) + eps * o;
      }
    }
  } else if constexpr (EPI == EPI_AINV) {
    const R id = R(A.inv_den);
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const R g5 = s < 2 ? R(1) : R(-1);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const cx<R> o = shfl1(acc[s][c]);
        // (a - i mubar g5 tau3) acc_f + epsbar acc_{1-f}
        out[s][c] = id * (a * acc[s][c] - (mub * g5 * t3) * ipl(acc[s][c]) + eps * o);
      }
    }
  } else {
    cx<R> xv[4][3];
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int c = 0; c < 3; ++c) xv[s][c] = {0, 0};
    if (valid) load_flav<S, R, true>(xv, A.xs, A.xs_sc, f, A.stride, h);
    const R hc = (EPI == EPI_QHAT || EPI == EPI_QHAT_SIG) ? R(-0.25) : R(A.hop_coef);
    const R ms = R(A.ms);
    // the site's own term a x, or M x = (a + C) x with the clover term
    cx<R> mx[4][3];
    if constexpr (CLV) {
#pragma unroll
      for (int chi = 0; chi < 2; ++chi) {
        cx<R> y6[6];
        if (valid) {
          herm6(A.clm, A.stride, h, 36 * chi, xv, chi, y6);
        } else {
#pragma unroll
          for (int i = 0; i < 6; ++i) y6[i] = {0, 0};
        }
#pragma unroll
        for (int i = 0; i < 6; ++i) mx[2 * chi + i / 3][i % 3] = y6[i];
      }
    } else {
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int c = 0; c < 3; ++c) mx[s][c] = a * xv[s][c];
    }
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const R g5 = s < 2 ? R(1) : R(-1);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const cx<R> xo = shfl1(xv[s][c]);
        // y_f = M x_f + i mubar g5 tau3 x_f - epsbar x_{1-f} + hc acc_f (+ i ms g5 x_{1-f})
        cx<R> y = mx[s][c] + (mub * g5 * t3) * ipl(xv[s][c]) - eps * xo + hc * acc[s][c];
        if constexpr (EPI == EPI_SITE || EPI == EPI_SITE_Q) y = y + (ms * g5) * ipl(xo);
        out[s][c] = y;
      }
    }
    if constexpr (RED == RED_MR) {
      // <out, x> and ||out||^2, x the site vector just read (zero off the lattice)
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const double ox = double(out[s][c].x), oy = double(out[s][c].y);
          const double xx = double(xv[s][c].x), xy = double(xv[s][c].y);
          red += ox * xx + oy * xy;
          red_im += ox * xy - oy * xx;
          red_tt += valid ? ox * ox + oy * oy : 0.0;
        }
    }
    if constexpr (EPI == EPI_QHAT || EPI == EPI_QHAT_SIG || EPI == EPI_SITE_Q) {
      // Gamma5 tau1: out_f = g5 y_{1-f}
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const R g5 = s < 2 ? R(1) : R(-1);
#pragma unroll
        for (int c = 0; c < 3; ++c) out[s][c] = g5 * shfl1(out[s][c]);
      }
    }
    if constexpr (EPI == EPI_QHAT_SIG) {
      cx<R> zv[4][3];
      if (valid) {
        load_flav<S, R, true>(zv, A.zs, A.zs_sc, f, A.stride, h);
        const R sgm = R(A.sigma);
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
          for (int c = 0; c < 3; ++c) out[s][c] = out[s][c] + sgm * zv[s][c];
        if constexpr (RED == RED_REDOT) {
#pragma unroll
          for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int c = 0; c < 3; ++c)
              red += double(zv[s][c].x) * double(out[s][c].x) + double(zv[s][c].y) * double(out[s][c].y);
        }
      }
    }
  }

  if constexpr (RED == RED_NORM) {
    if (valid) {
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int c = 0; c < 3; ++c)
          red += double(out[s][c].x) * double(out[s][c].x) + double(out[s][c].y) * double(out[s][c].y);
    }
  }

  // ---- store ----
  R inv_sc = 1;
  if constexpr (kHalf<S>) {
    R mx = 0;
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int c = 0; c < 3; ++c) mx = fmaxf(mx, fmaxf(fabsf(out[s][c].x), fabsf(out[s][c].y)));
    mx = fmaxf(mx, __shfl_xor(mx, 1));
    inv_sc = mx > 0 ? R(1) / mx : R(0);
    if (valid && f == 0) A.out_sc[h] = mx;
  }
  if (valid) {
    if constexpr (kGrouped<S>) {
      constexpr int G = kG<S>;
      const unsigned vout = group_off<S>(f, A.stride, h);
#pragma unroll
      for (int g = 0; g < 12 / G; ++g) {
        Grp<S> u;
#pragma unroll
        for (int q = 0; q < G; ++q) {
          const cx<R> o = inv_sc * out[(G * g + q) / 3][(G * g + q) % 3];
          if constexpr (kHalf<S>) u.e[q] = __float22half2_rn(make_float2(o.x, o.y));
          else u.e[q] = make_float2(o.x, o.y);
        }
        v4u* dst = reinterpret_cast<v4u*>(reinterpret_cast<char*>(A.out + (long)g * A.stride * G) + vout);
        __builtin_nontemporal_store(u.w, dst);
      }
    } else {
      const unsigned vout = flav_off<S>(f, A.stride, h);
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int c = 0; c < 3; ++c) stc_nt(at(A.out, (long)(s * 3 + c) * A.stride, vout), out[s][c]);
    }
  }
  if constexpr (RED == RED_MR) block_reduce_store3(red, red_im, red_tt, A.partials);
  else if constexpr (RED != RED_NONE) block_reduce_store(red, A.partials);
}

// Largest divisor bz of Lz whose bz-plane window of input spinors (the reuse
// distance of the t-neighbours) stays within 3 MB of an XCD's 4 MB L2 (a sweep of
// (z, y) tiles at 96x48^3 found whole-plane chunks of 6 planes best, within 1% of
// the best y-split tiles).
int hop_chunk(const Geom& g, int site_bytes) {
  const double plane = (double)g.Ly * (g.Lx / 2);
  const double budget = 3.0 * 1024.0 * 1024.0;
  int bz = g.Lz;
  while (bz > 1 && (g.Lz % bz != 0 || bz * plane * site_bytes > budget)) --bz;
  return bz;
}

template <class S, class L>
void launch_typed(int epi, int red, const Geom& g, int parity, const OpParams& op, const void* Uo,
                  const void* Ui, const HalfField& in, const HalfField& out, const HalfField* xs,
                  const HalfField* zs, double ms, double hop_coef, double sigma, double* partials,
                  hipStream_t st) {
  HopArgs<S, L> A;
  A.in = static_cast<const S*>(in.v);
  A.in_sc = in.sc;
  A.Uo = static_cast<const L*>(Uo);
  A.Ui = static_cast<const L*>(Ui);
  A.out = static_cast<S*>(out.v);
  A.out_sc = out.sc;
  A.xs = xs ? static_cast<const S*>(xs->v) : nullptr;
  A.xs_sc = xs ? xs->sc : nullptr;
  A.zs = zs ? static_cast<const S*>(zs->v) : nullptr;
  A.zs_sc = zs ? zs->sc : nullptr;
  A.partials = partials;
  A.skip = op.skip;
  using CT = typename RealOf<S>::T;
  const int cp = std::is_same<S, double2>::value ? 0 : 1;
  A.clm = static_cast<const CT*>(op.clv_m[cp][parity]);
  A.clinv = parity == 0 ? static_cast<const CT*>(op.clv_inv[cp]) : nullptr;
  const bool clv = op.clover != 0;
  A.T = g.T;
  A.Lz = g.Lz;
  A.Ly = g.Ly;
  A.Lx = g.Lx;
  A.vh = g.vh;
  A.stride = g.stride;
  A.parity = parity;
  A.antiperiodic = g.antiperiodic;
  A.bz = op.chunk > 0 ? op.chunk : hop_chunk(g, sizeof(S) * 24 + (kHalf<S> ? 4 : 0));
  A.by = op.chunk_y > 0 ? op.chunk_y : g.Ly;
  A.a = op.a;
  A.mubar = op.mubar;
  A.epsbar = op.epsbar;
  A.inv_den = op.inv_den;
  A.ms = ms;
  A.hop_coef = hop_coef;
  A.sigma = sigma;
  const dim3 grid(hop_grid(g)), block(kBlock);
  // FP64 with SU(3) links in eight parameters: the link pointers go to those arrays
  constexpr bool kF64 = std::is_same<S, double2>::value;
  const bool r8 = kF64 && op.recon12 && op.u8[parity] && op.u8[1 - parity];
  if (r8) {
    A.Uo = reinterpret_cast<const L*>(op.u8[parity]);
    A.Ui = reinterpret_cast<const L*>(op.u8[1 - parity]);
  }
#define NDTM_HOP(E, RD)                                                                         \
  do {                                                                                          \
    if (clv && E != EPI_PLAIN) {                                                                \
      if constexpr (kF64) if (r8) { hipLaunchKernelGGL((hop_kernel<S, L, E, RD, true, true, true>), grid, block, 0, st, A); break; } \
      if (op.recon12) hipLaunchKernelGGL((hop_kernel<S, L, E, RD, true, true>), grid, block, 0, st, A);   \
      else hipLaunchKernelGGL((hop_kernel<S, L, E, RD, false, true>), grid, block, 0, st, A);             \
    } else {                                                                                    \
      if constexpr (kF64) if (r8) { hipLaunchKernelGGL((hop_kernel<S, L, E, RD, true, false, true>), grid, block, 0, st, A); break; } \
      if (op.recon12) hipLaunchKernelGGL((hop_kernel<S, L, E, RD, true, false>), grid, block, 0, st, A);  \
      else hipLaunchKernelGGL((hop_kernel<S, L, E, RD, false, false>), grid, block, 0, st, A);            \
    }                                                                                           \
  } while (0)
  switch (epi) {
    case EPI_PLAIN: NDTM_HOP(EPI_PLAIN, RED_NONE); break;
    case EPI_AINV: NDTM_HOP(EPI_AINV, RED_NONE); break;
    case EPI_QHAT:
      if (red == RED_NORM) NDTM_HOP(EPI_QHAT, RED_NORM);
      else NDTM_HOP(EPI_QHAT, RED_NONE);
      break;
    case EPI_QHAT_SIG:
      if (red == RED_REDOT) NDTM_HOP(EPI_QHAT_SIG, RED_REDOT);
      else NDTM_HOP(EPI_QHAT_SIG, RED_NONE);
      break;
    case EPI_SITE:
      if (red == RED_MR) NDTM_HOP(EPI_SITE, RED_MR);
      else NDTM_HOP(EPI_SITE, RED_NONE);
      break;
    case EPI_SITE_Q:
      NDTM_HOP(EPI_SITE_Q, RED_NONE);
      break;
  }
#undef NDTM_HOP
}

// ---- Schwarz alternating procedure (section 3's smoother): block solves of one colour ----
// One work-group per block of the given colour, two lanes per site (one per flavour) as in
// the stencil.  The block's residual s_B stays in LDS while mr_iters minimal-residual steps
//   q = D'_B s_B,  w = <q, s_B> / <q, q>,  e += w s_B,  s_B -= w q
// run on it, with D'_B the full-lattice operator D' = a + i mubar g5 tau3 - epsbar tau1 +
// hop_coef H (+ i ms g5 tau1 on odd sites) restricted to the block: hops that leave the
// block are dropped.  Then z += e at the block's sites.  The blocks of one colour do not
// touch each other (the block grid has even extents), so they run side by side.
//
// Block extents are even, so a block starts on an even site and holds NS/2 sites of each
// parity.  The work-group takes the even sites first, then the odd ones (local half-site
// order, x fastest): every wavefront then serves one parity, and the link arrays and fields
// of that parity are wave-uniform (scalar base plus a 32-bit lane offset, as in the stencil).

template <class S, class L>
struct SapArgs {
  const S* s[2];  // residual, parity halves
  S* z[2];        // iterate, parity halves
  const L* U[2];  // links per parity (nine components, or two rows with R12)
  int Lz, Ly, Lx, stride;
  int bt, bz, by, bx;
  int nbz, nby, nbxh;  // blocks per direction in z and y; half the blocks in x
  int colour, mr_iters;
  double a, mubar, epsbar, ms, hop_coef;
};

template <class R, class S>
__device__ __forceinline__ S to_store(cx<R> v) {
  if constexpr (std::is_same<S, double2>::value) return make_double2(v.x, v.y);
  else return make_float2(v.x, v.y);
}

// one hop of the block operator: the neighbour's s_B from LDS, the link from memory
template <int MU, bool FWD, bool R12, int NS, class S, class L, class R>
__device__ __forceinline__ void sap_hop(cx<R> (&acc)[4][3], const S* ls, int f, int jn, const L* U, int stride,
                                        int hl) {
  Raw<S, L> raw;
#pragma unroll
  for (int k = 0; k < 12; ++k) raw.p[k] = ls[(f * 12 + k) * NS + jn];
  raw.sc = 1.0f;
  load_link<MU, R12, false>(raw, U, stride, hl);
  hop_compute<MU, FWD, false, R12, false>(acc, raw, R(1));
}

// the same hop with the link taken from LDS, where the work-group staged the two-row
// links of its block's internal hops (hop d = 2 MU + backward, NLG words of 16 bytes
// each, in lk[(d * NLG + g) * NS + j] for site j)
template <int MU, bool FWD, bool R12, int NS, int NLG, class S, class L, class R>
__device__ __forceinline__ void sap_hop_lds(cx<R> (&acc)[4][3], const S* ls, const v4u* lk, int f, int jn, int j) {
  Raw<S, L> raw;
#pragma unroll
  for (int k = 0; k < 12; ++k) raw.p[k] = ls[(f * 12 + k) * NS + jn];
  raw.sc = 1.0f;
  constexpr int GL = kG<L>, d = 2 * MU + (FWD ? 0 : 1);
#pragma unroll
  for (int g = 0; g < NLG; ++g) {
    Grp<L> u;
    u.w = lk[(d * NLG + g) * NS + j];
#pragma unroll
    for (int q = 0; q < GL; ++q)
      if (GL * g + q < 9) raw.u[GL * g + q] = u.e[q];
  }
  hop_compute<MU, FWD, false, R12, false>(acc, raw, R(1));
}

template <class S, class L, bool R12, int NS>
__global__ __launch_bounds__(2 * NS) void sap_block_kernel(SapArgs<S, L> A) {
  using R = typename RealOf<S>::T;
  // s_B: component k of flavour f at local site j in ls[(f * 12 + k) * NS + j]
  __shared__ S ls[24 * NS];
  __shared__ double wred[3][2 * NS / 64];
  // FP32 fields with two-row FP32 or FP16 links: the links of the block's internal hops are
  // read once into LDS (96 or 64 KB at 256 sites); otherwise every step reads them through
  // the L2
  constexpr bool kStage = kGrouped<S> && R12;
  constexpr int NLG = kStage ? (6 + kG<L> - 1) / kG<L> : 1;
  __shared__ v4u lk[kStage ? 8 * NLG * NS : 1];
  const int f = threadIdx.x & 1, j = threadIdx.x >> 1;
  // the work-group's block among those of this colour, x fastest
  int rest = blockIdx.x;
  const int jx = rest % A.nbxh;
  rest /= A.nbxh;
  const int By = rest % A.nby;
  rest /= A.nby;
  const int Bz = rest % A.nbz, Bt = rest / A.nbz;
  const int Bx = 2 * jx + ((A.colour + Bt + Bz + By) & 1);
  // this lane's site: parity (uniform over the wavefront), then local half-site order
  constexpr int NH = NS / 2;
  const int par = __builtin_amdgcn_readfirstlane(j / NH);
  const int bxh = A.bx >> 1;
  const int jh = j - par * NH;
  const int lxh = jh % bxh, ly = (jh / bxh) % A.by, lz = (jh / (bxh * A.by)) % A.bz;
  const int lt = jh / (bxh * A.by * A.bz);
  const int lx = 2 * lxh + ((lt + lz + ly + par) & 1);
  const int t = Bt * A.bt + lt, z = Bz * A.bz + lz, y = By * A.by + ly, x = Bx * A.bx + lx;
  const int Lxh = A.Lx >> 1;
  auto half = [&](int tt, int zz, int yy, int xx) { return ((tt * A.Lz + zz) * A.Ly + yy) * Lxh + (xx >> 1); };
  const int h = half(t, z, y, x);
  // neighbours inside the block: local index in the other parity's half (-1 outside)
  const int op = (1 - par) * NH;
  auto loc = [&](int a, int b, int c, int d) { return op + ((a * A.bz + b) * A.by + c) * bxh + (d >> 1); };
  const int jtp = lt + 1 < A.bt ? loc(lt + 1, lz, ly, lx) : -1, jtm = lt > 0 ? loc(lt - 1, lz, ly, lx) : -1;
  const int jxp = lx + 1 < A.bx ? loc(lt, lz, ly, lx + 1) : -1, jxm = lx > 0 ? loc(lt, lz, ly, lx - 1) : -1;
  const int jyp = ly + 1 < A.by ? loc(lt, lz, ly + 1, lx) : -1, jym = ly > 0 ? loc(lt, lz, ly - 1, lx) : -1;
  const int jzp = lz + 1 < A.bz ? loc(lt, lz + 1, ly, lx) : -1, jzm = lz > 0 ? loc(lt, lz - 1, ly, lx) : -1;
  const int htm = lt > 0 ? half(t - 1, z, y, x) : 0, hxm = lx > 0 ? half(t, z, y, x - 1) : 0;
  const int hym = ly > 0 ? half(t, z, y - 1, x) : 0, hzm = lz > 0 ? half(t, z - 1, y, x) : 0;
  const L* Uo = par ? A.U[1] : A.U[0];
  const L* Ui = par ? A.U[0] : A.U[1];
  const S* sv = par ? A.s[1] : A.s[0];
  S* zp = par ? A.z[1] : A.z[0];
  if constexpr (kStage) {
    // lane f = 0 stages the four forward links (at its own site), f = 1 the four backward
    // ones (at the neighbours); only hops that stay inside the block are used
    const L* U = f == 0 ? Uo : Ui;
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
      const int jn = f == 0 ? (mu == 0 ? jtp : mu == 1 ? jxp : mu == 2 ? jyp : jzp)
                            : (mu == 0 ? jtm : mu == 1 ? jxm : mu == 2 ? jym : jzm);
      const int hl = f == 0 ? h : (mu == 0 ? htm : mu == 1 ? hxm : mu == 2 ? hym : hzm);
      if (jn >= 0) {
        const int d = 2 * mu + f;
#pragma unroll
        for (int g = 0; g < NLG; ++g)
          lk[(d * NLG + g) * NS + j] = ld_group<true>(U, (8 / kG<L>) * mu + g, A.stride, (unsigned)hl * 16u).w;
      }
    }
  }

  cx<R> r[4][3], e[4][3];
  load_flav<S, R>(r, sv, nullptr, f, A.stride, h);
#pragma unroll
  for (int sp = 0; sp < 4; ++sp)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      e[sp][c] = {0, 0};
      ls[(f * 12 + sp * 3 + c) * NS + j] = to_store<R, S>(r[sp][c]);
    }
  const R a = R(A.a), mub = R(A.mubar), eps = R(A.epsbar), hc = R(A.hop_coef);
  const R ms = par ? R(A.ms) : R(0);
  const R t3 = f == 0 ? R(1) : R(-1);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int it = 0; it < A.mr_iters; ++it) {
    __syncthreads();
    cx<R> acc[4][3];
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
      for (int c = 0; c < 3; ++c) acc[sp][c] = {0, 0};
    if constexpr (kStage) {
      if (jtp >= 0) sap_hop_lds<0, true, R12, NS, NLG, S, L>(acc, ls, lk, f, jtp, j);
      if (jtm >= 0) sap_hop_lds<0, false, R12, NS, NLG, S, L>(acc, ls, lk, f, jtm, j);
      if (jxp >= 0) sap_hop_lds<1, true, R12, NS, NLG, S, L>(acc, ls, lk, f, jxp, j);
      if (jxm >= 0) sap_hop_lds<1, false, R12, NS, NLG, S, L>(acc, ls, lk, f, jxm, j);
      if (jyp >= 0) sap_hop_lds<2, true, R12, NS, NLG, S, L>(acc, ls, lk, f, jyp, j);
      if (jym >= 0) sap_hop_lds<2, false, R12, NS, NLG, S, L>(acc, ls, lk, f, jym, j);
      if (jzp >= 0) sap_hop_lds<3, true, R12, NS, NLG, S, L>(acc, ls, lk, f, jzp, j);
      if (jzm >= 0) sap_hop_lds<3, false, R12, NS, NLG, S, L>(acc, ls, lk, f, jzm, j);
    } else {
      if (jtp >= 0) sap_hop<0, true, R12, NS>(acc, ls, f, jtp, Uo, A.stride, h);
      if (jtm >= 0) sap_hop<0, false, R12, NS>(acc, ls, f, jtm, Ui, A.stride, htm);
      if (jxp >= 0) sap_hop<1, true, R12, NS>(acc, ls, f, jxp, Uo, A.stride, h);
      if (jxm >= 0) sap_hop<1, false, R12, NS>(acc, ls, f, jxm, Ui, A.stride, hxm);
      if (jyp >= 0) sap_hop<2, true, R12, NS>(acc, ls, f, jyp, Uo, A.stride, h);
      if (jym >= 0) sap_hop<2, false, R12, NS>(acc, ls, f, jym, Ui, A.stride, hym);
      if (jzp >= 0) sap_hop<3, true, R12, NS>(acc, ls, f, jzp, Uo, A.stride, h);
      if (jzm >= 0) sap_hop<3, false, R12, NS>(acc, ls, f, jzm, Ui, A.stride, hzm);
    }
    // site terms, then <q, s_B> and <q, q>
    cx<R> q[4][3];
    double v0 = 0.0, v1 = 0.0, v2 = 0.0;
#pragma unroll
    for (int sp = 0; sp < 4; ++sp) {
      const R g5 = sp < 2 ? R(1) : R(-1);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const cx<R> xo = shfl1(r[sp][c]);
        q[sp][c] = a * r[sp][c] + (mub * g5 * t3) * ipl(r[sp][c]) - eps * xo + hc * acc[sp][c] + (ms * g5) * ipl(xo);
        const double qx = double(q[sp][c].x), qy = double(q[sp][c].y);
        const double rx = double(r[sp][c].x), ry = double(r[sp][c].y);
        v0 += qx * rx + qy * ry;
        v1 += qx * ry - qy * rx;
        v2 += qx * qx + qy * qy;
      }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      v0 += __shfl_xor(v0, off);
      v1 += __shfl_xor(v1, off);
      v2 += __shfl_xor(v2, off);
    }
    if (lane == 0) {
      wred[0][wv] = v0;
      wred[1][wv] = v1;
      wred[2][wv] = v2;
    }
    __syncthreads();
    double qs_re = 0.0, qs_im = 0.0, qq = 0.0;
#pragma unroll
    for (int i = 0; i < 2 * NS / 64; ++i) {
      qs_re += wred[0][i];
      qs_im += wred[1][i];
      qq += wred[2][i];
    }
    if (!(qq > 0.0)) break;  // the same sums in every lane: the whole work-group leaves
    const cx<R> w = {R(qs_re / qq), R(qs_im / qq)};
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        e[sp][c] = e[sp][c] + mul(w, r[sp][c]);
        r[sp][c] = r[sp][c] - mul(w, q[sp][c]);
        ls[(f * 12 + sp * 3 + c) * NS + j] = to_store<R, S>(r[sp][c]);
      }
  }
  // z += e
  cx<R> zv[4][3];
  load_flav<S, R>(zv, zp, nullptr, f, A.stride, h);
  if constexpr (kGrouped<S>) {
    constexpr int G = kG<S>;
    const unsigned vo = group_off<S>(f, A.stride, h);
#pragma unroll
    for (int g = 0; g < 12 / G; ++g) {
      Grp<S> u;
#pragma unroll
      for (int qi = 0; qi < G; ++qi) {
        const int k = G * g + qi;
        u.e[qi] = to_store<R, S>(zv[k / 3][k % 3] + e[k / 3][k % 3]);
      }
      *reinterpret_cast<v4u*>(reinterpret_cast<char*>(zp + (long)g * A.stride * G) + vo) = u.w;
    }
  } else {
    const unsigned vo = flav_off<S>(f, A.stride, h);
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
      for (int c = 0; c < 3; ++c) *at(zp, (long)(sp * 3 + c) * A.stride, vo) = to_store<R, S>(zv[sp][c] + e[sp][c]);
  }
}

template <class S, class L, bool R12>
void launch_sap_ns(int ns, int nblk, const SapArgs<S, L>& A, hipStream_t st) {
  switch (ns) {
    case 64: hipLaunchKernelGGL((sap_block_kernel<S, L, R12, 64>), dim3(nblk), dim3(128), 0, st, A); break;
    case 128: hipLaunchKernelGGL((sap_block_kernel<S, L, R12, 128>), dim3(nblk), dim3(256), 0, st, A); break;
    default: hipLaunchKernelGGL((sap_block_kernel<S, L, R12, 256>), dim3(nblk), dim3(512), 0, st, A); break;
  }
}

template <class S, class L>
void launch_sap_typed(const Geom& g, const int block[4], int colour, int mr_iters, const OpParams& op,
                      const void* U0, const void* U1, const HalfField& s_e, const HalfField& s_o,
                      const HalfField& z_e, const HalfField& z_o, double ms, double hop_coef, hipStream_t st) {
  SapArgs<S, L> A;
  A.s[0] = static_cast<const S*>(s_e.v);
  A.s[1] = static_cast<const S*>(s_o.v);
  A.z[0] = static_cast<S*>(z_e.v);
  A.z[1] = static_cast<S*>(z_o.v);
  A.U[0] = static_cast<const L*>(U0);
  A.U[1] = static_cast<const L*>(U1);
  A.Lz = g.Lz;
  A.Ly = g.Ly;
  A.Lx = g.Lx;
  A.stride = g.stride;
  A.bt = block[0];
  A.bz = block[1];
  A.by = block[2];
  A.bx = block[3];
  A.nbz = g.Lz / block[1];
  A.nby = g.Ly / block[2];
  A.nbxh = g.Lx / block[3] / 2;
  A.colour = colour;
  A.mr_iters = mr_iters;
  A.a = op.a;
  A.mubar = op.mubar;
  A.epsbar = op.epsbar;
  A.ms = ms;
  A.hop_coef = hop_coef;
  const int ns = block[0] * block[1] * block[2] * block[3];
  const int nblk = (g.T / block[0]) * A.nbz * A.nby * A.nbxh;
  if (op.recon12) launch_sap_ns<S, L, true>(ns, nblk, A, st);
  else launch_sap_ns<S, L, false>(ns, nblk, A, st);
}

}  // namespace

int hop_grid(const Geom& g) { return (g.vh + kSitesPerBlock - 1) / kSitesPerBlock; }

void launch_hop(int prec, int epi, int red, const Geom& g, int parity, const OpParams& op,
                const void* Uo, const void* Ui, const HalfField& in, const HalfField& out,
                const HalfField* xs, const HalfField* zs, double ms, double hop_coef, double sigma,
                double* partials, hipStream_t st) {
  switch (prec) {
    case P64:
      launch_typed<double2, double2>(epi, red, g, parity, op, Uo, Ui, in, out, xs, zs, ms, hop_coef,
                                     sigma, partials, st);
      break;
    case P32:
      launch_typed<float2, float2>(epi, red, g, parity, op, Uo, Ui, in, out, xs, zs, ms, hop_coef,
                                   sigma, partials, st);
      break;
    case P32H:
      launch_typed<float2, __half2>(epi, red, g, parity, op, Uo, Ui, in, out, xs, zs, ms, hop_coef,
                                    sigma, partials, st);
      break;
    default:
      launch_typed<__half2, __half2>(epi, red, g, parity, op, Uo, Ui, in, out, xs, zs, ms, hop_coef,
                                     sigma, partials, st);
      break;
  }
}

bool sap_block_ok(const Geom& g, const int block[4]) {
  const int ext[4] = {g.T, g.Lz, g.Ly, g.Lx};
  int n = 1;
  for (int mu = 0; mu < 4; ++mu) {
    // even block extents (blocks start on even sites) and an even number of blocks
    if (block[mu] < 2 || block[mu] % 2 != 0 || ext[mu] % block[mu] != 0 || (ext[mu] / block[mu]) % 2 != 0)
      return false;
    n *= block[mu];
  }
  // 64, 128 or 256 sites: each parity fills whole wavefronts
  return n == 64 || n == 128 || n == 256;
}

void launch_sap_block(int prec, const Geom& g, const int block[4], int colour, int mr_iters, const OpParams& op,
                      const void* U0, const void* U1, const HalfField& s_e, const HalfField& s_o,
                      const HalfField& z_e, const HalfField& z_o, double ms, double hop_coef, hipStream_t st) {
  switch (prec) {
    case P64:
      launch_sap_typed<double2, double2>(g, block, colour, mr_iters, op, U0, U1, s_e, s_o, z_e, z_o, ms, hop_coef, st);
      break;
    case P32:
      launch_sap_typed<float2, float2>(g, block, colour, mr_iters, op, U0, U1, s_e, s_o, z_e, z_o, ms, hop_coef, st);
      break;
    case P32H:
      launch_sap_typed<float2, __half2>(g, block, colour, mr_iters, op, U0, U1, s_e, s_o, z_e, z_o, ms, hop_coef, st);
      break;
    default:
      break;
  }
}

}  // namespace ndtm
