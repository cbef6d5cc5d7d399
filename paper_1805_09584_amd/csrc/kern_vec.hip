// Vector kernels for the multigrid cycle and the coarse Krylov solver, for
// complex vectors stored as double2 or float2.  Reductions accumulate in FP64,
// one partial per block, and are finalised in a fixed order (deterministic).
// Coefficients of the Krylov updates are read from device memory so that a
// whole fixed-length Arnoldi loop runs without a host round trip.
#include <type_traits>

#include "vec.h"
#include "reduce.h"

namespace ndtm {
namespace {

constexpr int kVB = 256;
constexpr int kVGrid = 1024;
constexpr int kMaxBasis = 40;

template <class T2>
struct Basis {
  const T2* v[kMaxBasis];
  __device__ __forceinline__ const T2* at(int j) const { return v[j]; }
};
// k systems' bases back to back: vector j of this system at base + j ldv
struct StridedBasis {
  const double2* base;
  size_t ldv;
  __device__ __forceinline__ const double2* at(int j) const { return base + j * ldv; }
};

// reductions: at most 256 blocks (the completion of each block costs a release
// fence and an atomic on one counter, which grows with the block count), 1024 on
// vectors of 2^23 elements or more, where one block per CU kept too few loads in
// flight (a 12-vector multi-dot at 96x48^3 reached 2.4 TB/s); the reduction
// workspace holds 48 complex sums over 1024 blocks
inline unsigned rgrid(size_t n) {
  size_t g = (n + kVB - 1) / kVB;
  const size_t cap = n >= ((size_t)1 << 23) ? 1024 : 256;
  if (g > cap) g = cap;
  return (unsigned)(g ? g : 1);
}
// the batched (k-system) reductions size their workspaces for 256 blocks
inline unsigned rgrid_sys(size_t n) {
  size_t g = (n + kVB - 1) / kVB;
  if (g > 256) g = 256;
  return (unsigned)(g ? g : 1);
}

inline unsigned vgrid(size_t n) {
  size_t g = (n + kVB - 1) / kVB;
  if (g > (size_t)kVGrid) g = kVGrid;
  return (unsigned)(g ? g : 1);
}

__device__ __forceinline__ double2 ld2(const double2* p, size_t i) { return p[i]; }
__device__ __forceinline__ double2 ld2(const float2* p, size_t i) {
  const float2 v = p[i];
  return make_double2(v.x, v.y);
}
__device__ __forceinline__ void st2(double2* p, size_t i, double2 v) { p[i] = v; }
__device__ __forceinline__ void st2(float2* p, size_t i, double2 v) { p[i] = make_float2((float)v.x, (float)v.y); }

__device__ __forceinline__ double2 cm(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__device__ __forceinline__ double bsum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off);
  __shared__ double ws[kVB / 64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) ws[w] = v;
  __syncthreads();
  double s = 0;
  if (threadIdx.x == 0)
    for (int i = 0; i < kVB / 64; ++i) s += ws[i];
  return s;
}

// Reduction loops: a thread visits its grid-stride indices in increasing order, in
// batches of kRB whose loads are all issued before the first is used (a plain loop,
// even unrolled, waits on each load in turn).  The additions keep their order.
constexpr int kRB = 8;
#define BATCH_LOOP(b, n) \
  for (size_t b = blockIdx.x * (size_t)blockDim.x + threadIdx.x; b < (n); b += (size_t)kRB * gridDim.x * blockDim.x)
#define BATCH_IDX(b, j) ((b) + (size_t)(j) * gridDim.x * blockDim.x)
// the loads of a batch read index min(i, n - 1), so they need no branch (n >= 1 inside
// the loop); only the visits with i < n are added
#define BATCH_LD(p, b, j, n) (p)[BATCH_IDX(b, j) < (n) ? BATCH_IDX(b, j) : (n) - 1]
__device__ __forceinline__ double2 wide(double2 v) { return v; }
__device__ __forceinline__ double2 wide(float2 v) { return make_double2(v.x, v.y); }

__device__ __forceinline__ double2 rounded(const double2*, double2 v) { return v; }
__device__ __forceinline__ double2 rounded(const float2*, double2 v) { return make_double2((float)v.x, (float)v.y); }

// grid-stride loop of the elementwise kernels (the unrolled copies each keep their own
// bounds branch, so their loads do not overlap; the reductions use BATCH_LOOP)
#define GRID_LOOP(i, n)  \
  _Pragma("unroll 4") for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < (n); i += (size_t)gridDim.x * blockDim.x)

template <class A, class B>
__global__ __launch_bounds__(256) void convert_k(B* y, const A* x, size_t n) {
  GRID_LOOP(i, n) st2(y, i, ld2(x, i));
}

template <class T2>
__global__ __launch_bounds__(256) void zero_k(T2* y, size_t n) {
  GRID_LOOP(i, n) st2(y, i, make_double2(0, 0));
}

// y = a x + b y with a = sa * coef[0..1] (device) or host value
template <class T2>
__global__ __launch_bounds__(256) void axpby_k(T2* y, double2 a, const double* adev, double asgn, const T2* x, double2 b, size_t n) {
  double2 aa = a;
  if (adev) aa = make_double2(asgn * adev[0], asgn * adev[1]);
  GRID_LOOP(i, n) {
    const double2 xv = cm(aa, ld2(x, i));
    const double2 yv = cm(b, ld2(y, i));
    st2(y, i, make_double2(xv.x + yv.x, xv.y + yv.y));
  }
}

// y *= 1 / sqrt(*nrm2)
template <class T2>
__device__ __forceinline__ void scale_inv_sqrt_body(T2* y, const T2* x, const double* nrm2, size_t n) {
  const double s = *nrm2 > 1e-300 ? 1.0 / sqrt(*nrm2) : 0.0;
  GRID_LOOP(i, n) {
    const double2 v = ld2(x, i);
    st2(y, i, make_double2(s * v.x, s * v.y));
  }
}

// Single-launch deterministic reduction: every block writes its partial(s);
// the last block to finish (counted with a device-scope atomic) sums the
// partials of each of the `width` scalars in block order and writes dst, then
// resets the counter.  ws = [counter (8 doubles)][partials width x gridDim].
__device__ bool last_block_sum(double* ws, int width, double* dst) {
  __shared__ bool last;
  // the block's partials are written by thread 0 (after the block sum), so
  // only its wave needs the release fence before the counter
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    unsigned* cnt = reinterpret_cast<unsigned*>(ws);
    last = atomicAdd(cnt, 1u) == gridDim.x - 1;
  }
  __syncthreads();
  if (!last) return false;
  __threadfence();
  const double* part = ws + 8;
  // one wavefront per scalar: lanes stride over the block partials in a fixed
  // order, then a fixed-shape shuffle tree
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int j = w; j < width; j += nw) {
    double s = 0;
    for (int i = lane; i < (int)gridDim.x; i += 64) s += part[(size_t)j * gridDim.x + i];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off);
    if (lane == 0) dst[j] = s;
  }
  __syncthreads();
  if (threadIdx.x == 0) *reinterpret_cast<unsigned*>(ws) = 0u;
  return true;
}

template <class T2>
__global__ __launch_bounds__(256) void norm2_k(const T2* x, size_t n, double* ws, double* dst) {
  double s = 0;
  BATCH_LOOP(b, n) {
    T2 v[kRB];
#pragma unroll
    for (int j = 0; j < kRB; ++j) v[j] = BATCH_LD(x, b, j, n);
#pragma unroll
    for (int j = 0; j < kRB; ++j)
      if (BATCH_IDX(b, j) < n) {
        const double2 a = wide(v[j]);
        s += a.x * a.x + a.y * a.y;
      }
  }
  s = bsum(s);
  if (threadIdx.x == 0) ws[8 + blockIdx.x] = s;
  last_block_sum(ws, 1, dst);
}

// partials [2][nblk]: <x,y> re, im
template <class T2>
__global__ __launch_bounds__(256) void dot_k(const T2* x, const T2* y, size_t n, double* ws, double* dst) {
  double* part = ws + 8;
  double re = 0, im = 0;
  BATCH_LOOP(b0, n) {
    T2 xa[kRB], ya[kRB];
#pragma unroll
    for (int j = 0; j < kRB; ++j) {
      xa[j] = BATCH_LD(x, b0, j, n);
      ya[j] = BATCH_LD(y, b0, j, n);
    }
#pragma unroll
    for (int j = 0; j < kRB; ++j)
      if (BATCH_IDX(b0, j) < n) {
        const double2 a = wide(xa[j]), b = wide(ya[j]);
        re += a.x * b.x + a.y * b.y;
        im += a.x * b.y - a.y * b.x;
      }
  }
  re = bsum(re);
  im = bsum(im);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = re;
    part[gridDim.x + blockIdx.x] = im;
  }
  last_block_sum(ws, 2, dst);
}

template <class T2, int KM, class B>
__device__ __forceinline__ void multidot_body(const B& V, int k, const T2* w, size_t n, double* ws, double* dst) {
  double* part = ws + 8;
  double re[KM], im[KM];
#pragma unroll
  for (int j = 0; j < KM; ++j) re[j] = im[j] = 0;
  // up to KM + 1 independent loads per element already; no further unrolling
#pragma unroll 1
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const double2 wi = ld2(w, i);
#pragma unroll
    for (int j = 0; j < KM; ++j)
      if (j < k) {
        const double2 v = ld2(V.at(j), i);
        re[j] += v.x * wi.x + v.y * wi.y;
        im[j] += v.x * wi.y - v.y * wi.x;
      }
  }
  for (int j = 0; j < k; ++j) {
    const double a = bsum(re[j]);
    const double b = bsum(im[j]);
    if (threadIdx.x == 0) {
      part[(size_t)(2 * j) * gridDim.x + blockIdx.x] = a;
      part[(size_t)(2 * j + 1) * gridDim.x + blockIdx.x] = b;
    }
  }
  last_block_sum(ws, 2 * k, dst);
}

// w -= sum_j coef[j] V_j, then <V_j, w> for j < k (one pass: the first Gram-Schmidt
// pass's update and the second pass's overlaps; the overlaps use the stored w)
template <class T2, int KM, class B>
__device__ __forceinline__ void multi_axpy_dot_body(T2* w, const B& V, int k, const double* coef, size_t n,
                                                    double* ws, double* dst) {
  double* part = ws + 8;
  double re[KM], im[KM];
#pragma unroll
  for (int j = 0; j < KM; ++j) re[j] = im[j] = 0;
#pragma unroll 1
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    double2 acc = ld2(w, i);
    double2 v[KM];
#pragma unroll
    for (int j = 0; j < KM; ++j)
      if (j < k) {
        v[j] = ld2(V.at(j), i);
        const double2 t = cm(make_double2(coef[2 * j], coef[2 * j + 1]), v[j]);
        acc.x -= t.x;
        acc.y -= t.y;
      }
    st2(w, i, acc);
    const double2 r = rounded(w, acc);
#pragma unroll
    for (int j = 0; j < KM; ++j)
      if (j < k) {
        re[j] += v[j].x * r.x + v[j].y * r.y;
        im[j] += v[j].x * r.y - v[j].y * r.x;
      }
  }
  for (int j = 0; j < k; ++j) {
    const double a = bsum(re[j]);
    const double b = bsum(im[j]);
    if (threadIdx.x == 0) {
      part[(size_t)(2 * j) * gridDim.x + blockIdx.x] = a;
      part[(size_t)(2 * j + 1) * gridDim.x + blockIdx.x] = b;
    }
  }
  last_block_sum(ws, 2 * k, dst);
}

// sums column j of partials [width][nparts] into dst[j*dst_stride]
__global__ void finalize_k(const double* part, int nparts, double* dst, int dst_stride) {
  const double* p = part + (size_t)blockIdx.x * nparts;
  double s = strided_sum(p, nparts);
  s = bsum(s);
  if (threadIdx.x == 0) dst[(size_t)blockIdx.x * dst_stride] = s;
}

// w -= sum_j coef[j] V_j and ||w||^2 into dst (single launch)
template <class T2, class B>
__device__ __forceinline__ void multi_axpy_norm_body(T2* w, const B& V, int k, const double* coef, size_t n,
                                                     double* ws, double* dst) {
  double s = 0;
  GRID_LOOP(i, n) {
    double2 acc = ld2(w, i);
    for (int j = 0; j < k; ++j) {
      const double2 t = cm(make_double2(coef[2 * j], coef[2 * j + 1]), ld2(V.at(j), i));
      acc.x -= t.x;
      acc.y -= t.y;
    }
    st2(w, i, acc);
    const double2 r = rounded(w, acc);  // the stored value
    s += r.x * r.x + r.y * r.y;
  }
  s = bsum(s);
  if (threadIdx.x == 0) ws[8 + blockIdx.x] = s;
  last_block_sum(ws, 1, dst);
}

// sum of part[0..np) in a fixed order, valid in every thread of the block
__device__ double block_total(const double* part, int np) {
  __shared__ double wsum[kVB / 64];
  __shared__ double tot;
  double v = strided_sum(part, np);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += wsum[w];
    tot = s;
  }
  __syncthreads();
  return tot;
}

// minimal-residual update with omega = <t, s> / <t, t> taken from the partials of
// the stencil passes that formed t = D' s (part[q * np + i], q = re, im, norm): every
// block sums them in the same order, so all use the same omega
template <class T2>
__global__ __launch_bounds__(256) void mr_update_part_k(T2* z, T2* sv, const T2* t, const double* part, int np,
                                                        int update_s, size_t n) {
  // the vectors stream in batches of kRB visits with all loads issued first; the first
  // batch is in flight while omega is summed
  T2 za[kRB], sa[kRB], ta[kRB];
  size_t b0 = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  auto load = [&](size_t b) {
#pragma unroll
    for (int j = 0; j < kRB; ++j) {
      za[j] = BATCH_LD(z, b, j, n);
      sa[j] = BATCH_LD(sv, b, j, n);
      if (update_s) ta[j] = BATCH_LD(t, b, j, n);
    }
  };
  if (b0 < n) load(b0);
  const double re = block_total(part, np);
  const double im = block_total(part + np, np);
  const double tt = block_total(part + 2 * (size_t)np, np);
  const double2 w = tt > 0 ? make_double2(re / tt, im / tt) : make_double2(0.0, 0.0);
  while (b0 < n) {
#pragma unroll
    for (int j = 0; j < kRB; ++j) {
      const size_t i = BATCH_IDX(b0, j);
      if (i < n) {
        const double2 sval = wide(sa[j]);
        const double2 zs = cm(w, sval);
        const double2 zv = wide(za[j]);
        st2(z, i, make_double2(zv.x + zs.x, zv.y + zs.y));
        if (update_s) {
          const double2 tw = cm(w, wide(ta[j]));
          st2(sv, i, make_double2(sval.x - tw.x, sval.y - tw.y));
        }
      }
    }
    b0 += (size_t)kRB * gridDim.x * blockDim.x;
    if (b0 < n) load(b0);
  }
}

// y (+)= sum_j coef[j] V_j   (coef device)
template <class T2>
__global__ __launch_bounds__(256) void lincomb_dev_k(T2* y, Basis<T2> V, int k, const double* coef, int accumulate, size_t n) {
  GRID_LOOP(i, n) {
    double2 acc = accumulate ? ld2(y, i) : make_double2(0, 0);
    for (int j = 0; j < k; ++j) {
      const double2 t = cm(make_double2(coef[2 * j], coef[2 * j + 1]), ld2(V.v[j], i));
      acc.x += t.x;
      acc.y += t.y;
    }
    st2(y, i, acc);
  }
}


// Least squares of a (m+1) x m Hessenberg system by Givens rotations, one thread.
// H column-major with leading dimension ldh (complex, 2 doubles); beta = sqrt(*beta2).
__global__ void hess_lsq_k(const double* H, const double* H2, int ldh, int m, const double* beta2, const double* sub2,
                           double* y) {
  // small dense work in LDS (a private array would live in scratch memory)
  __shared__ double2 R[kMaxBasis + 1][kMaxBasis];
  __shared__ double2 g[kMaxBasis + 1];
  __shared__ double2 cs[kMaxBasis], sn[kMaxBasis];
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  for (int j = 0; j < m; ++j)
  {
    for (int i = 0; i <= j; ++i) {
      const size_t e = 2 * ((size_t)j * ldh + i);
      R[i][j] = H2 ? make_double2(H[e] + H2[e], H[e + 1] + H2[e + 1]) : make_double2(H[e], H[e + 1]);
    }
    R[j + 1][j] = make_double2(sqrt(fmax(sub2[j], 0.0)), 0.0);
  }
  for (int i = 0; i <= m; ++i) g[i] = make_double2(0, 0);
  g[0] = make_double2(sqrt(*beta2), 0);
  int mm = m;
  for (int j = 0; j < m; ++j) {
    for (int i = 0; i < j; ++i) {
      const double2 a = R[i][j], b = R[i + 1][j];
      // G = [[conj(c), conj(s)], [-s, c]]
      const double2 ca = make_double2(cs[i].x * a.x + cs[i].y * a.y, cs[i].x * a.y - cs[i].y * a.x);
      const double2 sb = make_double2(sn[i].x * b.x + sn[i].y * b.y, sn[i].x * b.y - sn[i].y * b.x);
      R[i][j] = make_double2(ca.x + sb.x, ca.y + sb.y);
      const double2 t1 = cm(sn[i], a), t2 = cm(cs[i], b);
      R[i + 1][j] = make_double2(t2.x - t1.x, t2.y - t1.y);
    }
    const double2 a = R[j][j], b = R[j + 1][j];
    const double den = sqrt(a.x * a.x + a.y * a.y + b.x * b.x + b.y * b.y);
    if (!(den > 0) || !isfinite(den)) {
      mm = j;
      break;
    }
    cs[j] = make_double2(a.x / den, a.y / den);
    sn[j] = make_double2(b.x / den, b.y / den);
    R[j][j] = make_double2(den, 0);
    R[j + 1][j] = make_double2(0, 0);
    const double2 gj = g[j];
    const double2 t = cm(sn[j], gj);
    g[j + 1] = make_double2(-t.x, -t.y);
    g[j] = make_double2(cs[j].x * gj.x + cs[j].y * gj.y, cs[j].x * gj.y - cs[j].y * gj.x);
  }
  for (int j = 0; j < m; ++j) y[2 * j] = y[2 * j + 1] = 0.0;
  for (int i = mm - 1; i >= 0; --i) {
    double2 s = g[i];
    for (int j = i + 1; j < mm; ++j) {
      const double2 t = cm(R[i][j], make_double2(y[2 * j], y[2 * j + 1]));
      s.x -= t.x;
      s.y -= t.y;
    }
    const double2 d = R[i][i];
    const double dd = d.x * d.x + d.y * d.y;
    y[2 * i] = (s.x * d.x + s.y * d.y) / dd;
    y[2 * i + 1] = (s.y * d.x - s.x * d.y) / dd;
  }
}

// ---- kernels: the bodies above, one system per launch or k systems per launch ----
template <class T2>
__global__ __launch_bounds__(256) void scale_inv_sqrt_k(T2* y, const T2* x, const double* nrm2, size_t n) {
  scale_inv_sqrt_body(y, x, nrm2, n);
}
template <class T2, int KM>
__global__ __launch_bounds__(256) void multidot_k(Basis<T2> V, int k, const T2* w, size_t n, double* ws, double* dst) {
  multidot_body<T2, KM>(V, k, w, n, ws, dst);
}
template <class T2, int KM>
__global__ __launch_bounds__(256) void multi_axpy_dot_k(T2* w, Basis<T2> V, int k, const double* coef, size_t n,
                                                        double* ws, double* dst) {
  multi_axpy_dot_body<T2, KM>(w, V, k, coef, n, ws, dst);
}
template <class T2>
__global__ __launch_bounds__(256) void multi_axpy_norm_k(T2* w, Basis<T2> V, int k, const double* coef, size_t n,
                                                         double* ws, double* dst) {
  multi_axpy_norm_body<T2>(w, V, k, coef, n, ws, dst);
}

// k systems per launch (system s = blockIdx.y): basis vector i of system s at
// V + i ldv + s n, its vector w + s n, its coefficients coef + s cs, its reduction
// workspace ws + s wss (own counter and partials), its outputs dst + s ds
struct SysArgs {
  size_t ldv, wss, cs, ds;
};
template <int KM>
__global__ __launch_bounds__(256) void multidot_sys_k(const double2* V, int cnt, const double2* w, size_t n,
                                                      double* ws, double* dst, SysArgs a) {
  const size_t s = blockIdx.y;
  multidot_body<double2, KM>(StridedBasis{V + s * n, a.ldv}, cnt, w + s * n, n, ws + s * a.wss, dst + s * a.ds);
}
template <int KM>
__global__ __launch_bounds__(256) void multi_axpy_dot_sys_k(double2* w, const double2* V, int cnt, const double* coef,
                                                            size_t n, double* ws, double* dst, SysArgs a) {
  const size_t s = blockIdx.y;
  multi_axpy_dot_body<double2, KM>(w + s * n, StridedBasis{V + s * n, a.ldv}, cnt, coef + s * a.cs, n,
                                   ws + s * a.wss, dst + s * a.ds);
}
__global__ __launch_bounds__(256) void multi_axpy_norm_sys_k(double2* w, const double2* V, int cnt,
                                                             const double* coef, size_t n, double* ws, double* dst,
                                                             SysArgs a) {
  const size_t s = blockIdx.y;
  multi_axpy_norm_body<double2>(w + s * n, StridedBasis{V + s * n, a.ldv}, cnt, coef + s * a.cs, n, ws + s * a.wss,
                                dst + s * a.ds);
}
__global__ __launch_bounds__(256) void scale_inv_sqrt_sys_k(double2* y, const double2* x, const double* nrm2,
                                                            size_t n, size_t ds) {
  const size_t s = blockIdx.y;
  scale_inv_sqrt_body(y + s * n, x + s * n, nrm2 + s * ds, n);
}

template <class T2>
Basis<T2> basis(const void* const* V, int k) {
  Basis<T2> B;
  for (int j = 0; j < k && j < kMaxBasis; ++j) B.v[j] = static_cast<const T2*>(V[j]);
  return B;
}

}  // namespace

#define DISPATCH(prec, F, ...)      \
  do {                              \
    if ((prec) == P64) F<double2>(__VA_ARGS__); \
    else F<float2>(__VA_ARGS__);    \
  } while (0)

template <class T2>
static void vzero_t(void* y, size_t n, hipStream_t st) {
  hipLaunchKernelGGL(zero_k<T2>, dim3(vgrid(n)), dim3(kVB), 0, st, static_cast<T2*>(y), n);
}
void vzero(int prec, void* y, size_t n, hipStream_t st) { DISPATCH(prec, vzero_t, y, n, st); }

// per site and component: the two precisions order a half field's elements differently
template <class TS, class TD>
__global__ __launch_bounds__(256) void convert_field_k(TD* y, int pd, const TS* x, int ps, int nhalves, int vh, int stride) {
  const long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (e >= (long)nhalves * vh) return;
  const long k = e / vh, h = e - k * vh;
  const long base = k * 24L * stride;
  for (int c = 0; c < 24; ++c) {
    const TS v = x[base + fidx(ps, c, stride, h)];
    TD w;
    w.x = v.x;
    w.y = v.y;
    y[base + fidx(pd, c, stride, h)] = w;
  }
}

void vconvert_field(int prec_dst, void* y, int prec_src, const void* x, int nhalves, int vh, int stride,
                    hipStream_t st) {
  const dim3 g((unsigned)(((long)nhalves * vh + 255) / 256)), b(256);
  if (prec_src == P64 && prec_dst == P32)
    hipLaunchKernelGGL((convert_field_k<double2, float2>), g, b, 0, st, static_cast<float2*>(y), prec_dst,
                       static_cast<const double2*>(x), prec_src, nhalves, vh, stride);
  else if (prec_src == P32 && prec_dst == P64)
    hipLaunchKernelGGL((convert_field_k<float2, double2>), g, b, 0, st, static_cast<double2*>(y), prec_dst,
                       static_cast<const float2*>(x), prec_src, nhalves, vh, stride);
  else
    vconvert(prec_dst, y, prec_src, x, (size_t)nhalves * 24 * stride, st);  // same precision: same layout
}

void vconvert(int prec_dst, void* y, int prec_src, const void* x, size_t n, hipStream_t st) {
  const dim3 g(vgrid(n)), b(kVB);
  if (prec_src == P64 && prec_dst == P64)
    hipLaunchKernelGGL((convert_k<double2, double2>), g, b, 0, st, static_cast<double2*>(y), static_cast<const double2*>(x), n);
  else if (prec_src == P64)
    hipLaunchKernelGGL((convert_k<double2, float2>), g, b, 0, st, static_cast<float2*>(y), static_cast<const double2*>(x), n);
  else if (prec_dst == P64)
    hipLaunchKernelGGL((convert_k<float2, double2>), g, b, 0, st, static_cast<double2*>(y), static_cast<const float2*>(x), n);
  else
    hipLaunchKernelGGL((convert_k<float2, float2>), g, b, 0, st, static_cast<float2*>(y), static_cast<const float2*>(x), n);
}

template <class T2>
static void vaxpby_t(void* y, double2 a, const double* adev, double asgn, const void* x, double2 b, size_t n,
                     hipStream_t st) {
  hipLaunchKernelGGL(axpby_k<T2>, dim3(vgrid(n)), dim3(kVB), 0, st, static_cast<T2*>(y), a, adev, asgn,
                     static_cast<const T2*>(x), b, n);
}
void vaxpby(int prec, void* y, double2 a, const void* x, double2 b, size_t n, hipStream_t st) {
  DISPATCH(prec, vaxpby_t, y, a, nullptr, 1.0, x, b, n, st);
}
void vaxpy_dev(int prec, void* y, const double* adev, double asgn, const void* x, size_t n, hipStream_t st) {
  DISPATCH(prec, vaxpby_t, y, make_double2(0, 0), adev, asgn, x, make_double2(1, 0), n, st);
}

template <class T2>
static void vscale_inv_sqrt_t(void* y, const void* x, const double* nrm2, size_t n, hipStream_t st) {
  hipLaunchKernelGGL(scale_inv_sqrt_k<T2>, dim3(vgrid(n)), dim3(kVB), 0, st, static_cast<T2*>(y),
                     static_cast<const T2*>(x), nrm2, n);
}
void vscale_inv_sqrt(int prec, void* y, const void* x, const double* nrm2, size_t n, hipStream_t st) {
  DISPATCH(prec, vscale_inv_sqrt_t, y, x, nrm2, n, st);
}

void vfinalize(const double* part, int nparts, int width, double* dst, int dst_stride, hipStream_t st) {
  hipLaunchKernelGGL(finalize_k, dim3(width), dim3(kVB), 0, st, part, nparts, dst, dst_stride);
}

template <class T2>
static void vnorm2_t(const void* x, size_t n, double* ws, double* dst, hipStream_t st) {
  hipLaunchKernelGGL(norm2_k<T2>, dim3(rgrid(n)), dim3(kVB), 0, st, static_cast<const T2*>(x), n, ws, dst);
}
void vnorm2(int prec, const void* x, size_t n, double* ws, double* dst, hipStream_t st) {
  DISPATCH(prec, vnorm2_t, x, n, ws, dst, st);
}

template <class T2>
static void vdot_t(const void* x, const void* y, size_t n, double* ws, double* dst, hipStream_t st) {
  hipLaunchKernelGGL(dot_k<T2>, dim3(rgrid(n)), dim3(kVB), 0, st, static_cast<const T2*>(x),
                     static_cast<const T2*>(y), n, ws, dst);
}
void vdot(int prec, const void* x, const void* y, size_t n, double* ws, double* dst, hipStream_t st) {
  DISPATCH(prec, vdot_t, x, y, n, ws, dst, st);
}

template <class T2>
static void vmultidot_t(const void* const* V, int k, const void* w, size_t n, double* part, double* dst,
                        hipStream_t st) {
  const unsigned g = rgrid(n);
  auto B = basis<T2>(V, k);
  const T2* wp = static_cast<const T2*>(w);
  if (k <= 4)
    hipLaunchKernelGGL((multidot_k<T2, 4>), dim3(g), dim3(kVB), 0, st, B, k, wp, n, part, dst);
  else if (k <= 8)
    hipLaunchKernelGGL((multidot_k<T2, 8>), dim3(g), dim3(kVB), 0, st, B, k, wp, n, part, dst);
  else if (k <= 16)
    hipLaunchKernelGGL((multidot_k<T2, 16>), dim3(g), dim3(kVB), 0, st, B, k, wp, n, part, dst);
  else if (k <= 24)
    hipLaunchKernelGGL((multidot_k<T2, 24>), dim3(g), dim3(kVB), 0, st, B, k, wp, n, part, dst);
  else
    hipLaunchKernelGGL((multidot_k<T2, kMaxBasis>), dim3(g), dim3(kVB), 0, st, B, k, wp, n, part, dst);
}
void vmultidot(int prec, const void* const* V, int k, const void* w, size_t n, double* part, double* dst,
               hipStream_t st) {
  DISPATCH(prec, vmultidot_t, V, k, w, n, part, dst, st);
}

// ---- k systems per launch (FP64) ----
template <class F>
static void by_km(int cnt, F f) {
  if (cnt <= 4) f(std::integral_constant<int, 4>{});
  else if (cnt <= 8) f(std::integral_constant<int, 8>{});
  else if (cnt <= 16) f(std::integral_constant<int, 16>{});
  else if (cnt <= 24) f(std::integral_constant<int, 24>{});
  else f(std::integral_constant<int, kMaxBasis>{});
}
void vmultidot_sys(const double2* V, size_t ldv, int cnt, const double2* w, size_t n, int k, double* ws, size_t wss,
                   double* dst, size_t ds, hipStream_t st) {
  const SysArgs a{ldv, wss, 0, ds};
  const dim3 g(rgrid_sys(n), k);
  by_km(cnt, [&](auto km) {
    hipLaunchKernelGGL((multidot_sys_k<decltype(km)::value>), g, dim3(kVB), 0, st, V, cnt, w, n, ws, dst, a);
  });
}
void vmulti_axpy_multidot_sys(double2* w, const double2* V, size_t ldv, int cnt, const double* coef, size_t cs,
                              size_t n, int k, double* ws, size_t wss, double* dst, size_t ds, hipStream_t st) {
  const SysArgs a{ldv, wss, cs, ds};
  const dim3 g(rgrid_sys(n), k);
  by_km(cnt, [&](auto km) {
    hipLaunchKernelGGL((multi_axpy_dot_sys_k<decltype(km)::value>), g, dim3(kVB), 0, st, w, V, cnt, coef, n, ws, dst,
                       a);
  });
}
void vmulti_axpy_norm_sys(double2* w, const double2* V, size_t ldv, int cnt, const double* coef, size_t cs, size_t n,
                          int k, double* ws, size_t wss, double* dst, size_t ds, hipStream_t st) {
  const SysArgs a{ldv, wss, cs, ds};
  hipLaunchKernelGGL(multi_axpy_norm_sys_k, dim3(rgrid_sys(n), k), dim3(kVB), 0, st, w, V, cnt, coef, n, ws, dst, a);
}
void vscale_inv_sqrt_sys(double2* y, const double2* x, const double* nrm2, size_t ds, size_t n, int k,
                         hipStream_t st) {
  hipLaunchKernelGGL(scale_inv_sqrt_sys_k, dim3(vgrid(n), k), dim3(kVB), 0, st, y, x, nrm2, n, ds);
}

template <class T2>
static void vmulti_axpy_dot_t(void* w, const void* const* V, int k, const double* coef, size_t n, double* part,
                              double* dst, hipStream_t st) {
  const unsigned g = rgrid(n);
  auto B = basis<T2>(V, k);
  T2* wp = static_cast<T2*>(w);
  if (k <= 4)
    hipLaunchKernelGGL((multi_axpy_dot_k<T2, 4>), dim3(g), dim3(kVB), 0, st, wp, B, k, coef, n, part, dst);
  else if (k <= 8)
    hipLaunchKernelGGL((multi_axpy_dot_k<T2, 8>), dim3(g), dim3(kVB), 0, st, wp, B, k, coef, n, part, dst);
  else if (k <= 16)
    hipLaunchKernelGGL((multi_axpy_dot_k<T2, 16>), dim3(g), dim3(kVB), 0, st, wp, B, k, coef, n, part, dst);
  else if (k <= 24)
    hipLaunchKernelGGL((multi_axpy_dot_k<T2, 24>), dim3(g), dim3(kVB), 0, st, wp, B, k, coef, n, part, dst);
  else
    hipLaunchKernelGGL((multi_axpy_dot_k<T2, kMaxBasis>), dim3(g), dim3(kVB), 0, st, wp, B, k, coef, n, part, dst);
}
void vmulti_axpy_multidot(int prec, void* w, const void* const* V, int k, const double* coef, size_t n, double* part,
                          double* dst, hipStream_t st) {
  DISPATCH(prec, vmulti_axpy_dot_t, w, V, k, coef, n, part, dst, st);
}

template <class T2>
static void vlincomb_t(void* y, const void* const* V, int k, const double* coef, int acc, size_t n,
                       hipStream_t st) {
  hipLaunchKernelGGL(lincomb_dev_k<T2>, dim3(vgrid(n)), dim3(kVB), 0, st, static_cast<T2*>(y), basis<T2>(V, k), k,
                     coef, acc, n);
}
void vlincomb_dev(int prec, void* y, const void* const* V, int k, const double* coef, int accumulate, size_t n,
                  hipStream_t st) {
  DISPATCH(prec, vlincomb_t, y, V, k, coef, accumulate, n, st);
}

template <class T2>
static void vmulti_axpy_norm_t(void* w, const void* const* V, int k, const double* coef, size_t n, double* ws,
                               double* dst, hipStream_t st) {
  hipLaunchKernelGGL(multi_axpy_norm_k<T2>, dim3(rgrid(n)), dim3(kVB), 0, st, static_cast<T2*>(w), basis<T2>(V, k),
                     k, coef, n, ws, dst);
}
void vmulti_axpy_norm_dev(int prec, void* w, const void* const* V, int k, const double* coef, size_t n, double* ws,
                          double* dst, hipStream_t st) {
  DISPATCH(prec, vmulti_axpy_norm_t, w, V, k, coef, n, ws, dst, st);
}

template <class T2>
static void vmr_update_part_t(void* z, void* s, const void* t, const double* part, int np, int update_s, size_t n,
                              hipStream_t st) {
  hipLaunchKernelGGL(mr_update_part_k<T2>, dim3(vgrid(n)), dim3(kVB), 0, st, static_cast<T2*>(z),
                     static_cast<T2*>(s), static_cast<const T2*>(t), part, np, update_s, n);
}
void vmr_update_part(int prec, void* z, void* s, const void* t, const double* part, int np, int update_s, size_t n,
                     hipStream_t st) {
  DISPATCH(prec, vmr_update_part_t, z, s, t, part, np, update_s, n, st);
}



void hess_lsq(const double* H, const double* H2, int ldh, int m, const double* beta2, const double* sub2, double* y,
              hipStream_t st) {
  hipLaunchKernelGGL(hess_lsq_k, dim3(1), dim3(64), 0, st, H, H2, ldh, m, beta2, sub2, y);
}

}  // namespace ndtm
