// Conversions between the canonical complex128 layouts of the C-ABI and the
// internal structure-of-arrays even-odd storage in FP64, FP32 and FP16 (with
// one FP32 scale per site: the largest |real| or |imag| part of the site's
// 48 reals, values stored as binary16 of x/scale, round to nearest even).
#include "ndtm_internal.h"

namespace ndtm {
namespace {

__device__ __forceinline__ int site_parity(long s, int T, int Lz, int Ly, int Lx) {
  const int x = s % Lx;
  const long r = s / Lx;
  const int y = r % Ly;
  const long r2 = r / Ly;
  const int z = r2 % Lz;
  const int t = r2 / Lz;
  return (t + z + y + x) & 1;
}

__global__ void pack_gauge_k(Geom g, const double2* U, double2* U64e, double2* U64o, float2* U32e,
                             float2* U32o, __half2* U16e, __half2* U16o) {
  const long V = 2L * g.vh;
  const long s = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (s >= V) return;
  const int p = site_parity(s, g.T, g.Lz, g.Ly, g.Lx);
  const long h = s >> 1;
  double2* d64 = p ? U64o : U64e;
  float2* d32 = p ? U32o : U32e;
  __half2* d16 = p ? U16o : U16e;
  for (int k = 0; k < 36; ++k) {
    const double2 u = U[s * 36 + k];
    const long o = (long)k * g.stride + h;
    d64[o] = u;
    d32[lidx32(k / 9, k % 9, g.stride, h)] = make_float2((float)u.x, (float)u.y);
    d16[lidx16(k / 9, k % 9, g.stride, h)] = __floats2half2_rn((float)u.x, (float)u.y);
  }
}

// store one site's 24 complex values into a half field of any precision
__device__ __forceinline__ void put_site(const HalfField& f, int stride, long h, const double2* v) {
  if (f.prec == P64) {
    double2* d = static_cast<double2*>(f.v);
    for (int c = 0; c < 24; ++c) d[(long)c * stride + h] = v[c];
  } else if (f.prec == P32) {
    float2* d = static_cast<float2*>(f.v);
    for (int c = 0; c < 24; ++c) d[idx32(c, stride, h)] = make_float2((float)v[c].x, (float)v[c].y);
  } else {
    double mx = 0;
    for (int c = 0; c < 24; ++c) mx = fmax(mx, fmax(fabs(v[c].x), fabs(v[c].y)));
    const float sc = (float)mx;
    const double inv = sc > 0 ? 1.0 / (double)sc : 0.0;
    __half2* d = static_cast<__half2*>(f.v);
    for (int c = 0; c < 24; ++c)
      d[idx16(c, stride, h)] = __floats2half2_rn((float)(v[c].x * inv), (float)(v[c].y * inv));
    f.sc[h] = sc;
  }
}

__device__ __forceinline__ void get_site(const HalfField& f, int stride, long h, double2* v) {
  if (f.prec == P64) {
    const double2* d = static_cast<const double2*>(f.v);
    for (int c = 0; c < 24; ++c) v[c] = d[(long)c * stride + h];
  } else if (f.prec == P32) {
    const float2* d = static_cast<const float2*>(f.v);
    for (int c = 0; c < 24; ++c) v[c] = make_double2(d[idx32(c, stride, h)].x, d[idx32(c, stride, h)].y);
  } else {
    const __half2* d = static_cast<const __half2*>(f.v);
    const double sc = f.sc[h];
    for (int c = 0; c < 24; ++c) {
      const float2 t = __half22float2(d[idx16(c, stride, h)]);
      v[c] = make_double2(t.x * sc, t.y * sc);
    }
  }
}

__global__ void pack_half_k(Geom g, const double2* canon, HalfField f) {
  const long h = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (h >= g.vh) return;
  double2 v[24];
  for (int c = 0; c < 24; ++c) v[c] = canon[h * 24 + c];
  put_site(f, g.stride, h, v);
}

__global__ void unpack_half_k(Geom g, HalfField f, double2* canon) {
  const long h = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (h >= g.vh) return;
  double2 v[24];
  get_site(f, g.stride, h, v);
  for (int c = 0; c < 24; ++c) canon[h * 24 + c] = v[c];
}

__global__ void pack_full_k(Geom g, const double2* canon, HalfField fe, HalfField fo) {
  const long s = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (s >= 2L * g.vh) return;
  const int p = site_parity(s, g.T, g.Lz, g.Ly, g.Lx);
  double2 v[24];
  for (int c = 0; c < 24; ++c) v[c] = canon[s * 24 + c];
  put_site(p ? fo : fe, g.stride, s >> 1, v);
}

__global__ void unpack_full_k(Geom g, HalfField fe, HalfField fo, double2* canon) {
  const long s = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (s >= 2L * g.vh) return;
  const int p = site_parity(s, g.T, g.Lz, g.Ly, g.Lx);
  double2 v[24];
  get_site(p ? fo : fe, g.stride, s >> 1, v);
  for (int c = 0; c < 24; ++c) canon[s * 24 + c] = v[c];
}

__global__ void convert_half_k(Geom g, HalfField src, HalfField dst) {
  const long h = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (h >= g.vh) return;
  double2 v[24];
  get_site(src, g.stride, h, v);
  put_site(dst, g.stride, h, v);
}

// out = Gamma5 x tau1 in (site-local: out_{f,s} = g5_s in_{1-f,s}), FP64 half fields
__global__ void g5t1_k(Geom g, const double2* in, double2* out) {
  const long h = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (h >= g.vh) return;
  for (int f = 0; f < 2; ++f)
    for (int sc = 0; sc < 12; ++sc) {
      const double g5 = sc < 6 ? 1.0 : -1.0;
      const double2 v = in[(long)((1 - f) * 12 + sc) * g.stride + h];
      out[(long)(f * 12 + sc) * g.stride + h] = make_double2(g5 * v.x, g5 * v.y);
    }
}

inline unsigned nblk(long n, int b) { return (unsigned)((n + b - 1) / b); }

// SU(3) links satisfy row 2 = conj(row 0 x row 1); the deviation decides
// whether the stencil may rebuild the third row instead of loading it
__global__ __launch_bounds__(256) void su3_check_k(long nlinks, const double2* U, double* part) {
  double dev = 0;
  for (long l = blockIdx.x * (long)blockDim.x + threadIdx.x; l < nlinks; l += (long)gridDim.x * blockDim.x) {
    const double2* u = U + l * 9;
    for (int c = 0; c < 3; ++c) {
      const int a = (c + 1) % 3, b = (c + 2) % 3;
      // (row0 x row1)_c = u0a u1b - u0b u1a
      const double2 p = u[a], q = u[3 + b], r = u[b], t = u[3 + a];
      const double xr = p.x * q.x - p.y * q.y - (r.x * t.x - r.y * t.y);
      const double xi = p.x * q.y + p.y * q.x - (r.x * t.y + r.y * t.x);
      const double2 w = u[6 + c];
      dev = fmax(dev, fmax(fabs(w.x - xr), fabs(w.y + xi)));
    }
  }
  for (int off = 32; off > 0; off >>= 1) dev = fmax(dev, __shfl_down(dev, off));
  __shared__ double ws[4];
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = dev;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = fmax(fmax(ws[0], ws[1]), fmax(ws[2], ws[3]));
}

// SU(3) links of one parity ([mu 9 + k][stride], FP64) in eight real parameters: per
// link four complex words [mu 4 + j][stride]: U01, U02, the smaller in magnitude of
// U10 and U20 (kept exactly), and (arg U00, arg of the other + 8 if the kept one is U20).
// The stencil rebuilds |U00| from the first row's norm, the other first-column entry's
// magnitude from the column norm (the larger of the two, so no cancellation), and the
// remaining 2x2 block from unitarity and det U = 1 (a division by |U01|^2 + |U02|^2).
// part[block] receives the smallest |U01|^2 + |U02|^2 of the block's links.
__global__ __launch_bounds__(256) void pack_r8_k(int vh, int stride, const double2* U, double2* U8, double* part) {
  double mn = 1.0;
  for (long q = blockIdx.x * (long)blockDim.x + threadIdx.x; q < 4L * vh; q += (long)gridDim.x * blockDim.x) {
    const int mu = (int)(q / vh), h = (int)(q - (long)mu * vh);
    const double2 u00 = U[(long)(mu * 9 + 0) * stride + h], u01 = U[(long)(mu * 9 + 1) * stride + h],
                  u02 = U[(long)(mu * 9 + 2) * stride + h], u10 = U[(long)(mu * 9 + 3) * stride + h],
                  u20 = U[(long)(mu * 9 + 6) * stride + h];
    const double na = u01.x * u01.x + u01.y * u01.y + u02.x * u02.x + u02.y * u02.y;
    mn = fmin(mn, na);
    const bool keep20 = u20.x * u20.x + u20.y * u20.y < u10.x * u10.x + u10.y * u10.y;
    const double2 kept = keep20 ? u20 : u10, other = keep20 ? u10 : u20;
    U8[(long)(mu * 4 + 0) * stride + h] = u01;
    U8[(long)(mu * 4 + 1) * stride + h] = u02;
    U8[(long)(mu * 4 + 2) * stride + h] = kept;
    U8[(long)(mu * 4 + 3) * stride + h] = make_double2(atan2(u00.y, u00.x), atan2(other.y, other.x) + (keep20 ? 8.0 : 0.0));
  }
  for (int off = 32; off > 0; off >>= 1) mn = fmin(mn, __shfl_down(mn, off));
  __shared__ double ws[4];
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = mn;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = fmin(fmin(ws[0], ws[1]), fmin(ws[2], ws[3]));
}

}  // namespace

int launch_pack_r8(const Geom& g, const double2* U64, double2* U8, double* part, hipStream_t st) {
  hipLaunchKernelGGL(pack_r8_k, dim3(1024), dim3(256), 0, st, g.vh, g.stride, U64, U8, part);
  return 1024;
}

int launch_su3_check(long V, const double2* U, double* part, hipStream_t st) {
  hipLaunchKernelGGL(su3_check_k, dim3(1024), dim3(256), 0, st, 4 * V, U, part);
  return 1024;
}

void launch_g5t1(const Geom& g, const double2* in, double2* out, hipStream_t st) {
  hipLaunchKernelGGL(g5t1_k, dim3(nblk(g.vh, 256)), dim3(256), 0, st, g, in, out);
}

void launch_pack_gauge(const Geom& g, const double2* U, double2* U64e, double2* U64o, float2* U32e,
                       float2* U32o, __half2* U16e, __half2* U16o, hipStream_t st) {
  hipLaunchKernelGGL(pack_gauge_k, dim3(nblk(2L * g.vh, 256)), dim3(256), 0, st, g, U, U64e, U64o,
                     U32e, U32o, U16e, U16o);
}
void launch_pack_half(const Geom& g, const double2* canon, const HalfField& f, hipStream_t st) {
  hipLaunchKernelGGL(pack_half_k, dim3(nblk(g.vh, 256)), dim3(256), 0, st, g, canon, f);
}
void launch_unpack_half(const Geom& g, const HalfField& f, double2* canon, hipStream_t st) {
  hipLaunchKernelGGL(unpack_half_k, dim3(nblk(g.vh, 256)), dim3(256), 0, st, g, f, canon);
}
void launch_pack_full(const Geom& g, const double2* canon, const HalfField& fe, const HalfField& fo,
                      hipStream_t st) {
  hipLaunchKernelGGL(pack_full_k, dim3(nblk(2L * g.vh, 256)), dim3(256), 0, st, g, canon, fe, fo);
}
void launch_unpack_full(const Geom& g, const HalfField& fe, const HalfField& fo, double2* canon,
                        hipStream_t st) {
  hipLaunchKernelGGL(unpack_full_k, dim3(nblk(2L * g.vh, 256)), dim3(256), 0, st, g, fe, fo, canon);
}
void launch_convert_half(const Geom& g, const HalfField& src, const HalfField& dst, hipStream_t st) {
  hipLaunchKernelGGL(convert_half_k, dim3(nblk(g.vh, 256)), dim3(256), 0, st, g, src, dst);
}

}  // namespace ndtm
