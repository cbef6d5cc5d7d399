// Two-level aggregation multigrid kernels (section 3 and section 3.2):
// block orthonormalisation of the test vectors, the Galerkin coarse operator
// D_W,c = P^+ D_W P and C_o's block P^+ P_odd P, restriction (P x I2)^+,
// prolongation (P x I2), and the coarse doublet stencil
//   D'_c = D_W,c x I2 + i d mubar Gamma5_c x tau3 - epsbar I x tau1 + i m (Gamma5_c P^+P_odd P) x tau1.
//
// Storage: P[X][l][row][k] (row = spin*3 + colour, k < N_v; a row belongs to
// chirality spin/2, so column (chi, k) of P is nonzero only on its chirality's
// rows), coarse blocks D[X][b][j][i] (column-major so that the threads of one
// output row i read consecutive addresses), coarse vectors [X][flavour][chi*N_v + k].
#include <algorithm>
#include <cstdint>

#include "vec.h"

namespace ndtm {
namespace {

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cmulc(double2 a, double2 b) {  // conj(a) b
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }

struct SiteLoc {
  int par, h, t, z, y, x;
};

__device__ __forceinline__ SiteLoc agg_site(const MGGeom& m, int X, int l) {
  int r = X;
  const int cx = r % m.CX;
  r /= m.CX;
  const int cy = r % m.CY;
  r /= m.CY;
  const int cz = r % m.CZ;
  const int ct = r / m.CZ;
  int q = l;
  const int lx = q % m.bx;
  q /= m.bx;
  const int ly = q % m.by;
  q /= m.by;
  const int lz = q % m.bz;
  const int lt = q / m.bz;
  SiteLoc s;
  s.t = ct * m.bt + lt;
  s.z = cz * m.bz + lz;
  s.y = cy * m.by + ly;
  s.x = cx * m.bx + lx;
  const long site = (((long)s.t * m.Lz + s.z) * m.Ly + s.y) * m.Lx + s.x;
  s.par = (s.t + s.z + s.y + s.x) & 1;
  s.h = (int)(site >> 1);
  return s;
}

__device__ __forceinline__ void agg_local(const MGGeom& m, int l, int loc[4]) {
  // loc indexed by direction mu: 0 t, 1 x, 2 y, 3 z
  int q = l;
  loc[1] = q % m.bx;
  q /= m.bx;
  loc[2] = q % m.by;
  q /= m.by;
  loc[3] = q % m.bz;
  loc[0] = q / m.bz;
}

__device__ __forceinline__ int local_index(const MGGeom& m, const int loc[4]) {
  return ((loc[0] * m.bz + loc[3]) * m.by + loc[2]) * m.bx + loc[1];
}

// parity of coarse site X (sum of its coarse coordinates mod 2)
__device__ __forceinline__ int coarse_parity(const MGGeom& m, int X) {
  int r = X;
  const int cx = r % m.CX;
  r /= m.CX;
  const int cy = r % m.CY;
  r /= m.CY;
  const int cz = r % m.CZ;
  const int ct = r / m.CZ;
  return (ct + cz + cy + cx) & 1;
}

// neighbouring coarse site in direction mu (+1 or -1), periodic
__device__ __forceinline__ int coarse_nbr(const MGGeom& m, int X, int mu, int dir) {
  int r = X;
  int c[4];
  c[1] = r % m.CX;
  r /= m.CX;
  c[2] = r % m.CY;
  r /= m.CY;
  c[3] = r % m.CZ;
  c[0] = r / m.CZ;
  const int ext[4] = {m.CT, m.CX, m.CY, m.CZ};
  c[mu] = (c[mu] + dir + ext[mu]) % ext[mu];
  return ((c[0] * m.CZ + c[3]) * m.CY + c[2]) * m.CX + c[1];
}

// block sum of cnt doubles per thread; result in out[0..cnt) (shared), all threads synchronised
__device__ void block_reduce_batch(double* v, int cnt, double* lds, double* out) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  for (int i = 0; i < cnt; ++i) {
    double s = v[i];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off);
    if (lane == 0) lds[w * cnt + i] = s;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < cnt; i += blockDim.x) {
    double s = 0;
    for (int q = 0; q < nw; ++q) s += lds[q * cnt + i];
    out[i] = s;
  }
  __syncthreads();
}

// ---------------- test vectors -> P ----------------
__global__ void tv_to_P_k(MGGeom m, const double2* tv, double2* P) {
  const long idx = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (idx >= (long)m.Vc * m.nloc) return;
  const int X = idx / m.nloc, l = idx % m.nloc;
  const SiteLoc s = agg_site(m, X, l);
  const long site = (((long)s.t * m.Lz + s.z) * m.Ly + s.y) * m.Lx + s.x;
  const long V = (long)m.T * m.Lz * m.Ly * m.Lx;
  for (int r = 0; r < 12; ++r)
    for (int k = 0; k < m.Nv; ++k) P[(idx * 12 + r) * m.Nv + k] = tv[((long)k * V + site) * 12 + r];
}

struct FieldList {
  const double2* f[16];
};

__global__ void fields_to_P_k(MGGeom m, FieldList F, double2* P) {
  const long idx = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (idx >= (long)m.Vc * m.nloc) return;
  const int X = idx / m.nloc, l = idx % m.nloc;
  const SiteLoc s = agg_site(m, X, l);
  const long half = 24L * m.stride;
  for (int k = 0; k < m.Nv; ++k) {
    const double2* base = F.f[k >> 1] + s.par * half;
    const int f = k & 1;
    for (int r = 0; r < 12; ++r) P[(idx * 12 + r) * m.Nv + k] = base[(long)(f * 12 + r) * m.stride + s.h];
  }
}

// ---------------- block orthonormalisation ----------------
// one block per (X, chi); thread l holds the 6 rows of chirality chi at site l.
__global__ __launch_bounds__(256) void orthonormalize_k(MGGeom m, double2* P) {
  const int X = blockIdx.x >> 1, chi = blockIdx.x & 1;
  const int l = threadIdx.x;
  const bool on = l < m.nloc;
  __shared__ double lds[4 * 64];
  __shared__ double red[64];
  const int Nv = m.Nv;
  double2* Pl = P + ((long)X * m.nloc + (on ? l : 0)) * 12 * Nv;
  for (int k = 0; k < Nv; ++k) {
    double2 v[6];
    for (int r = 0; r < 6; ++r) v[r] = on ? Pl[(6 * chi + r) * Nv + k] : make_double2(0, 0);
    for (int pass = 0; pass < 2; ++pass) {
      // classical Gram-Schmidt against q_0..q_{k-1}, in chunks of 16 coefficients
      for (int j0 = 0; j0 < k; j0 += 16) {
        const int cnt = min(16, k - j0);
        double d[32];
        for (int j = 0; j < cnt; ++j) {
          double2 s = make_double2(0, 0);
          if (on)
            for (int r = 0; r < 6; ++r) s = cadd(s, cmulc(Pl[(6 * chi + r) * Nv + j0 + j], v[r]));
          d[2 * j] = s.x;
          d[2 * j + 1] = s.y;
        }
        block_reduce_batch(d, 2 * cnt, lds, red);
        if (on)
          for (int j = 0; j < cnt; ++j) {
            const double2 c = make_double2(red[2 * j], red[2 * j + 1]);
            for (int r = 0; r < 6; ++r) {
              const double2 t = cmul(c, Pl[(6 * chi + r) * Nv + j0 + j]);
              v[r].x -= t.x;
              v[r].y -= t.y;
            }
          }
        __syncthreads();
      }
    }
    double nn[1] = {0};
    for (int r = 0; r < 6; ++r) nn[0] += v[r].x * v[r].x + v[r].y * v[r].y;
    block_reduce_batch(nn, 1, lds, red);
    const double inv = 1.0 / sqrt(red[0]);
    if (on)
      for (int r = 0; r < 6; ++r) Pl[(6 * chi + r) * Nv + k] = make_double2(v[r].x * inv, v[r].y * inv);
    __syncthreads();
  }
}

// ---------------- Galerkin coarse operator ----------------
// Stored coarse blocks per coarse site: the self block and the forward hop of each
// direction, (2 N_v)^2 each; a backward hop is the Gamma5_c-conjugated adjoint of the
// neighbour's forward hop (D_c^+ = Gamma5_c D_c Gamma5_c).
constexpr int kCoarseBlocks = 5;
// gamma matrices of the chiral basis (same as the fine stencil): gamma[mu][row][col]
__constant__ double2 kGamma[4][4][4] = {
    // gamma_0 = [[0,-1],[-1,0]]
    {{{0, 0}, {0, 0}, {-1, 0}, {0, 0}},
     {{0, 0}, {0, 0}, {0, 0}, {-1, 0}},
     {{-1, 0}, {0, 0}, {0, 0}, {0, 0}},
     {{0, 0}, {-1, 0}, {0, 0}, {0, 0}}},
    // gamma_1 = [[0,-i s1],[i s1,0]], s1 = [[0,1],[1,0]]
    {{{0, 0}, {0, 0}, {0, 0}, {0, -1}},
     {{0, 0}, {0, 0}, {0, -1}, {0, 0}},
     {{0, 0}, {0, 1}, {0, 0}, {0, 0}},
     {{0, 1}, {0, 0}, {0, 0}, {0, 0}}},
    // gamma_2 = [[0,-i s2],[i s2,0]], s2 = [[0,-i],[i,0]] -> -i s2 = [[0,-1],[1,0]]
    {{{0, 0}, {0, 0}, {0, 0}, {-1, 0}},
     {{0, 0}, {0, 0}, {1, 0}, {0, 0}},
     {{0, 0}, {1, 0}, {0, 0}, {0, 0}},
     {{-1, 0}, {0, 0}, {0, 0}, {0, 0}}},
    // gamma_3 = [[0,-i s3],[i s3,0]], s3 = diag(1,-1)
    {{{0, 0}, {0, 0}, {0, -1}, {0, 0}},
     {{0, 0}, {0, 0}, {0, 0}, {0, 1}},
     {{0, 1}, {0, 0}, {0, 0}, {0, 0}},
     {{0, 0}, {0, -1}, {0, 0}, {0, 0}}}};

struct GalArgs {
  MGGeom m;
  const double2* U[2];  // FP64 links per parity, [(mu*9 + r*3 + c)*stride + h]
  int antiperiodic;
  const double2* P;
  double2* D;
  double2* scratch;
};

// block (X, dd): dd < 8 -> directional block d = dd from aggregate-boundary pairs;
// dd >= 8 -> partial self block from interior pairs of direction d = dd - 8.
__global__ __launch_bounds__(256) void galerkin_k(GalArgs A) {
  const MGGeom& m = A.m;
  const int X = blockIdx.x >> 4, dd = blockIdx.x & 15;
  const bool face = dd < 8;
  const int d = dd & 7, mu = d >> 1, bwd = d & 1;
  // the backward hopping blocks are not stored: D_c^+ = Gamma5_c D_c Gamma5_c gives them
  // from the forward block of the neighbour (section 3, Gamma5-compatible P)
  if (face && bwd) return;
  const int Nv = m.Nv, n2 = 2 * Nv;
  extern __shared__ double2 sm[];
  double2* Px = sm;               // 12 * Nv
  double2* Py = Px + 12 * Nv;     // 12 * Nv
  double2* Tm = Py + 12 * Nv;     // 12 * n2, [r][j]
  double2* Ul = Tm + 12 * n2;     // 9
  const int ntot = n2 * n2;
  constexpr int kPer = 16;        // output entries per thread (256*16 >= 64*64)
  double2 acc[kPer];
  for (int q = 0; q < kPer; ++q) acc[q] = make_double2(0, 0);
  const int bext[4] = {m.bt, m.bx, m.by, m.bz};
  for (int l = 0; l < m.nloc; ++l) {
    int loc[4];
    agg_local(m, l, loc);
    const bool at_face = bwd ? loc[mu] == 0 : loc[mu] == bext[mu] - 1;
    if (at_face != face) continue;
    // neighbour y = x +- mu: local index within its aggregate and its aggregate
    int nl[4] = {loc[0], loc[1], loc[2], loc[3]};
    int Y = X;
    if (at_face) {
      nl[mu] = bwd ? bext[mu] - 1 : 0;
      Y = coarse_nbr(m, X, mu, bwd ? -1 : 1);
    } else {
      nl[mu] += bwd ? -1 : 1;
    }
    const int ly = local_index(m, nl);
    const SiteLoc sx = agg_site(m, X, l);
    const SiteLoc sy = agg_site(m, Y, ly);
    const int ext[4] = {m.T, m.Lx, m.Ly, m.Lz};
    const int cx[4] = {sx.t, sx.x, sx.y, sx.z};
    double sg = 1.0;
    if (A.antiperiodic && mu == 0 && ((!bwd && cx[0] == ext[0] - 1) || (bwd && cx[0] == 0))) sg = -1.0;
    __syncthreads();
    for (int e = threadIdx.x; e < 12 * Nv; e += blockDim.x) {
      Px[e] = A.P[((long)X * m.nloc + l) * 12 * Nv + e];
      Py[e] = A.P[((long)Y * m.nloc + ly) * 12 * Nv + e];
    }
    if (threadIdx.x < 9) {
      // forward: U_mu(x) at x; backward: U_mu(y) at y (used daggered)
      const SiteLoc& su = bwd ? sy : sx;
      Ul[threadIdx.x] = A.U[su.par][(long)(mu * 9 + threadIdx.x) * m.stride + su.h];
    }
    __syncthreads();
    // T[r][j] = -1/2 sg ((1 -+ gamma_mu) x U^(+)) P_y[:, j]
    for (int e = threadIdx.x; e < 12 * n2; e += blockDim.x) {
      const int r = e / n2, j = e % n2;
      const int s = r / 3, c = r % 3;
      const int chj = j / Nv, kj = j % Nv;
      double2 up[2];  // (U P_y)[s'][c][j] for the two spins s' of chirality chj
      for (int q = 0; q < 2; ++q) {
        const int sp = 2 * chj + q;
        double2 t = make_double2(0, 0);
        for (int cc = 0; cc < 3; ++cc) {
          const double2 pv = Py[(sp * 3 + cc) * Nv + kj];
          t = cadd(t, bwd ? cmulc(Ul[cc * 3 + c], pv) : cmul(Ul[c * 3 + cc], pv));
        }
        up[q] = t;
      }
      double2 tv = make_double2(0, 0);
      if ((s >> 1) == chj) tv = up[s & 1];
      for (int q = 0; q < 2; ++q) {
        const double2 gm = cmul(kGamma[mu][s][2 * chj + q], up[q]);
        tv.x += bwd ? gm.x : -gm.x;
        tv.y += bwd ? gm.y : -gm.y;
      }
      Tm[e] = make_double2(-0.5 * sg * tv.x, -0.5 * sg * tv.y);
    }
    __syncthreads();
    for (int q = 0; q < kPer; ++q) {
      const int o = threadIdx.x + q * blockDim.x;
      if (o >= ntot) break;
      const int j = o / n2, i = o % n2;
      const int chi = i / Nv, ki = i % Nv;
      double2 s = acc[q];
      for (int rr = 0; rr < 6; ++rr) {
        const int r = 6 * chi + rr;
        s = cadd(s, cmulc(Px[r * Nv + ki], Tm[r * n2 + j]));
      }
      acc[q] = s;
    }
  }
  double2* out = face ? A.D + ((long)X * kCoarseBlocks + 1 + mu) * ntot : A.scratch + ((long)X * 8 + d) * ntot;
  for (int q = 0; q < kPer; ++q) {
    const int o = threadIdx.x + q * blockDim.x;
    if (o < ntot) out[o] = acc[q];
  }
}

__global__ void galerkin_self_k(MGGeom m, double a, const double2* scratch, double2* D) {
  const int X = blockIdx.x;
  const int n2 = 2 * m.Nv, ntot = n2 * n2;
  for (int o = threadIdx.x; o < ntot; o += blockDim.x) {
    double2 s = make_double2((o / n2 == o % n2) ? a : 0.0, 0.0);
    for (int d = 0; d < 8; ++d) s = cadd(s, scratch[((long)X * 8 + d) * ntot + o]);
    D[(long)X * kCoarseBlocks * ntot + o] = s;
  }
}

// element (r, r') of the packed Hermitian 6x6 (6 real diagonal entries, then the upper
// entries row by row as re, im) at half-site h of component arrays of `stride` entries
__device__ double2 herm6_elem(const double* M, int stride, long h, int r, int rp) {
  if (r == rp) return make_double2(M[(long)r * stride + h], 0.0);
  const int i = r < rp ? r : rp, j = r < rp ? rp : r;
  const int k = 6 + 2 * (i * 6 - i * (i + 1) / 2 + (j - i - 1));
  const double re = M[(long)k * stride + h], im = M[(long)(k + 1) * stride + h];
  return r < rp ? make_double2(re, im) : make_double2(re, -im);
}

// Clover part of the Galerkin self block: D[X][0] += sum_l P_l^+ C(x_l) P_l per chirality,
// with C = M - a read from the fine site blocks M = a + C (eq:Wilson's clover term on the
// coarse grid, section 3).  Entry (row i, column j) sits at j * 2Nv + i.
__global__ void galerkin_clover_k(MGGeom m, const double2* P, const double* Me, const double* Mo, double a,
                                  double2* D) {
  const int X = blockIdx.x;
  const int Nv = m.Nv, n2 = 2 * Nv, nb = Nv * Nv;
  for (int o = threadIdx.x; o < 2 * nb; o += blockDim.x) {
    const int chi = o / nb, k = (o % nb) / Nv, kp = o % Nv;
    double2 s = make_double2(0, 0);
    for (int l = 0; l < m.nloc; ++l) {
      const SiteLoc sl = agg_site(m, X, l);
      const double* Mp = (sl.par ? Mo : Me) + (long)chi * 36 * m.stride;
      const double2* Pl = P + ((long)X * m.nloc + l) * 12 * Nv;
      for (int r = 0; r < 6; ++r) {
        double2 t = make_double2(0, 0);
        for (int rp = 0; rp < 6; ++rp) {
          double2 e = herm6_elem(Mp, m.stride, sl.h, r, rp);
          if (r == rp) e.x -= a;
          t = cadd(t, cmul(e, Pl[(6 * chi + rp) * Nv + kp]));
        }
        s = cadd(s, cmulc(Pl[(6 * chi + r) * Nv + k], t));
      }
    }
    const int i = chi * Nv + k, j = chi * Nv + kp;
    double2* d = D + (long)X * kCoarseBlocks * n2 * n2 + (long)j * n2 + i;
    *d = cadd(*d, s);
  }
}

// B_o[X][chi][k][k'] = sum_{odd l} sum_{rows of chi} conj(P[l][r][k]) P[l][r][k']
__global__ void odd_block_k(MGGeom m, const double2* P, double2* Bo) {
  const int X = blockIdx.x;
  const int Nv = m.Nv, nb = Nv * Nv;
  for (int o = threadIdx.x; o < 2 * nb; o += blockDim.x) {
    const int chi = o / nb, k = (o % nb) / Nv, kp = o % Nv;
    double2 s = make_double2(0, 0);
    for (int l = 0; l < m.nloc; ++l) {
      const SiteLoc sl = agg_site(m, X, l);
      if (!sl.par) continue;
      const double2* Pl = P + ((long)X * m.nloc + l) * 12 * Nv;
      for (int rr = 0; rr < 6; ++rr) {
        const int r = 6 * chi + rr;
        s = cadd(s, cmulc(Pl[r * Nv + k], Pl[r * Nv + kp]));
      }
    }
    Bo[(long)X * 2 * nb + o] = s;
  }
}

// ---------------- restriction / prolongation ----------------
template <class R>
struct C2;
template <>
struct C2<double> {
  using T = double2;
};
template <>
struct C2<float> {
  using T = float2;
};

template <class R>
__device__ __forceinline__ typename C2<R>::T mk(R x, R y) {
  typename C2<R>::T v;
  v.x = x;
  v.y = y;
  return v;
}

constexpr int kGroups = 8;       // thread groups per coarse site in the restriction
constexpr int kApplyGroups = 8;  // thread groups per coarse site in the coarse stencil

// element of component c at half-site h of a fine field in the cycle precision R
template <class R>
__device__ __forceinline__ long fine_idx(int c, int stride, long h) {
  if constexpr (sizeof(R) == 8) return (long)c * stride + h;
  else return idx32(c, stride, h);
}

// Coarse site of a transfer block: XCD k = blockIdx % 8 takes one contiguous range of
// coarse sites, so neighbouring aggregates, which share the cache lines of the fine
// field, run on the same XCD and its L2 (dealt round-robin, each XCD fetched every
// such line itself).  A bijection onto [0, gridDim) for any grid size.
__device__ __forceinline__ int xcd_site(int b, int nb) {
  const int q = nb >> 3, rem = nb & 7, xcd = b & 7, loc = b >> 3;
  return xcd * q + min(xcd, rem) + loc;
}

// P in the cycle precision, or (PH) in FP16 with one FP32 scale per fine site (the
// largest magnitude of the site's 12 N_v entries), read as scale * entry in FP32
template <class R, bool PH>
struct PStore {
  using T = typename C2<R>::T;
};
template <>
struct PStore<float, true> {
  using T = __half2;
};
template <class R, bool PH>
__device__ __forceinline__ typename C2<R>::T p_at(const typename PStore<R, PH>::T* P, long i, R sc) {
  if constexpr (PH) {
    const float2 f = __half22float2(P[i]);
    return mk<R>(sc * f.x, sc * f.y);
  } else {
    return P[i];
  }
}

template <class R, bool PH>
__global__ __launch_bounds__(1024) void restrict_k(MGGeom m, const typename PStore<R, PH>::T* P, const float* Psc,
                                                  const typename C2<R>::T* fe, const typename C2<R>::T* fo,
                                                  typename C2<R>::T* vc) {
  using T2 = typename C2<R>::T;
  using PT = typename PStore<R, PH>::T;
  const int X = xcd_site(blockIdx.x, gridDim.x);
  const int Nv = m.Nv, n2 = 2 * Nv, nout = 2 * n2;
  __shared__ int ph[1024];
  __shared__ R red[kGroups][2][128];
  for (int l = threadIdx.x; l < m.nloc; l += blockDim.x) {
    const SiteLoc s = agg_site(m, X, l);
    ph[l] = (s.h << 1) | s.par;
  }
  __syncthreads();
  // lane t of a group takes flavour t & 1 of output row t >> 1: the two flavour lanes
  // of a row are neighbours, so their loads of the same element of P are one request
  // (with the flavours n2 lanes apart they fell in different waves, and the second
  // read could miss the L2)
  const int t = threadIdx.x % nout, q = threadIdx.x / nout;
  R ax = 0, ay = 0;
  if (q < kGroups) {
    const int f = t & 1, i = t >> 1, chi = i / Nv, k = i % Nv;
    const PT* PX = P + (long)X * m.nloc * 12 * Nv;
    for (int l = q; l < m.nloc; l += kGroups) {
      const int hp = ph[l];
      const T2* F = (hp & 1) ? fo : fe;
      const int h = hp >> 1;
      const R sc = PH ? (R)Psc[(long)X * m.nloc + l] : R(1);
#pragma unroll
      for (int rr = 0; rr < 6; ++rr) {
        const int r = 6 * chi + rr;
        const T2 p = p_at<R, PH>(PX, ((long)l * 12 + r) * Nv + k, sc);
        const T2 v = F[fine_idx<R>(f * 12 + r, m.stride, h)];
        ax += p.x * v.x + p.y * v.y;
        ay += p.x * v.y - p.y * v.x;
      }
    }
    red[q][0][t] = ax;
    red[q][1][t] = ay;
  }
  __syncthreads();
  if (threadIdx.x < nout) {
    // output element (f, i) = threadIdx.x = f n2 + i, held by lane 2 i + f
    const int tt = 2 * (threadIdx.x % n2) + threadIdx.x / n2;
    R sx = 0, sy = 0;
    for (int g = 0; g < kGroups; ++g) {
      sx += red[g][0][tt];
      sy += red[g][1][tt];
    }
    vc[(long)X * nout + threadIdx.x] = mk<R>(sx, sy);
  }
}

template <class R, bool PH>
__global__ __launch_bounds__(256) void prolong_k(MGGeom m, const typename PStore<R, PH>::T* P, const float* Psc,
                                                 const typename C2<R>::T* vc, typename C2<R>::T* fe,
                                                 typename C2<R>::T* fo) {
  using T2 = typename C2<R>::T;
  using PT = typename PStore<R, PH>::T;
  const int X = xcd_site(blockIdx.x, gridDim.x);
  const int Nv = m.Nv, n2 = 2 * Nv;
  __shared__ T2 cv[2 * 64];
  __shared__ int ph[1024];
  for (int e = threadIdx.x; e < 2 * n2; e += blockDim.x) cv[e] = vc[(long)X * 2 * n2 + e];
  for (int l = threadIdx.x; l < m.nloc; l += blockDim.x) {
    const SiteLoc s = agg_site(m, X, l);
    ph[l] = (s.h << 1) | s.par;
  }
  __syncthreads();
  const PT* PX = P + (long)X * m.nloc * 12 * Nv;
  for (int e = threadIdx.x; e < m.nloc * 12; e += blockDim.x) {
    const int l = e / 12, r = e % 12, chi = r / 6;
    R a0x = 0, a0y = 0, a1x = 0, a1y = 0;
    const PT* pr = PX + ((long)l * 12 + r) * Nv;
    const R sc = PH ? (R)Psc[(long)X * m.nloc + l] : R(1);
    for (int k = 0; k < Nv; ++k) {
      const T2 p = p_at<R, PH>(pr, k, sc);
      const T2 c0 = cv[chi * Nv + k], c1 = cv[n2 + chi * Nv + k];
      a0x += p.x * c0.x - p.y * c0.y;
      a0y += p.x * c0.y + p.y * c0.x;
      a1x += p.x * c1.x - p.y * c1.y;
      a1y += p.x * c1.y + p.y * c1.x;
    }
    const int hp = ph[l];
    T2* F = (hp & 1) ? fo : fe;
    const int h = hp >> 1;
    F[fine_idx<R>(r, m.stride, h)] = mk<R>(a0x, a0y);
    F[fine_idx<R>(12 + r, m.stride, h)] = mk<R>(a1x, a1y);
  }
}

// ---------------- coarse stencil ----------------
// y = D'_c x.  With xnorm2 the input is x / sqrt(*xnorm2) (scaled as it is read,
// with the rounding of a separate scaling pass), and xout, when given, receives the
// scaled input of the block's own site: the coarse Arnoldi step normalises its new
// basis vector this way instead of in a pass of its own.
template <class R>
__global__ __launch_bounds__(512) void coarse_apply_k(MGGeom m, const typename C2<R>::T* D,
                                                      const typename C2<R>::T* Bo, const typename C2<R>::T* x,
                                                      typename C2<R>::T* y, double mubar_c, double epsbar,
                                                      double mm, const double* xnorm2, typename C2<R>::T* xout,
                                                      int par_out) {
  using T2 = typename C2<R>::T;
  const int X = blockIdx.x;
  // par_out >= 0: only the output sites of that coarse parity (the others keep their values)
  if (par_out >= 0 && coarse_parity(m, X) != par_out) return;
  const int Nv = m.Nv, n2 = 2 * Nv, ntot = n2 * n2, nout = 2 * n2;
  __shared__ T2 xs[9][2 * 64];
  __shared__ int nb[9];
  __shared__ R red2[kApplyGroups][2][128];
  if (threadIdx.x < 9) {
    const int b = threadIdx.x;
    nb[b] = b == 0 ? X : coarse_nbr(m, X, (b - 1) >> 1, ((b - 1) & 1) ? -1 : 1);
  }
  __syncthreads();
  const double sc = xnorm2 ? (*xnorm2 > 1e-300 ? 1.0 / sqrt(*xnorm2) : 0.0) : 1.0;
  for (int e = threadIdx.x; e < 9 * nout; e += blockDim.x) {
    const int b = e / nout, q = e % nout;
    const T2 v = x[(long)nb[b] * nout + q];
    xs[b][q] = xnorm2 ? mk<R>(R(sc * double(v.x)), R(sc * double(v.y))) : v;
  }
  __syncthreads();
  if (xout)
    for (int e = threadIdx.x; e < nout; e += blockDim.x) xout[(long)X * nout + e] = xs[0][e];
  // thread (q, i): row i of both flavours (each block element is read once and
  // used for the two flavour columns) over the pairs p = b * n2 + j with
  // p = q mod kApplyGroups
  {
    const int i = threadIdx.x % n2, q = threadIdx.x / n2;
    if (q < kApplyGroups) {
      R a0x = 0, a0y = 0, a1x = 0, a1y = 0;
      const R si = i < Nv ? R(1) : R(-1);
#pragma unroll 4
      for (int pidx = q; pidx < 9 * n2; pidx += kApplyGroups) {
        const int b = pidx / n2, j = pidx % n2;
        T2 dv;
        if (b == 0 || (b & 1)) {
          // self block and forward hops: stored at the site, entry (i, j) at j * 2Nv + i
          dv = D[((long)X * kCoarseBlocks + (b + 1) / 2) * ntot + (long)j * n2 + i];
        } else {
          // backward hop mu: Gamma5_c F^+ Gamma5_c with F the forward block of the
          // neighbour X - mu, entry (i, j) = s_i s_j conj(F_ji)
          const T2 f = D[((long)nb[b] * kCoarseBlocks + b / 2) * ntot + (long)i * n2 + j];
          const R sg = (j < Nv ? R(1) : R(-1)) * si;
          dv = mk<R>(sg * f.x, -sg * f.y);
        }
        const T2 v0 = xs[b][j], v1 = xs[b][n2 + j];
        a0x += dv.x * v0.x - dv.y * v0.y;
        a0y += dv.x * v0.y + dv.y * v0.x;
        a1x += dv.x * v1.x - dv.y * v1.y;
        a1y += dv.x * v1.y + dv.y * v1.x;
      }
      red2[q][0][i] = a0x;
      red2[q][1][i] = a0y;
      red2[q][0][n2 + i] = a1x;
      red2[q][1][n2 + i] = a1y;
    }
  }
  __syncthreads();
  if (threadIdx.x >= nout) return;
  const int t = threadIdx.x, f = t / n2, i = t % n2;
  R ax = 0, ay = 0;
  for (int g = 0; g < kApplyGroups; ++g) {
    ax += red2[g][0][t];
    ay += red2[g][1][t];
  }
  const int chi = i / Nv, k = i % Nv;
  const R g5 = chi == 0 ? R(1) : R(-1);
  const R t3 = f == 0 ? R(1) : R(-1);
  const T2 xself = xs[0][f * n2 + i];
  const T2 xoth = xs[0][(1 - f) * n2 + i];
  // + i d mubar g5 tau3 x_f - epsbar x_{1-f}
  ax += -R(mubar_c) * g5 * t3 * xself.y - R(epsbar) * xoth.x;
  ay += R(mubar_c) * g5 * t3 * xself.x - R(epsbar) * xoth.y;
  if (mm != 0.0) {
    // + i m g5 sum_k' Bo[chi][k][k'] x_{1-f}[chi, k']
    const T2* B = Bo + ((long)X * 2 + chi) * Nv * Nv + (long)k * Nv;
    const T2* xo = xs[0] + (1 - f) * n2 + chi * Nv;
    R bx = 0, by = 0;
    for (int kp = 0; kp < Nv; ++kp) {
      const T2 bv = B[kp], v = xo[kp];
      bx += bv.x * v.x - bv.y * v.y;
      by += bv.x * v.y + bv.y * v.x;
    }
    ax += -R(mm) * g5 * by;
    ay += R(mm) * g5 * bx;
  }
  y[((long)X * 2 + f) * n2 + i] = mk<R>(ax, ay);
}

// ---------------- batched coarse stencil on MFMA ----------------
// Up to kMultiMax coarse systems D'_c(m_r) x_r at once (FP64).  The hopping and
// self blocks D_b are shared by all systems and both flavours, so per coarse site
// the products form one complex (2Nv) x (9 * 2Nv) by (9 * 2Nv) x (2k) matrix
// product, columns n = f k + r.  Each wave takes a tile of 16 rows and all 2k <= 16
// columns with v_mfma_f64_16x16x4f64 (four real products per complex one):
//   A (16x4): lane l holds row l % 16, column l / 16 of the D block;
//   B (4x16): lane l holds row l / 16, column l % 16 of the neighbour vectors;
//   C (16x16): lane l, register q holds row 4 q + l / 16, column l % 16.
// The site terms (i d mubar Gamma5 tau3, -epsbar tau1, i m_r C_o tau1) follow per
// output element, as in coarse_apply_k.  Rows beyond 2Nv are masked.
struct MultiM {
  double m[kMultiMax];
};
typedef double mf_d4 __attribute__((ext_vector_type(4)));

// The nine blocks are split over kMultiBGroups groups of waves (more waves in
// flight per coarse site); the groups' partial tiles are summed through LDS.
constexpr int kMultiBGroups = 3;
constexpr int kMultiMaxTiles = 4;  // 2 N_v <= 64
__global__ __launch_bounds__(64 * kMultiBGroups * kMultiMaxTiles) void coarse_apply_multi_k(
    MGGeom g, const double2* D, const double2* Bo, const double2* X, double2* Y, int k, MultiM ms, double mubar_c,
    double epsbar) {
  const int site = blockIdx.x;
  const int Nv = g.Nv, n2 = 2 * Nv, ntot = n2 * n2;
  const size_t vstride = (size_t)g.Vc * 2 * n2;  // one system's coarse vector
  __shared__ int nb[9];
  if (threadIdx.x < 9) {
    const int b = threadIdx.x;
    nb[b] = b == 0 ? site : coarse_nbr(g, site, (b - 1) >> 1, ((b - 1) & 1) ? -1 : 1);
  }
  __shared__ double part[kMultiBGroups - 1][kMultiMaxTiles][2][4][64];
  __syncthreads();
  const int tiles = (n2 + 15) / 16;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, mt = w % tiles, bg = w / tiles;
  const int ia = mt * 16 + (lane & 15), kq = lane >> 4;  // A element of this lane
  const int col = lane & 15;                             // B column / C column
  const bool cvalid = col < 2 * k;
  const int cf = cvalid ? col / k : 0, cr = cvalid ? col % k : 0;
  mf_d4 accr = {0, 0, 0, 0}, acci = {0, 0, 0, 0};
  // operands of four k-steps are loaded (from clamped, always valid addresses) before
  // their products, so that the loads are in flight together; masked entries are zeroed
  const int iac = ia < n2 ? ia : n2 - 1;
  const bool rowok = ia < n2;
  const double si = iac < Nv ? 1.0 : -1.0;
  for (int b = bg * (9 / kMultiBGroups); b < (bg + 1) * (9 / kMultiBGroups); ++b) {
    // logical block b: self (0), forward hop mu (1 + 2 mu), backward hop mu (2 + 2 mu), the
    // latter from the neighbour's stored forward block as Gamma5_c F^+ Gamma5_c
    const bool adj = b > 0 && !(b & 1);
    const double2* Db = adj ? D + ((size_t)nb[b] * kCoarseBlocks + b / 2) * ntot
                            : D + ((size_t)site * kCoarseBlocks + (b + 1) / 2) * ntot;
    const double2* xb = X + (size_t)cr * vstride + ((size_t)nb[b] * 2 + cf) * n2;
    for (int kk = 0; kk < n2; kk += 16) {
      double2 a[4], v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int jj = kk + 4 * u + kq;
        const int jc = jj < n2 ? jj : n2 - 1;
        if (adj) {
          const double2 f = Db[(size_t)iac * n2 + jc];
          const double sg = (jc < Nv ? 1.0 : -1.0) * si;
          a[u] = make_double2(sg * f.x, -sg * f.y);
        } else {
          a[u] = Db[(size_t)jc * n2 + iac];
        }
        v[u] = xb[jc];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int jj = kk + 4 * u + kq;
        const double fa = (rowok && jj < n2) ? 1.0 : 0.0, fv = (cvalid && jj < n2) ? 1.0 : 0.0;
        const double ar = fa * a[u].x, ai = fa * a[u].y, vr = fv * v[u].x, vi = fv * v[u].y;
        accr = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, vr, accr, 0, 0, 0);
        accr = __builtin_amdgcn_mfma_f64_16x16x4f64(-ai, vi, accr, 0, 0, 0);
        acci = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, vi, acci, 0, 0, 0);
        acci = __builtin_amdgcn_mfma_f64_16x16x4f64(ai, vr, acci, 0, 0, 0);
      }
    }
  }
  if (bg > 0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      part[bg - 1][mt][0][q][lane] = accr[q];
      part[bg - 1][mt][1][q][lane] = acci[q];
    }
  }
  __syncthreads();
  if (bg > 0) return;
#pragma unroll
  for (int q = 0; q < 4; ++q)
    for (int h = 0; h < kMultiBGroups - 1; ++h) {
      accr[q] += part[h][mt][0][q][lane];
      acci[q] += part[h][mt][1][q][lane];
    }
  if (!cvalid) return;
  const double2* xs = X + (size_t)cr * vstride + (size_t)site * 2 * n2;
  const double mm = ms.m[cr];
  const double t3 = cf == 0 ? 1.0 : -1.0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int i = mt * 16 + 4 * q + (lane >> 4);
    if (i >= n2) continue;
    const int chi = i / Nv, kk = i % Nv;
    const double g5 = chi == 0 ? 1.0 : -1.0;
    const double2 xself = xs[cf * n2 + i], xoth = xs[(1 - cf) * n2 + i];
    double ax = accr[q], ay = acci[q];
    // + i d mubar g5 tau3 x_f - epsbar x_{1-f}
    ax += -mubar_c * g5 * t3 * xself.y - epsbar * xoth.x;
    ay += mubar_c * g5 * t3 * xself.x - epsbar * xoth.y;
    if (mm != 0.0) {
      // + i m g5 sum_k' Bo[chi][k][k'] x_{1-f}[chi, k']
      const double2* B = Bo + ((size_t)site * 2 + chi) * Nv * Nv + (size_t)kk * Nv;
      const double2* xo = xs + (1 - cf) * n2 + chi * Nv;
      double bx = 0, by = 0;
      for (int kp = 0; kp < Nv; ++kp) {
        const double2 bv = B[kp], v = xo[kp];
        bx += bv.x * v.x - bv.y * v.y;
        by += bv.x * v.y + bv.y * v.x;
      }
      ax += -mm * g5 * by;
      ay += mm * g5 * bx;
    }
    Y[(size_t)cr * vstride + ((size_t)site * 2 + cf) * n2 + i] = make_double2(ax, ay);
  }
}

// ---------------- random test vectors ----------------
__device__ __forceinline__ uint64_t splitmix(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__global__ void random_fill_k(int vh, int stride, double2* fe, double2* fo, unsigned long long seed) {
  const long idx = blockIdx.x * (long)blockDim.x + threadIdx.x;  // over 2 * 24 * vh
  if (idx >= 48L * vh) return;
  const int half = idx / (24L * vh);
  const long r = idx % (24L * vh);
  const int comp = r / vh, h = r % vh;
  const uint64_t a = splitmix(seed * 0x100000001B3ull + (uint64_t)idx * 2);
  const uint64_t b = splitmix(seed * 0x100000001B3ull + (uint64_t)idx * 2 + 1);
  const double u1 = ((a >> 11) + 0.5) * (1.0 / 9007199254740992.0);
  const double u2 = ((b >> 11) + 0.5) * (1.0 / 9007199254740992.0);
  const double rad = sqrt(-2.0 * log(u1));
  double sn, cs;
  sincos(6.283185307179586 * u2, &sn, &cs);
  (half ? fo : fe)[(long)comp * stride + h] = make_double2(rad * cs, rad * sn);
}

inline unsigned nb(long n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

void mg_tv_to_P(const MGGeom& m, const double2* tv, double2* P, hipStream_t st) {
  hipLaunchKernelGGL(tv_to_P_k, dim3(nb((long)m.Vc * m.nloc, 128)), dim3(128), 0, st, m, tv, P);
}

void mg_fields_to_P(const MGGeom& m, const double2* const* fields, int nfields, double2* P, hipStream_t st) {
  FieldList F{};
  for (int i = 0; i < nfields && i < 16; ++i) F.f[i] = fields[i];
  hipLaunchKernelGGL(fields_to_P_k, dim3(nb((long)m.Vc * m.nloc, 128)), dim3(128), 0, st, m, F, P);
}

void mg_orthonormalize(const MGGeom& m, double2* P, hipStream_t st) {
  hipLaunchKernelGGL(orthonormalize_k, dim3(2 * m.Vc), dim3(256), 0, st, m, P);
}

void mg_galerkin(const MGGeom& m, const double2* U64e, const double2* U64o, int antiperiodic, double a,
                 const double2* P, double2* D, double2* scratch, double2* Bo, hipStream_t st) {
  GalArgs A;
  A.m = m;
  A.U[0] = U64e;
  A.U[1] = U64o;
  A.antiperiodic = antiperiodic;
  A.P = P;
  A.D = D;
  A.scratch = scratch;
  const int n2 = 2 * m.Nv;
  const size_t shmem = (size_t)(24 * m.Nv + 12 * n2 + 9) * sizeof(double2);
  hipLaunchKernelGGL(galerkin_k, dim3(16 * m.Vc), dim3(256), shmem, st, A);
  hipLaunchKernelGGL(galerkin_self_k, dim3(m.Vc), dim3(256), 0, st, m, a, scratch, D);
  hipLaunchKernelGGL(odd_block_k, dim3(m.Vc), dim3(256), 0, st, m, P, Bo);
}

void mg_galerkin_clover(const MGGeom& m, const double2* P, const double* Me, const double* Mo, double a, double2* D,
                        hipStream_t st) {
  hipLaunchKernelGGL(galerkin_clover_k, dim3(m.Vc), dim3(256), 0, st, m, P, Me, Mo, a, D);
}

void mg_restrict(int prec, const MGGeom& m, const void* P, const float* Psc, const void* fe, const void* fo, void* vc,
                 hipStream_t st) {
  const dim3 grid(m.Vc), blk(4 * m.Nv * kGroups);
  if (prec == P64)
    hipLaunchKernelGGL((restrict_k<double, false>), grid, blk, 0, st, m, (const double2*)P, nullptr,
                       (const double2*)fe, (const double2*)fo, (double2*)vc);
  else if (Psc)
    hipLaunchKernelGGL((restrict_k<float, true>), grid, blk, 0, st, m, (const __half2*)P, Psc, (const float2*)fe,
                       (const float2*)fo, (float2*)vc);
  else
    hipLaunchKernelGGL((restrict_k<float, false>), grid, blk, 0, st, m, (const float2*)P, nullptr,
                       (const float2*)fe, (const float2*)fo, (float2*)vc);
}

void mg_prolong(int prec, const MGGeom& m, const void* P, const float* Psc, const void* vc, void* fe, void* fo,
                hipStream_t st) {
  if (prec == P64)
    hipLaunchKernelGGL((prolong_k<double, false>), dim3(m.Vc), dim3(256), 0, st, m, (const double2*)P, nullptr,
                       (const double2*)vc, (double2*)fe, (double2*)fo);
  else if (Psc)
    hipLaunchKernelGGL((prolong_k<float, true>), dim3(m.Vc), dim3(256), 0, st, m, (const __half2*)P, Psc,
                       (const float2*)vc, (float2*)fe, (float2*)fo);
  else
    hipLaunchKernelGGL((prolong_k<float, false>), dim3(m.Vc), dim3(256), 0, st, m, (const float2*)P, nullptr,
                       (const float2*)vc, (float2*)fe, (float2*)fo);
}

// P (FP64, [aggregate][site][row][k]) to FP16 entries with one FP32 scale per fine site
__global__ void p_to_half_k(long nsites, int per, const double2* P, __half2* P16, float* Psc) {
  const long s = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (s >= nsites) return;
  const double2* src = P + s * per;
  double mx = 0;
  for (int i = 0; i < per; ++i) mx = fmax(mx, fmax(fabs(src[i].x), fabs(src[i].y)));
  const float sc = (float)mx;
  const double inv = sc > 0.f ? 1.0 / (double)sc : 0.0;
  for (int i = 0; i < per; ++i) P16[s * per + i] = __floats2half2_rn((float)(src[i].x * inv), (float)(src[i].y * inv));
  Psc[s] = sc;
}

void mg_p_to_half(const MGGeom& m, const void* P64, void* P16, float* Psc, hipStream_t st) {
  const long ns = (long)m.Vc * m.nloc;
  hipLaunchKernelGGL(p_to_half_k, dim3((unsigned)((ns + 255) / 256)), dim3(256), 0, st, ns, 12 * m.Nv,
                     (const double2*)P64, (__half2*)P16, Psc);
}

void mg_coarse_apply(int prec, const MGGeom& g, const void* D, const void* Bo, const void* x, void* y,
                     double mubar_c, double epsbar, double m, hipStream_t st, const double* xnorm2, void* xout,
                     int par_out) {
  const dim3 blk(std::max(2 * g.Nv * kApplyGroups, 4 * g.Nv));
  if (prec == P64)
    hipLaunchKernelGGL(coarse_apply_k<double>, dim3(g.Vc), blk, 0, st, g, (const double2*)D, (const double2*)Bo,
                       (const double2*)x, (double2*)y, mubar_c, epsbar, m, xnorm2, (double2*)xout, par_out);
  else
    hipLaunchKernelGGL(coarse_apply_k<float>, dim3(g.Vc), blk, 0, st, g, (const float2*)D, (const float2*)Bo,
                       (const float2*)x, (float2*)y, mubar_c, epsbar, m, xnorm2, (float2*)xout, par_out);
}

// ---------------- even-odd coarsest level ----------------
// The site term of D'_c(m) at coarse site X couples both flavours:
//   rows/columns (f, i), i < 2Nv:  (f, f): S_X + i d mubar g5_i tau3_f;
//   (f, 1-f): -epsbar + i m g5_i Bo_X (chirality-diagonal),
// S_X the self block.  One workgroup per even coarse site inverts it in FP64 by
// Gauss-Jordan elimination with partial pivoting on [A | 1] (rows of 4 n2 complex in
// the scratch), and stores -A^-1 in the cycle precision, entry (r, c) at c * 2n2 + r,
// at the even site's compact index X / 2.  *bad counts singular site terms.
template <class R>
__global__ __launch_bounds__(256) void einv_build_k(MGGeom m, int X0, const typename C2<R>::T* D,
                                                     const typename C2<R>::T* Bo, double mubar_c, double epsbar,
                                                     double mm, double2* scratch, typename C2<R>::T* Einv,
                                                     unsigned* bad) {
  using T2 = typename C2<R>::T;
  const int X = X0 + blockIdx.x;  // X0 even; the scratch holds the chunk's even sites
  if (X >= m.Vc || coarse_parity(m, X) != 0) return;
  const int Nv = m.Nv, n2 = 2 * Nv, N = 2 * n2, W = 2 * N;
  double2* A = scratch + (size_t)((X - X0) >> 1) * N * W;  // [row][W]
  const T2* S = D + (size_t)X * kCoarseBlocks * n2 * n2;
  const T2* B = Bo + (size_t)X * 2 * Nv * Nv;
  for (int e = threadIdx.x; e < N * W; e += blockDim.x) {
    const int r = e / W, c = e % W;
    double2 v = make_double2(0, 0);
    if (c < N) {
      const int fr = r / n2, i = r % n2, fc = c / n2, j = c % n2;
      const double g5 = i < Nv ? 1.0 : -1.0;
      if (fr == fc) {
        const T2 d = S[(size_t)j * n2 + i];
        v = make_double2(double(d.x), double(d.y));
        if (i == j) v.y += mubar_c * g5 * (fr == 0 ? 1.0 : -1.0);
      } else {
        if (i == j) v.x -= epsbar;
        const int chi = i / Nv;
        if (mm != 0.0 && j / Nv == chi) {
          const T2 b = B[((size_t)chi * Nv + i % Nv) * Nv + j % Nv];
          // + i m g5 b
          v.x -= mm * g5 * double(b.y);
          v.y += mm * g5 * double(b.x);
        }
      }
    } else if (c - N == r) {
      v = make_double2(1, 0);
    }
    A[e] = v;
  }
  __shared__ double bv[256];
  __shared__ int bi[256];
  __shared__ double2 piv;
  __shared__ int prow;
  __shared__ double2 fcol[128];
  for (int c = 0; c < N; ++c) {
    __syncthreads();
    // pivot: largest |A[r][c]| over r >= c
    double best = -1.0;
    int bestr = c;
    for (int r = c + threadIdx.x; r < N; r += blockDim.x) {
      const double2 a = A[(size_t)r * W + c];
      const double v = a.x * a.x + a.y * a.y;
      if (v > best) {
        best = v;
        bestr = r;
      }
    }
    bv[threadIdx.x] = best;
    bi[threadIdx.x] = bestr;
    __syncthreads();
    if (threadIdx.x == 0) {
      double b = -1.0;
      int rr = c;
      for (int t = 0; t < (int)blockDim.x; ++t)
        if (bv[t] > b) {
          b = bv[t];
          rr = bi[t];
        }
      prow = rr;
      if (!(b > 0.0)) atomicAdd(bad, 1u);
    }
    __syncthreads();
    const int p = prow;
    if (p != c)
      for (int j = threadIdx.x; j < W; j += blockDim.x) {
        const double2 t = A[(size_t)c * W + j];
        A[(size_t)c * W + j] = A[(size_t)p * W + j];
        A[(size_t)p * W + j] = t;
      }
    __syncthreads();
    if (threadIdx.x == 0) {
      const double2 d = A[(size_t)c * W + c];
      const double n = d.x * d.x + d.y * d.y;
      piv = n > 0.0 ? make_double2(d.x / n, -d.y / n) : make_double2(0, 0);
    }
    __syncthreads();
    for (int j = threadIdx.x; j < W; j += blockDim.x) A[(size_t)c * W + j] = cmul(A[(size_t)c * W + j], piv);
    __syncthreads();
    // eliminate column c from every other row with the column's factors staged in LDS
    // (read before any thread changes them); the pivot row is only read
    for (int r = threadIdx.x; r < N; r += blockDim.x) fcol[r] = A[(size_t)r * W + c];
    __syncthreads();
    for (int e = threadIdx.x; e < N * W; e += blockDim.x) {
      const int r = e / W, j = e % W;
      if (r == c) continue;
      const double2 t = cmul(fcol[r], A[(size_t)c * W + j]);
      A[(size_t)r * W + j] = make_double2(A[(size_t)r * W + j].x - t.x, A[(size_t)r * W + j].y - t.y);
    }
  }
  __syncthreads();
  T2* E = Einv + (size_t)(X >> 1) * N * N;
  for (int e = threadIdx.x; e < N * N; e += blockDim.x) {
    const int c = e / N, r = e % N;
    const double2 v = A[(size_t)r * W + N + c];
    E[e] = mk<R>(R(-v.x), R(-v.y));
  }
}

// out = (-A_ee^-1 u_e) on the even coarse sites and out = v on the odd ones (the
// input of the odd Schur complement's second coarse stencil), Einv holding -A^-1.
// The N x N product of each even site is split over kEinvGroups thread groups, each
// summing a quarter of the columns (a row's dependent chain of loads and FMAs is a
// quarter as long), then the groups' partial rows are added in LDS in a fixed order.
constexpr int kEinvGroups = 4;
template <class R>
__global__ __launch_bounds__(128 * kEinvGroups) void einv_apply_k(MGGeom m, const typename C2<R>::T* Einv,
                                                                  const typename C2<R>::T* u,
                                                                  const typename C2<R>::T* v,
                                                                  typename C2<R>::T* out) {
  using T2 = typename C2<R>::T;
  const int X = blockIdx.x;
  const int N = 4 * m.Nv;
  if (coarse_parity(m, X) != 0) {
    for (int r = threadIdx.x; r < N; r += blockDim.x) out[(size_t)X * N + r] = v ? v[(size_t)X * N + r] : mk<R>(R(0), R(0));
    return;
  }
  __shared__ T2 us[128];
  __shared__ R part[kEinvGroups][2][128];
  for (int r = threadIdx.x; r < N; r += blockDim.x) us[r] = u[(size_t)X * N + r];
  __syncthreads();
  const T2* E = Einv + (size_t)(X >> 1) * N * N;
  const int r = threadIdx.x & 127, q = threadIdx.x >> 7;
  const int c0 = q * N / kEinvGroups, c1 = (q + 1) * N / kEinvGroups;
  if (r < N) {
    R ax = 0, ay = 0;
    for (int c = c0; c < c1; ++c) {
      const T2 e = E[(size_t)c * N + r], w = us[c];
      ax += e.x * w.x - e.y * w.y;
      ay += e.x * w.y + e.y * w.x;
    }
    part[q][0][r] = ax;
    part[q][1][r] = ay;
  }
  __syncthreads();
  if (threadIdx.x < N) {
    R sx = 0, sy = 0;
#pragma unroll
    for (int g = 0; g < kEinvGroups; ++g) {
      sx += part[g][0][threadIdx.x];
      sy += part[g][1][threadIdx.x];
    }
    out[(size_t)X * N + threadIdx.x] = mk<R>(sx, sy);
  }
}

// zero the coarse vector on the sites of coarse parity par
template <class R>
__global__ void coarse_zero_parity_k(MGGeom m, typename C2<R>::T* x, int par) {
  const int X = blockIdx.x;
  if (coarse_parity(m, X) != par) return;
  const int N = 4 * m.Nv;
  for (int r = threadIdx.x; r < N; r += blockDim.x) x[(size_t)X * N + r] = mk<R>(R(0), R(0));
}

void mg_einv_build(int prec, const MGGeom& g, int X0, int count, const void* D, const void* Bo, double mubar_c,
                   double epsbar, double m, double2* scratch, void* Einv, unsigned* bad, hipStream_t st) {
  if (prec == P64)
    hipLaunchKernelGGL(einv_build_k<double>, dim3(count), dim3(256), 0, st, g, X0, (const double2*)D,
                       (const double2*)Bo, mubar_c, epsbar, m, scratch, (double2*)Einv, bad);
  else
    hipLaunchKernelGGL(einv_build_k<float>, dim3(count), dim3(256), 0, st, g, X0, (const float2*)D,
                       (const float2*)Bo, mubar_c, epsbar, m, scratch, (float2*)Einv, bad);
}

void mg_einv_apply(int prec, const MGGeom& g, const void* Einv, const void* u, const void* v, void* out,
                   hipStream_t st) {
  if (prec == P64)
    hipLaunchKernelGGL(einv_apply_k<double>, dim3(g.Vc), dim3(128 * kEinvGroups), 0, st, g, (const double2*)Einv, (const double2*)u,
                       (const double2*)v, (double2*)out);
  else
    hipLaunchKernelGGL(einv_apply_k<float>, dim3(g.Vc), dim3(128 * kEinvGroups), 0, st, g, (const float2*)Einv, (const float2*)u,
                       (const float2*)v, (float2*)out);
}

void mg_coarse_zero_parity(int prec, const MGGeom& g, void* x, int par, hipStream_t st) {
  if (prec == P64)
    hipLaunchKernelGGL(coarse_zero_parity_k<double>, dim3(g.Vc), dim3(128), 0, st, g, (double2*)x, par);
  else
    hipLaunchKernelGGL(coarse_zero_parity_k<float>, dim3(g.Vc), dim3(128), 0, st, g, (float2*)x, par);
}

void mg_coarse_apply_multi(const MGGeom& g, const double2* D, const double2* Bo, const double2* x, double2* y, int k,
                           const double* m, double mubar_c, double epsbar, hipStream_t st) {
  MultiM ms;
  for (int r = 0; r < kMultiMax; ++r) ms.m[r] = r < k ? m[r] : 0.0;
  const int tiles = (2 * g.Nv + 15) / 16;
  hipLaunchKernelGGL(coarse_apply_multi_k, dim3(g.Vc), dim3(64 * tiles * kMultiBGroups), 0, st, g, D, Bo, x, y, k, ms,
                     mubar_c, epsbar);
}

void mg_random_fill(const MGGeom& m, int vh, double2* fe, double2* fo, unsigned long long seed, hipStream_t st) {
  hipLaunchKernelGGL(random_fill_k, dim3(nb(48L * vh, 256)), dim3(256), 0, st, vh, m.stride, fe, fo, seed);
}

}  // namespace ndtm
