// Clover term of eq:Wilson on the GPU: the site blocks of the even-odd operator.
//
// The clover term -c_sw/32 sum_{mu,nu} gamma_mu gamma_nu x (Q_mu_nu - Q_nu_mu) is
// block diagonal in chirality (gamma_mu gamma_nu commutes with gamma5), so each site
// carries two 6x6 Hermitian blocks over (spin pair, colour).  With
// F_mu_nu = Q_mu_nu - Q_mu_nu^+ (the reversed clover leaf is the adjoint) and the
// chiral basis, gamma_0 gamma_k = diag(-i s_k, i s_k) and gamma_j gamma_k =
// diag(i e_jkl s_l, i e_jkl s_l), the block of chirality chi (upper sign for the
// spins 0, 1) is
//   C_chi = -c_sw/16 sum_l s_l x G_l,   G_l = i (-+ F_0l + E_l),
//   E_1 = F_yz, E_2 = -F_xz, E_3 = F_xy,
// i.e. [[G_3, G_1 - i G_2], [G_1 + i G_2, -G_3]] in 3x3 colour blocks.
//
// Stored per site and chirality, packed Hermitian (6 real diagonal entries, then
// the 15 upper entries row by row as (re, im)): M = a + C on both parities, and
// on the even sites N = (M^2 + mubar^2 - epsbar^2)^-1 and M N.  The site block of
// the doublet is A = M x 1 + i mubar gamma5 tau3 - epsbar tau1; in each chirality
// its flavour blocks are functions of M and commute, so
//   A^-1 = [[M - i mubar g5, epsbar], [epsbar, M + i mubar g5]] N,
// which the stencil's epilogue applies as M N v_f - i mubar g5 tau3 N v_f + epsbar N v_{1-f}.
#include "ndtm_internal.h"

namespace ndtm {
namespace {

struct c3 {
  double2 m[3][3];
};

__device__ __forceinline__ double2 cm(double2 a, double2 b) { return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
__device__ __forceinline__ double2 ca(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }

__device__ c3 mul(const c3& A, const c3& B) {
  c3 C;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      double2 s = make_double2(0, 0);
#pragma unroll
      for (int k = 0; k < 3; ++k) s = ca(s, cm(A.m[i][k], B.m[k][j]));
      C.m[i][j] = s;
    }
  return C;
}

__device__ c3 dag(const c3& A) {
  c3 C;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) C.m[i][j] = make_double2(A.m[j][i].x, -A.m[j][i].y);
  return C;
}

struct Coord {
  int c[4];  // indexed by direction: t, x, y, z
};

__device__ c3 link(const Geom& g, const double2* Ue, const double2* Uo, Coord x, int mu) {
  const int t = x.c[0], xx = x.c[1], y = x.c[2], z = x.c[3];
  const int par = (t + xx + y + z) & 1;
  const long h = (((long)t * g.Lz + z) * g.Ly + y) * (g.Lx >> 1) + (xx >> 1);
  const double2* U = par ? Uo : Ue;
  c3 M;
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) M.m[r][c] = U[(long)(mu * 9 + r * 3 + c) * g.stride + h];
  return M;
}

__device__ Coord step(const Geom& g, Coord x, int mu, int d) {
  const int ext[4] = {g.T, g.Lx, g.Ly, g.Lz};
  x.c[mu] = (x.c[mu] + d + ext[mu]) % ext[mu];
  return x;
}

// Q_mu_nu(x): the four plaquettes of the mu-nu plane at x (clover leaf)
__device__ c3 leaf_sum(const Geom& g, const double2* Ue, const double2* Uo, Coord x, int mu, int nu) {
  const Coord xm = step(g, x, mu, 1), xn = step(g, x, nu, 1);
  const Coord xmm = step(g, x, mu, -1), xnm = step(g, x, nu, -1);
  const Coord xnm_mm = step(g, xn, mu, -1);    // x + nu - mu
  const Coord xmm_nm = step(g, xmm, nu, -1);   // x - mu - nu
  const Coord xnm_mp = step(g, xnm, mu, 1);    // x - nu + mu
  c3 Q = mul(mul(link(g, Ue, Uo, x, mu), link(g, Ue, Uo, xm, nu)),
             mul(dag(link(g, Ue, Uo, xn, mu)), dag(link(g, Ue, Uo, x, nu))));
  const c3 l2 = mul(mul(link(g, Ue, Uo, x, nu), dag(link(g, Ue, Uo, xnm_mm, mu))),
                    mul(dag(link(g, Ue, Uo, xmm, nu)), link(g, Ue, Uo, xmm, mu)));
  const c3 l3 = mul(mul(dag(link(g, Ue, Uo, xmm, mu)), dag(link(g, Ue, Uo, xmm_nm, nu))),
                    mul(link(g, Ue, Uo, xmm_nm, mu), link(g, Ue, Uo, xnm, nu)));
  const c3 l4 = mul(mul(dag(link(g, Ue, Uo, xnm, nu)), link(g, Ue, Uo, xnm, mu)),
                    mul(link(g, Ue, Uo, xnm_mp, nu), dag(link(g, Ue, Uo, x, mu))));
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) Q.m[i][j] = ca(ca(Q.m[i][j], l2.m[i][j]), ca(l3.m[i][j], l4.m[i][j]));
  return Q;
}

// index of the upper entry (i < j) in the packed Hermitian 6x6 layout
__device__ __forceinline__ int up_index(int i, int j) { return 6 + 2 * (i * 6 - i * (i + 1) / 2 + (j - i - 1)); }

__device__ void store_packed(double* dst, long stride, long h, const double2 (&H)[6][6]) {
#pragma unroll
  for (int i = 0; i < 6; ++i) dst[(long)i * stride + h] = H[i][i].x;
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int j = i + 1; j < 6; ++j) {
      const int k = up_index(i, j);
      dst[(long)k * stride + h] = H[i][j].x;
      dst[(long)(k + 1) * stride + h] = H[i][j].y;
    }
}

// Gauss-Jordan inverse of a complex 6x6 with partial pivoting; returns false if singular
__device__ bool inverse6(double2 (&A)[6][6], double2 (&B)[6][6]) {
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int j = 0; j < 6; ++j) B[i][j] = make_double2(i == j ? 1.0 : 0.0, 0.0);
  for (int c = 0; c < 6; ++c) {
    int p = c;
    double best = A[c][c].x * A[c][c].x + A[c][c].y * A[c][c].y;
    for (int r = c + 1; r < 6; ++r) {
      const double v = A[r][c].x * A[r][c].x + A[r][c].y * A[r][c].y;
      if (v > best) {
        best = v;
        p = r;
      }
    }
    if (!(best > 0.0)) return false;
    if (p != c)
      for (int j = 0; j < 6; ++j) {
        const double2 t = A[c][j];
        A[c][j] = A[p][j];
        A[p][j] = t;
        const double2 u = B[c][j];
        B[c][j] = B[p][j];
        B[p][j] = u;
      }
    const double2 d = A[c][c];
    const double inv_n = 1.0 / (d.x * d.x + d.y * d.y);
    const double2 id = make_double2(d.x * inv_n, -d.y * inv_n);
    for (int j = 0; j < 6; ++j) {
      A[c][j] = cm(A[c][j], id);
      B[c][j] = cm(B[c][j], id);
    }
    for (int r = 0; r < 6; ++r) {
      if (r == c) continue;
      const double2 f = A[r][c];
      for (int j = 0; j < 6; ++j) {
        const double2 a = cm(f, A[c][j]), b = cm(f, B[c][j]);
        A[r][j] = make_double2(A[r][j].x - a.x, A[r][j].y - a.y);
        B[r][j] = make_double2(B[r][j].x - b.x, B[r][j].y - b.y);
      }
    }
  }
  return true;
}

// One thread per (site, chirality) of one parity: M = a + C_chi, and on the even
// parity N and M N.  *bad counts sites whose block could not be inverted.
__global__ __launch_bounds__(64) void clover_build_k(Geom g, const double2* Ue, const double2* Uo, int parity, double a, double csw,
                               double shift2, double* Mout, double* Ninv, unsigned* bad) {
  const long tid = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (tid >= 2L * g.vh) return;
  const int chi = (int)(tid & 1);
  const long h = tid >> 1;
  const int Lxh = g.Lx >> 1;
  const long row = h / Lxh;
  const int xh = (int)(h - row * Lxh);
  const int y = (int)(row % g.Ly);
  const long tz = row / g.Ly;
  const int z = (int)(tz % g.Lz), t = (int)(tz / g.Lz);
  const int x = 2 * xh + ((parity + t + z + y) & 1);
  Coord s;
  s.c[0] = t;
  s.c[1] = x;
  s.c[2] = y;
  s.c[3] = z;
  // F_mu_nu = Q_mu_nu - Q_mu_nu^+ for the six planes mu < nu
  c3 F[4][4];
  for (int mu = 0; mu < 4; ++mu)
    for (int nu = mu + 1; nu < 4; ++nu) {
      const c3 Q = leaf_sum(g, Ue, Uo, s, mu, nu);
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
          F[mu][nu].m[i][j] = make_double2(Q.m[i][j].x - Q.m[j][i].x, Q.m[i][j].y + Q.m[j][i].y);
    }
  // G_l = i (sgn F_0l + E_l), sgn = -1 for chirality 0, +1 for chirality 1
  const double sg = chi == 0 ? -1.0 : 1.0;
  c3 G[3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const double2 e1 = F[2][3].m[i][j], e2 = make_double2(-F[1][3].m[i][j].x, -F[1][3].m[i][j].y),
                    e3 = F[1][2].m[i][j];
      const double2 e[3] = {e1, e2, e3};
#pragma unroll
      for (int l = 0; l < 3; ++l) {
        const double2 v = make_double2(sg * F[0][l + 1].m[i][j].x + e[l].x, sg * F[0][l + 1].m[i][j].y + e[l].y);
        G[l].m[i][j] = make_double2(-v.y, v.x);  // i v
      }
    }
  const double cf = -csw / 16.0;
  double2 M[6][6];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const double2 g1 = G[0].m[i][j], g2 = G[1].m[i][j], g3 = G[2].m[i][j];
      M[i][j] = make_double2(cf * g3.x, cf * g3.y);
      M[3 + i][3 + j] = make_double2(-cf * g3.x, -cf * g3.y);
      M[i][3 + j] = make_double2(cf * (g1.x + g2.y), cf * (g1.y - g2.x));   // G1 - i G2
      M[3 + i][j] = make_double2(cf * (g1.x - g2.y), cf * (g1.y + g2.x));   // G1 + i G2
    }
#pragma unroll
  for (int i = 0; i < 6; ++i) M[i][i].x += a;
  store_packed(Mout + (long)chi * 36 * g.stride, g.stride, h, M);
  if (!Ninv) return;
  double2 K[6][6], Nm[6][6], MN[6][6];
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      double2 v = make_double2(i == j ? shift2 : 0.0, 0.0);
#pragma unroll
      for (int k = 0; k < 6; ++k) v = ca(v, cm(M[i][k], M[k][j]));
      K[i][j] = v;
    }
  if (!inverse6(K, Nm)) {
    atomicAdd(bad, 1u);
    return;
  }
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      double2 v = make_double2(0, 0);
#pragma unroll
      for (int k = 0; k < 6; ++k) v = ca(v, cm(M[i][k], Nm[k][j]));
      MN[i][j] = v;
    }
  store_packed(Ninv + (long)chi * 36 * g.stride, g.stride, h, Nm);
  store_packed(Ninv + (long)(72 + chi * 36) * g.stride, g.stride, h, MN);
}

__global__ void to_f32_k(const double* src, float* dst, long n) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    dst[i] = (float)src[i];
}

}  // namespace

// Builds the clover site blocks of one parity from the FP64 links (both parity
// arrays).  Mout: 72 x stride doubles; Ninv (even parity only, else null):
// 144 x stride doubles.  bad: device counter of singular blocks (cleared here).
void launch_clover_build(const Geom& g, const double2* Ue, const double2* Uo, int parity, double a, double csw,
                         double mubar, double epsbar, double* Mout, double* Ninv, unsigned* bad, hipStream_t st) {
  (void)hipMemsetAsync(bad, 0, sizeof(unsigned), st);
  const long n = 2L * g.vh;
  hipLaunchKernelGGL(clover_build_k, dim3((unsigned)((n + 63) / 64)), dim3(64), 0, st, g, Ue, Uo, parity, a, csw,
                     mubar * mubar - epsbar * epsbar, Mout, Ninv, bad);
}

void launch_to_f32(const double* src, float* dst, long n, hipStream_t st) {
  hipLaunchKernelGGL(to_f32_k, dim3(1024), dim3(256), 0, st, src, dst, n);
}

}  // namespace ndtm
