"""Two-level aggregation multigrid pieces of the oracle (section 3, section 3.2).

Conventions (the GPU library uses the same definitions):

* Aggregates are blocks of ``block = (bt, bz, by, bx)`` fine sites; the coarse
  lattice has dims (T/bt, Lz/bz, Ly/by, Lx/bx) with the same lexicographic
  order as the fine one.
* ``N_v`` single-flavour test vectors v_k (full lattice, 4 spins x 3 colours).
* Chirality split (Gamma5-compatible aggregation, section 3): chirality 0 =
  spins {0,1} (gamma5 = +1), chirality 1 = spins {2,3} (gamma5 = -1).  For each
  aggregate and chirality the N_v restricted vectors are orthonormalised in
  order k = 0..N_v-1 (Gram-Schmidt, i.e. the thin QR with positive real diagonal).
* Coarse dof per flavour: index chi*N_v + k, so a coarse doublet vector is
  (Vc, 2, 2*N_v) = [coarse site][flavour][dof]; Gamma5_c = +1 on chi=0, -1 on chi=1.
* P_ND = P x I_2 (eq:g5-t1-compatible with identical flavour components).
* Coarse doublet operator, eq:non-degenerate_coarse plus the odd-site shift:
  D'_c = D_W,c x I_2 + i mubar Gamma5_c x tau3 - epsbar I x tau1 +- i m C_o x tau1,
  D_W,c = P^dag D_W P and C_o = P^dag (Gamma5 P_odd) P = Gamma5_c P^dag P_odd P.
  With P^dag P = I this is exactly the Galerkin product P_ND^dag D' P_ND.
"""
from __future__ import annotations

import numpy as np

from .lattice import Lattice


def coarse_dims(dims, block):
    for d, b in zip(dims, block):
        if d % b:
            raise ValueError("aggregate size must divide the lattice extent")
    return tuple(d // b for d, b in zip(dims, block))


def aggregate_of_site(dims, block):
    """Coarse-site index of every fine site (lexicographic, x fastest)."""
    T, Z, Y, X = dims
    bt, bz, by, bx = block
    CT, CZ, CY, CX = coarse_dims(dims, block)
    t, z, y, x = np.meshgrid(np.arange(T), np.arange(Z), np.arange(Y), np.arange(X), indexing="ij")
    agg = (((t // bt) * CZ + z // bz) * CY + y // by) * CX + x // bx
    return agg.reshape(-1)


def build_prolongator(test_vectors, dims, block):
    """P as an array (V, 12, 2*N_v): P[x][spin*3+colour][chi*N_v + k].

    test_vectors: (N_v, V, 4, 3) complex.  Per aggregate and chirality, the
    restricted vectors are orthonormalised by classical Gram-Schmidt applied
    twice (numerically the same span and the same unique positive-diagonal
    QR factor as one exact Gram-Schmidt pass).
    """
    tv = np.asarray(test_vectors, dtype=np.complex128)
    Nv, V = tv.shape[0], tv.shape[1]
    agg = aggregate_of_site(dims, block)
    Vc = int(agg.max()) + 1
    P = np.zeros((V, 12, 2 * Nv), dtype=np.complex128)
    for X in range(Vc):
        sites = np.nonzero(agg == X)[0]
        for chi in range(2):
            spins = (0, 1) if chi == 0 else (2, 3)
            M = tv[:, sites][:, :, spins, :].reshape(Nv, -1).T  # (|X|*6, Nv)
            Q = np.zeros_like(M)
            for k in range(Nv):
                v = M[:, k].copy()
                for _ in range(2):
                    for j in range(k):
                        v = v - np.vdot(Q[:, j], v) * Q[:, j]
                nv = np.linalg.norm(v)
                if nv == 0:
                    raise ValueError("test vectors are linearly dependent on an aggregate")
                Q[:, k] = v / nv
            Qs = Q.reshape(len(sites), 2, 3, Nv)
            for si, s in enumerate(spins):
                P[sites, s * 3:(s + 1) * 3, chi * Nv:(chi + 1) * Nv] = Qs[:, si]
    return P


def prolong(P, vc, agg):
    """(P x I_2) vc: fine[x, f, :] = P[x] @ vc[agg(x), f, :]. vc: (Vc, 2, 2Nv) -> (V, 2, 4, 3)."""
    out = np.einsum("xij,xfj->xfi", P, vc[agg])
    return out.reshape(P.shape[0], vc.shape[1], 4, 3)


def restrict(P, v, agg, Vc):
    """(P x I_2)^dag v: vc[X, f, :] = sum_{x in X} P[x]^dag v[x, f, :]. v: (V, nf, 4, 3)."""
    nf = v.shape[1]
    contrib = np.einsum("xij,xfi->xfj", P.conj(), v.reshape(v.shape[0], nf, 12))
    vc = np.zeros((Vc, nf, P.shape[2]), dtype=np.complex128)
    np.add.at(vc, agg, contrib)
    return vc


def coarse_wilson_dense(lat: Lattice, a, P, agg, Vc):
    """Dense D_W,c = P^dag (a - H/2) P by brute force: apply the fine single-flavour
    Wilson operator to every prolonged coarse unit vector and restrict."""
    V = lat.V
    n2 = P.shape[2]
    Dc = np.zeros((Vc * n2, Vc * n2), dtype=np.complex128)
    for X in range(Vc):
        for j in range(n2):
            vc = np.zeros((Vc, 1, n2), dtype=np.complex128)
            vc[X, 0, j] = 1.0
            f = prolong(P, vc, agg)  # (V, 1, 4, 3)
            f4 = f.reshape(lat.dims + (1, 4, 3))
            Df = a * f4 - 0.5 * lat.hop(f4)
            col = restrict(P, Df.reshape(V, 1, 4, 3), agg, Vc)
            Dc[:, X * n2 + j] = col.reshape(-1)
    return Dc


def odd_projector_coarse(lat: Lattice, P, agg, Vc):
    """B_o = P^dag P_odd P, returned per coarse site as (Vc, 2Nv, 2Nv)."""
    odd = lat.parity.reshape(-1) == 1
    B = np.zeros((Vc, P.shape[2], P.shape[2]), dtype=np.complex128)
    for x in np.nonzero(odd)[0]:
        B[agg[x]] += P[x].conj().T @ P[x]
    return B


def gamma5_coarse(Nv):
    return np.concatenate([np.ones(Nv), -np.ones(Nv)])


def coarse_nd_apply(Dc_dense, B_o, vc, Nv, mubar, epsbar, m=0.0, d=1.0):
    """D'_c vc for the coarse doublet (vc: (Vc, 2, 2Nv)).

    D'_c = D_W,c x I_2 + i d mubar Gamma5_c x tau3 - epsbar I x tau1 + i m (Gamma5_c B_o) x tau1.
    """
    Vc = vc.shape[0]
    n2 = 2 * Nv
    g5 = gamma5_coarse(Nv)
    out = np.zeros_like(vc)
    for f in range(2):
        out[:, f, :] = (Dc_dense @ vc[:, f, :].reshape(-1)).reshape(Vc, n2)
    tau3 = np.array([1.0, -1.0])
    out += 1j * d * mubar * (g5[None, None, :] * tau3[None, :, None]) * vc
    swapped = vc[:, ::-1, :]  # tau1 swaps the flavours
    out += -epsbar * swapped
    if m != 0.0:
        Bs = np.einsum("xij,xfj->xfi", B_o, swapped)
        out += 1j * m * g5[None, None, :] * Bs
    return out


def dense_prolongator(P, agg, Vc):
    """Single-flavour P as a dense (V*12, Vc*2Nv) matrix (for brute-force pins)."""
    V, _, n2 = P.shape
    M = np.zeros((V * 12, Vc * n2), dtype=np.complex128)
    for x in range(V):
        M[x * 12:(x + 1) * 12, agg[x] * n2:(agg[x] + 1) * n2] = P[x]
    return M


def coarse_nd_dense(op, P, agg, Vc, m, d=1.0):
    """Dense D'_c(m) over the coarse doublet (index [X][f][dof] flattened): the columns of
    coarse_nd_apply on every coarse unit vector."""
    Nv = P.shape[2] // 2
    Dc = coarse_wilson_dense(op.lat, op.a, P, agg, Vc)
    Bo = odd_projector_coarse(op.lat, P, agg, Vc)
    n = Vc * 2 * 2 * Nv
    A = np.zeros((n, n), dtype=np.complex128)
    for j in range(n):
        e = np.zeros(n, dtype=np.complex128)
        e[j] = 1.0
        A[:, j] = coarse_nd_apply(Dc, Bo, e.reshape(Vc, 2, 2 * Nv), Nv, op.mubar, op.epsbar, m, d).reshape(-1)
    return A


def two_grid_cycle(op, m, r, P, agg, Vc, smoother="mr", steps=0, block=None, mr_iters=1):
    """One two-level cycle for D'(m) z = r (section 3, eq:error_propagation with no
    pre-smoothing): the coarse correction z0 = (P x I2) D'_c(m)^-1 (P x I2)^dag r with the
    coarse system solved exactly (dense), then `steps` post-smoothing iterations from z0:
    minimal-residual steps (smoother "mr") or SAP sweeps (smoother "sap", blocks `block`,
    `mr_iters` steps per block solve).  r: full-lattice doublet of shape dims + (2, 4, 3)."""
    from . import smoothers

    dims = op.lat.dims
    V = op.lat.V
    Nv = P.shape[2] // 2
    A = coarse_nd_dense(op, P, agg, Vc, m)
    rc = restrict(P, r.reshape(V, 2, 4, 3), agg, Vc)
    xc = np.linalg.solve(A, rc.reshape(-1)).reshape(Vc, 2, 2 * Nv)
    z = prolong(P, xc, agg).reshape(dims + (2, 4, 3))
    if smoother == "sap":
        return smoothers.sap_smooth_colour(op, m, r, z, block, steps, mr_iters)
    return smoothers.mr_smooth(op, m, r, z, steps)
