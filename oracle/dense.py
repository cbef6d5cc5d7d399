"""Brute-force dense matrices, assembled site by site with explicit loops.

Only for tiny lattices (2^4, 4^4).  This is a second, independent spelling of
eq:Wilson / eq:non-degenerate: it walks the neighbour list of every site and
writes the 12x12 (per flavour) hopping blocks into a dense matrix, without the
vectorised shifts of ``lattice``.  Vector index: ((s*2 + f)*4 + spin)*3 + colour,
s the lexicographic site index.
"""
from __future__ import annotations

import numpy as np

from .lattice import GAMMA, GAMMA5, TAU1, TAU3


def _coords(s, dims):
    T, Z, Y, X = dims
    x = s % X
    y = (s // X) % Y
    z = (s // (X * Y)) % Z
    t = s // (X * Y * Z)
    return [t, x, y, z]  # indexed by direction mu


def _site(c, dims):
    T, Z, Y, X = dims
    t, x, y, z = c
    return ((t * Z + z) * Y + y) * X + x


def _ext(dims):
    T, Z, Y, X = dims
    return [T, X, Y, Z]  # extent along direction mu


def _link(U, dims, c, mu):
    return U[_site(c, dims), mu]


def _step(c, mu, d, dims):
    e = list(c)
    ext = _ext(dims)
    e[mu] = (c[mu] + d) % ext[mu]
    return e


def dense_clover_site(U, dims, s, csw):
    """The clover term of eq:Wilson at site s, 12x12 over (spin, colour), walked out
    leaf by leaf with explicit coordinate steps (a second spelling of oracle.clover)."""
    c = _coords(s, dims)
    C = np.zeros((12, 12), dtype=np.complex128)
    dag = lambda m: m.conj().T
    for mu in range(4):
        for nu in range(4):
            if mu == nu:
                continue
            Q = {}
            for a, b in ((mu, nu), (nu, mu)):
                xa = _step(c, a, 1, dims)
                xb = _step(c, b, 1, dims)
                xab = _step(xb, a, -1, dims)      # x + b - a
                xma = _step(c, a, -1, dims)        # x - a
                xmab = _step(xma, b, -1, dims)     # x - a - b
                xmb = _step(c, b, -1, dims)        # x - b
                xmba = _step(xmb, a, 1, dims)      # x - b + a
                L = lambda cc, d: _link(U, dims, cc, d)
                Q[(a, b)] = (L(c, a) @ L(xa, b) @ dag(L(xb, a)) @ dag(L(c, b))
                             + L(c, b) @ dag(L(xab, a)) @ dag(L(xma, b)) @ L(xma, a)
                             + dag(L(xma, a)) @ dag(L(xmab, b)) @ L(xmab, a) @ L(xmb, b)
                             + dag(L(xmb, b)) @ L(xmb, a) @ L(xmba, b) @ dag(L(c, a)))
            C += np.kron(GAMMA[mu] @ GAMMA[nu], Q[(mu, nu)] - Q[(nu, mu)])
    return -csw / 32.0 * C


def dense_D_ND(dims, U, kappa, mubar, epsbar, antiperiodic_t=False, odd_shift=0.0, csw=0.0):
    """Dense D_ND (optionally + i*odd_shift*(Gamma5 x tau1) on odd sites, and with the
    clover term of eq:Wilson for csw != 0) on the full lattice."""
    V = int(np.prod(dims))
    U = np.asarray(U).reshape(V, 4, 3, 3)
    n = V * 24
    D = np.zeros((n, n), dtype=np.complex128)
    a = 1.0 / (2.0 * kappa)
    ext = _ext(dims)
    site_blk = (a * np.eye(8) + 1j * mubar * np.kron(TAU3, GAMMA5) - epsbar * np.kron(TAU1, np.eye(4)))
    g5t1 = np.kron(TAU1, GAMMA5)
    for s in range(V):
        c = _coords(s, dims)
        par = sum(c) % 2
        blk = site_blk + (1j * odd_shift * g5t1 if par == 1 else 0)
        D[s * 24:(s + 1) * 24, s * 24:(s + 1) * 24] += np.kron(blk, np.eye(3))
        if csw != 0.0:
            Cs = dense_clover_site(U, dims, s, csw)
            for f in range(2):
                D[s * 24 + f * 12:s * 24 + f * 12 + 12, s * 24 + f * 12:s * 24 + f * 12 + 12] += Cs
        for mu in range(4):
            # forward neighbour
            cf = list(c)
            cf[mu] = (c[mu] + 1) % ext[mu]
            sign_f = -1.0 if (antiperiodic_t and mu == 0 and c[0] == ext[0] - 1) else 1.0
            sf = _site(cf, dims)
            hop_f = np.kron(np.eye(4) - GAMMA[mu], U[s, mu])  # (spin x colour)
            cb = list(c)
            cb[mu] = (c[mu] - 1) % ext[mu]
            sign_b = -1.0 if (antiperiodic_t and mu == 0 and c[0] == 0) else 1.0
            sb = _site(cb, dims)
            hop_b = np.kron(np.eye(4) + GAMMA[mu], U[sb, mu].conj().T)
            for f in range(2):
                r0 = s * 24 + f * 12
                D[r0:r0 + 12, sf * 24 + f * 12: sf * 24 + f * 12 + 12] += -0.5 * sign_f * hop_f
                D[r0:r0 + 12, sb * 24 + f * 12: sb * 24 + f * 12 + 12] += -0.5 * sign_b * hop_b
    return D


def parity_indices(dims):
    """Dense-vector indices of even and odd sites (each site has 24 entries)."""
    V = int(np.prod(dims))
    par = np.array([sum(_coords(s, dims)) % 2 for s in range(V)])
    even = np.concatenate([np.arange(s * 24, s * 24 + 24) for s in range(V) if par[s] == 0])
    odd = np.concatenate([np.arange(s * 24, s * 24 + 24) for s in range(V) if par[s] == 1])
    return even, odd


def dense_schur_odd(D, dims):
    """S = D_oo - D_oe D_ee^-1 D_eo by dense inversion (independent of the closed-form A^-1)."""
    e, o = parity_indices(dims)
    Dee = D[np.ix_(e, e)]
    Deo = D[np.ix_(e, o)]
    Doe = D[np.ix_(o, e)]
    Doo = D[np.ix_(o, o)]
    return Doo - Doe @ np.linalg.solve(Dee, Deo)


def dense_g5t1(n_sites):
    """Gamma5 x tau1 on n_sites sites in the dense ordering."""
    return np.kron(np.eye(n_sites), np.kron(np.kron(TAU1, GAMMA5), np.eye(3)))


def odd_vec_to_dense(v_odd):
    """(V/2, 2, 4, 3) odd-site vector -> dense odd-index ordering (sites ascending)."""
    return np.asarray(v_odd).reshape(-1)


def dense_to_odd_vec(d):
    return np.asarray(d).reshape(-1, 2, 4, 3)
