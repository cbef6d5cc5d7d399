"""Clover term of eq:Wilson (the oracle's FP64 reference; test infrastructure).

eq:Wilson adds to the site term (m + 4) the clover term

    C(x) = - c_sw / 32  sum_{mu, nu = 0..3}  (gamma_mu gamma_nu) x (Q_mu_nu(x) - Q_nu_mu(x)),

a 12 x 12 matrix per site over (spin, colour).  The paper refers the definition of
Q_mu_nu to the literature; the reading taken here is the usual clover leaf: the
sum of the four plaquettes of the mu-nu plane that start and end at x, each
traversed first along +mu or, rotating, along +nu, -mu, -nu:

    Q_mu_nu(x) = U_mu(x) U_nu(x+mu) U_mu(x+nu)^+ U_nu(x)^+
               + U_nu(x) U_mu(x+nu-mu)^+ U_nu(x-mu)^+ U_mu(x-mu)
               + U_mu(x-mu)^+ U_nu(x-mu-nu)^+ U_mu(x-mu-nu) U_nu(x-nu)
               + U_nu(x-nu)^+ U_mu(x-nu) U_nu(x-nu+mu) U_mu(x)^+ .

Links are periodic (the antiperiodic option concerns the fermion field only).
Q_nu_mu is the same sum with the roles of mu and nu exchanged, computed as such
(the tests pin Q_nu_mu = Q_mu_nu^+).  Plain NumPy, no blocking: every leaf is
written out as four matrix products on link fields shifted by np.roll.
"""
from __future__ import annotations

import numpy as np

from .lattice import GAMMA, MU_AXIS


def _shift(f, mu, step):
    """f(x + step * mu_hat) for a field over the lattice axes (periodic)."""
    return np.roll(f, -step, axis=MU_AXIS[mu])


def _dag(m):
    return np.conj(np.swapaxes(m, -1, -2))


def clover_leaf_sum(U, mu, nu):
    """Q_mu_nu(x) for every site; U has shape dims + (4, 3, 3); returns dims + (3, 3)."""
    Um, Un = U[..., mu, :, :], U[..., nu, :, :]

    def at(f, dmu, dnu):
        g = _shift(f, mu, dmu) if dmu else f
        return _shift(g, nu, dnu) if dnu else g

    leaf1 = Um @ at(Un, 1, 0) @ _dag(at(Um, 0, 1)) @ _dag(Un)
    leaf2 = Un @ _dag(at(Um, -1, 1)) @ _dag(at(Un, -1, 0)) @ at(Um, -1, 0)
    leaf3 = _dag(at(Um, -1, 0)) @ _dag(at(Un, -1, -1)) @ at(Um, -1, -1) @ at(Un, 0, -1)
    leaf4 = _dag(at(Un, 0, -1)) @ at(Um, 0, -1) @ at(Un, 1, -1) @ _dag(Um)
    return leaf1 + leaf2 + leaf3 + leaf4


def clover_term(U, csw):
    """C(x) = -c_sw/32 sum_{mu,nu} (gamma_mu gamma_nu) x (Q_mu_nu - Q_nu_mu): dims + (12, 12),
    index spin * 3 + colour."""
    sh = U.shape[:-3]
    C = np.zeros(sh + (12, 12), dtype=np.complex128)
    for mu in range(4):
        for nu in range(4):
            if mu == nu:
                continue
            F = clover_leaf_sum(U, mu, nu) - clover_leaf_sum(U, nu, mu)
            g = GAMMA[mu] @ GAMMA[nu]
            C += np.einsum("st,...ab->...satb", g, F).reshape(sh + (12, 12))
    return -csw / 32.0 * C


def apply_clover(C, psi):
    """C acting on each flavour of psi (dims + (nf, 4, 3))."""
    sh = psi.shape
    v = psi.reshape(sh[:-3] + (sh[-3], 12))
    return np.einsum("...ij,...fj->...fi", C, v).reshape(sh)
