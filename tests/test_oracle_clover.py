"""Pins of the oracle's clover term (eq:Wilson with c_sw != 0).

* U = 1: every leaf is the identity, Q_mu_nu = Q_nu_mu = 4, so C = 0;
* Q_nu_mu = Q_mu_nu^+ (reversed plaquettes), C Hermitian and block diagonal in
  chirality (it commutes with gamma5), so D_ND keeps its (Gamma5 x tau1)-hermiticity;
* abelian closed form: for links U_mu(x) = exp(i phi_mu(x)) I the leaves are phases
  of the lattice curl theta_mu_nu = phi_mu(x) + phi_nu(x+mu) - phi_mu(x+nu) - phi_nu(x),
  and Q_mu_nu - Q_nu_mu = 2i (sin theta(x) + sin theta(x-mu) + sin theta(x-mu-nu) + sin theta(x-nu));
* gauge covariance: C(x) -> (1 x Omega(x)) C(x) (1 x Omega(x)^+);
* the vectorised operator with the clover term equals the loop-by-loop dense assembly
  on 2^4 and on a mixed-extent lattice, the even-odd Schur identity holds with the
  numerically inverted site blocks, and Q = Gamma5 tau1 S stays Hermitian.
"""
import numpy as np
import pytest

import synth
from oracle import clover, dense
from oracle.lattice import GAMMA5, MU_AXIS, Lattice, NDOperator

K, MB, EB = synth.KAPPA, synth.MUBAR, synth.EPSBAR
CSW = 1.76


def _U(dims, seed=11):
    return synth.gauge_field(dims, seed, 0.3).reshape(tuple(dims) + (4, 3, 3))


def test_unit_links_give_zero():
    dims = (4, 4, 2, 2)
    U = synth.unit_gauge(dims).reshape(dims + (4, 3, 3))
    assert np.abs(clover.clover_term(U, CSW)).max() == 0.0
    for mu in range(4):
        for nu in range(4):
            if mu != nu:
                assert np.allclose(clover.clover_leaf_sum(U, mu, nu), 4 * np.eye(3))


def test_reversed_leaves_hermitian_and_chirality_blocks():
    dims = (4, 2, 4, 2)
    U = _U(dims)
    for mu in range(4):
        for nu in range(mu + 1, 4):
            Q = clover.clover_leaf_sum(U, mu, nu)
            R = clover.clover_leaf_sum(U, nu, mu)
            assert np.abs(R - np.conj(np.swapaxes(Q, -1, -2))).max() < 1e-14
    C = clover.clover_term(U, CSW)
    assert np.abs(C - np.conj(np.swapaxes(C, -1, -2))).max() < 1e-14
    g5 = np.kron(GAMMA5, np.eye(3))
    assert np.abs(np.einsum("ij,...jk->...ik", g5, C) - np.einsum("...ij,jk->...ik", C, g5)).max() < 1e-14
    assert np.abs(C).max() > 0.05  # not trivially zero


def test_abelian_closed_form():
    dims = (4, 4, 2, 6)
    rng = np.random.default_rng(5)
    phi = rng.uniform(-0.7, 0.7, dims + (4,))
    U = np.exp(1j * phi)[..., None, None] * np.eye(3)
    C = clover.clover_term(U, CSW)
    want = np.zeros(dims + (4, 4), dtype=complex)
    from oracle.lattice import GAMMA
    sh = lambda f, mu, d: np.roll(f, -d, axis=MU_AXIS[mu])
    for mu in range(4):
        for nu in range(4):
            if mu == nu:
                continue
            th = phi[..., mu] + sh(phi[..., nu], mu, 1) - sh(phi[..., mu], nu, 1) - phi[..., nu]
            s = np.sin(th) + sh(np.sin(th), mu, -1) + sh(sh(np.sin(th), mu, -1), nu, -1) + sh(np.sin(th), nu, -1)
            want += np.einsum("st,...->...st", GAMMA[mu] @ GAMMA[nu], 2j * s)
    want = -CSW / 32.0 * want
    got = C.reshape(dims + (4, 3, 4, 3))
    assert np.abs(got[..., :, 0, :, 0] - want).max() < 1e-14
    assert np.abs(got[..., :, 0, :, 1]).max() < 1e-14  # colour-diagonal


def test_gauge_covariance():
    dims = (4, 2, 2, 4)
    U = _U(dims, 3)
    V = int(np.prod(dims))
    Om = synth.random_su3(V, 9).reshape(dims + (3, 3))
    Ug = np.empty_like(U)
    for mu in range(4):
        Ug[..., mu, :, :] = Om @ U[..., mu, :, :] @ np.conj(np.swapaxes(np.roll(Om, -1, axis=MU_AXIS[mu]), -1, -2))
    C = clover.clover_term(U, CSW)
    Cg = clover.clover_term(Ug, CSW)
    W = np.einsum("st,...ab->...satb", np.eye(4), Om).reshape(dims + (12, 12))
    want = W @ C @ np.conj(np.swapaxes(W, -1, -2))
    assert np.abs(Cg - want).max() < 1e-13


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (4, 2, 2, 2)])
def test_dense_bruteforce_with_clover(dims):
    U = synth.gauge_field(dims, 13, 0.3)
    lat = Lattice(dims, U)
    op = NDOperator(lat, K, MB, EB, csw=CSW)
    D = dense.dense_D_ND(dims, U, K, MB, EB, csw=CSW)
    v = synth.gaussian_spinor(dims, 4, "full")
    got = op.D_full(v.reshape(dims + (2, 4, 3))).reshape(-1)
    assert np.abs(got - D @ v.reshape(-1)).max() < 1e-13
    # even-odd: [D^-1]_oo = S^-1 with the numerically inverted even site blocks
    e, o = dense.parity_indices(dims)
    n = len(o)
    S = np.zeros((n, n), dtype=complex)
    Q = np.zeros((n, n), dtype=complex)
    for j in range(n):
        ej = np.zeros(n, dtype=complex)
        ej[j] = 1
        S[:, j] = op.S_hat(ej.reshape(-1, 2, 4, 3)).reshape(-1)
        Q[:, j] = op.Q_hat(ej.reshape(-1, 2, 4, 3)).reshape(-1)
    assert np.abs(np.linalg.inv(S) - np.linalg.inv(D)[np.ix_(o, o)]).max() < 1e-11
    assert np.abs(S - dense.dense_schur_odd(D, dims)).max() < 1e-12
    # (Gamma5 x tau1)-hermiticity survives the clover term: Q is Hermitian
    assert np.abs(Q - Q.conj().T).max() < 1e-12
