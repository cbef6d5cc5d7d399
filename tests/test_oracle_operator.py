"""Pins of the oracle's operators against mathematics fixed by the paper.

Pins: gamma algebra and gamma5 = diag(1,1,-1,-1) (section 2); the closed-form
site inverse; free-field plane waves (eq:Wilson at U = 1); an independent
site-by-site dense assembly on 2^4 (neighbours alias, so both hops must add);
(Gamma5 x tau1)-hermiticity (eq:g5tau1-hermiticity); gauge covariance; the
epsbar = 0 and mubar = 0 special cases (eq:non-degenerate, section 3.2.1);
the Schur identity [D^-1]_oo = S^-1 (even-odd reduction), also for the
shifted operator D' = D_ND + i m (Gamma5 x tau1) P_odd, whose odd Schur
complement is S + i m Gamma5 tau1 (the multigrid's reading of the shifted
odd system, section 3.1 with eq:g5tau1-hermiticity).
"""
import itertools

import numpy as np
import pytest

import synth
from oracle import dense
from oracle.lattice import GAMMA, GAMMA5, MU_AXIS, TAU1, TAU3, Lattice, NDOperator, norm2

K, MB, EB = synth.KAPPA, synth.MUBAR, synth.EPSBAR


def _op(dims, seed=11, amp=0.3, antiperiodic=False, mubar=MB, epsbar=EB):
    U = synth.gauge_field(dims, seed, amp)
    lat = Lattice(dims, U, antiperiodic_t=antiperiodic)
    return lat, NDOperator(lat, K, mubar, epsbar), U


def test_gamma_algebra():
    for a in range(4):
        assert np.allclose(GAMMA[a], GAMMA[a].conj().T)
        for b in range(4):
            ac = GAMMA[a] @ GAMMA[b] + GAMMA[b] @ GAMMA[a]
            assert np.allclose(ac, 2 * np.eye(4) * (a == b))
    assert np.allclose(GAMMA5, np.diag([1, 1, -1, -1]))


def test_site_inverse_closed_form():
    lat, op, _ = _op((2, 2, 2, 2))
    assert np.allclose(op.A_block @ op.Ainv_block, np.eye(8), atol=1e-15)
    assert np.allclose(np.linalg.inv(op.A_block), op.Ainv_block, atol=1e-15)


@pytest.mark.parametrize("antiperiodic", [False, True])
def test_free_field_plane_wave(antiperiodic):
    """U = 1: D_ND e^{ipx} u = e^{ipx} [ (m + sum(1-cos p) + i sum gamma sin p) x I2
    + i mubar g5 tau3 - epsbar tau1 ] u with m = a - 4."""
    dims = (4, 4, 2, 6)
    lat = Lattice(dims, synth.unit_gauge(dims), antiperiodic_t=antiperiodic)
    op = NDOperator(lat, K, MB, EB)
    ext = [dims[0], dims[3], dims[2], dims[1]]
    rng = np.random.default_rng(3)
    coords = np.meshgrid(*[np.arange(d) for d in dims], indexing="ij")
    xmu = [coords[MU_AXIS[mu]] for mu in range(4)]
    for _ in range(4):
        n = [rng.integers(0, e) for e in ext]
        p = [2 * np.pi * n[mu] / ext[mu] for mu in range(4)]
        if antiperiodic:
            p[0] = (2 * n[0] + 1) * np.pi / ext[0]
        u = rng.standard_normal((2, 4, 3)) + 1j * rng.standard_normal((2, 4, 3))
        phase = np.exp(1j * sum(p[mu] * xmu[mu] for mu in range(4)))
        psi = phase[..., None, None, None] * u
        m = op.a - 4.0
        Dw = (m + sum(1 - np.cos(p[mu]) for mu in range(4))) * np.eye(4) + 1j * sum(
            np.sin(p[mu]) * GAMMA[mu] for mu in range(4))
        Dp = np.kron(np.eye(2), Dw) + 1j * MB * np.kron(TAU3, GAMMA5) - EB * np.kron(TAU1, np.eye(4))
        want = phase[..., None, None, None] * (Dp @ u.reshape(8, 3)).reshape(2, 4, 3)
        got = op.D_full(psi)
        assert np.abs(got - want).max() < 1e-12


def test_free_field_even_odd_plane_wave():
    """Odd-site plane wave: S e^{ipx}u = e^{ipx}(A - h(p) A^-1 h(p)/4) u, h(p) = 2 sum cos p - 2i sum gamma sin p."""
    dims = (4, 4, 4, 4)
    lat = Lattice(dims, synth.unit_gauge(dims))
    op = NDOperator(lat, K, MB, EB)
    rng = np.random.default_rng(5)
    coords = np.meshgrid(*[np.arange(d) for d in dims], indexing="ij")
    xmu = [coords[MU_AXIS[mu]] for mu in range(4)]
    for _ in range(3):
        p = [2 * np.pi * rng.integers(0, 4) / 4 for _ in range(4)]
        u = rng.standard_normal((2, 4, 3)) + 1j * rng.standard_normal((2, 4, 3))
        phase = np.exp(1j * sum(p[mu] * xmu[mu] for mu in range(4)))
        psi = lat.take_odd(phase[..., None, None, None] * u)
        h = 2 * sum(np.cos(p)) * np.eye(4) - 2j * sum(np.sin(p[mu]) * GAMMA[mu] for mu in range(4))
        H8 = np.kron(np.eye(2), h)
        S = op.A_block - 0.25 * H8 @ op.Ainv_block @ H8
        Qp = np.kron(TAU1, GAMMA5) @ S
        want = lat.take_odd(phase[..., None, None, None] * (Qp @ u.reshape(8, 3)).reshape(2, 4, 3))
        got = op.Q_hat(psi)
        assert np.abs(got - want).max() < 1e-12


@pytest.mark.parametrize("antiperiodic", [False, True])
def test_dense_bruteforce_2x2x2x2(antiperiodic):
    dims = (2, 2, 2, 2)
    lat, op, U = _op(dims, antiperiodic=antiperiodic)
    D = dense.dense_D_ND(dims, U, K, MB, EB, antiperiodic_t=antiperiodic, odd_shift=0.37)
    v = synth.gaussian_spinor(dims, 7, "full")
    got = op.D_full(v.reshape(dims + (2, 4, 3)), odd_shift=0.37).reshape(-1)
    assert np.abs(got - D @ v.reshape(-1)).max() < 1e-13


def test_dense_bruteforce_mixed_extents():
    dims = (4, 2, 2, 6)
    lat, op, U = _op(dims, seed=4)
    D = dense.dense_D_ND(dims, U, K, MB, EB)
    v = synth.gaussian_spinor(dims, 8, "full")
    got = op.D_full(v.reshape(dims + (2, 4, 3))).reshape(-1)
    assert np.abs(got - D @ v.reshape(-1)).max() < 1e-13


def test_schur_identity_dense():
    dims = (2, 2, 2, 2)
    lat, op, U = _op(dims)
    D = dense.dense_D_ND(dims, U, K, MB, EB)
    e, o = dense.parity_indices(dims)
    Dinv = np.linalg.inv(D)
    n = len(o)
    S = np.zeros((n, n), dtype=complex)
    for j in range(n):
        ej = np.zeros(n, dtype=complex)
        ej[j] = 1
        S[:, j] = op.S_hat(ej.reshape(-1, 2, 4, 3)).reshape(-1)
    assert np.abs(np.linalg.inv(S) - Dinv[np.ix_(o, o)]).max() < 1e-12
    assert np.abs(S - dense.dense_schur_odd(D, dims)).max() < 1e-12


@pytest.mark.parametrize("m", [0.37, -0.37, 1e-3])
def test_shifted_schur_is_odd_complement_of_dprime(m):
    # D' = D_ND + i m (Gamma5 x tau1) on the odd sites only leaves the even-even block
    # untouched, so its odd Schur complement is S + i m Gamma5 tau1 exactly; the dense
    # side inverts D'_ee numerically and never uses the closed-form A^-1
    dims = (2, 2, 2, 2)
    lat, op, U = _op(dims)
    Dp = dense.dense_D_ND(dims, U, K, MB, EB, odd_shift=m)
    n = len(dense.parity_indices(dims)[1])
    S = np.zeros((n, n), dtype=complex)
    for j in range(n):
        ej = np.zeros(n, dtype=complex)
        ej[j] = 1
        S[:, j] = op.S_shift(ej.reshape(-1, 2, 4, 3), m).reshape(-1)
    assert np.abs(S - dense.dense_schur_odd(Dp, dims)).max() < 1e-12
    # and Gamma5 tau1 (S + i m Gamma5 tau1) = Q + i m is Q shifted by i m
    Q = np.zeros((n, n), dtype=complex)
    for j in range(n):
        ej = np.zeros(n, dtype=complex)
        ej[j] = 1
        Q[:, j] = op.Q_hat(ej.reshape(-1, 2, 4, 3)).reshape(-1)
    G = dense.dense_g5t1(n // 24)
    assert np.abs(G @ S - (Q + 1j * m * np.eye(n))).max() < 1e-12
    # the [D'^-1]_oo block is the inverse of the shifted Schur complement
    e, o = dense.parity_indices(dims)
    assert np.abs(np.linalg.inv(S) - np.linalg.inv(Dp)[np.ix_(o, o)]).max() < 1e-10


@pytest.mark.parametrize("antiperiodic", [False, True])
def test_g5tau1_hermiticity(antiperiodic):
    dims = (4, 4, 2, 2)
    lat, op, U = _op(dims, seed=9, antiperiodic=antiperiodic)
    x = synth.gaussian_spinor(dims, 1)
    y = synth.gaussian_spinor(dims, 2)
    lhs = np.vdot(y, op.Q_hat(x))
    rhs = np.vdot(op.Q_hat(y), x)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)
    xf = synth.gaussian_spinor(dims, 3, "full").reshape(dims + (2, 4, 3))
    yf = synth.gaussian_spinor(dims, 4, "full").reshape(dims + (2, 4, 3))
    l2 = np.vdot(yf, op.g5t1(op.D_full(xf)))
    r2 = np.vdot(op.g5t1(op.D_full(yf)), xf)
    assert abs(l2 - r2) < 1e-12 * abs(l2)


def test_gauge_covariance():
    dims = (4, 2, 4, 2)
    lat, op, U = _op(dims, seed=13, antiperiodic=True)
    V = lat.V
    G = synth.random_su3(V, 99).reshape(dims + (3, 3))
    U6 = lat.U
    Ug = np.empty_like(U6)
    for mu in range(4):
        Gf = np.roll(G, -1, axis=MU_AXIS[mu])
        Ug[..., mu, :, :] = G @ U6[..., mu, :, :] @ np.conj(np.swapaxes(Gf, -1, -2))
    latg = Lattice(dims, Ug.reshape(V, 4, 3, 3), antiperiodic_t=True)
    opg = NDOperator(latg, K, MB, EB)
    x = synth.gaussian_spinor(dims, 5)
    Go = lat.take_odd(G)
    gx = np.einsum("hab,hfsb->hfsa", Go, x)
    lhs = opg.Q_hat(gx)
    rhs = np.einsum("hab,hfsb->hfsa", Go, op.Q_hat(x))
    assert np.abs(lhs - rhs).max() < 1e-12


def test_epsbar_zero_splits_flavours():
    dims = (2, 2, 2, 4)
    lat, op, U = _op(dims, epsbar=0.0)
    lat2, opw, _ = _op(dims, mubar=0.0, epsbar=0.0)
    v = synth.gaussian_spinor(dims, 6, "full").reshape(dims + (2, 4, 3))
    v1 = v.copy()
    v1[..., 1, :, :] = 0
    out = op.D_full(v1)
    assert np.abs(out[..., 1, :, :]).max() == 0
    dw = opw.D_full(v1)[..., 0, :, :]
    g5v = np.einsum("st,...tc->...sc", GAMMA5, v1[..., 0, :, :])
    assert np.abs(out[..., 0, :, :] - (dw + 1j * MB * g5v)).max() < 1e-13
    v2 = v.copy()
    v2[..., 0, :, :] = 0
    out2 = op.D_full(v2)
    dw2 = opw.D_full(v2)[..., 1, :, :]
    g5v2 = np.einsum("st,...tc->...sc", GAMMA5, v2[..., 1, :, :])
    assert np.abs(out2[..., 1, :, :] - (dw2 - 1j * MB * g5v2)).max() < 1e-13


def test_mubar_zero_eigenvectors():
    """mubar = 0: with D_W v = lam v, D_ND(0, eps) (v, +-v) = (lam -+ eps) (v, +-v)
    (section 3.2.1; the sign follows eq:non-degenerate's -epsbar tau1)."""
    dims = (2, 2, 2, 2)
    U = synth.gauge_field(dims, 3, 0.3)
    Dw = dense.dense_D_ND(dims, U, K, 0.0, 0.0)
    # single-flavour block of the flavour-diagonal operator
    idx = np.concatenate([np.arange(s * 24, s * 24 + 12) for s in range(16)])
    lam, vecs = np.linalg.eig(Dw[np.ix_(idx, idx)])
    lat = Lattice(dims, U)
    op = NDOperator(lat, K, 0.0, EB)
    for j in (0, 7, 100):
        v = vecs[:, j].reshape(16, 4, 3)
        for sgn in (1, -1):
            w = np.stack([v, sgn * v], axis=1).reshape(dims + (2, 4, 3))
            out = op.D_full(w)
            assert np.abs(out - (lam[j] - sgn * EB) * w).max() < 1e-11


def test_q_hat_spectrum_positive_and_bounded():
    """Q^2 = S^dag S >= 0 and bounded above by ||A||^2(1 + 16 ||A^-1|| / 4)^2-type norm bound."""
    dims = (2, 2, 2, 2)
    lat, op, U = _op(dims, seed=21)
    n = lat.V // 2 * 24
    Q = np.zeros((n, n), dtype=complex)
    for j in range(n):
        ej = np.zeros(n, dtype=complex)
        ej[j] = 1
        Q[:, j] = op.Q_hat(ej.reshape(-1, 2, 4, 3)).reshape(-1)
    assert np.abs(Q - Q.conj().T).max() < 1e-13
    ev = np.linalg.eigvalsh(Q @ Q)
    assert ev.min() > 0
    nA = np.linalg.norm(op.A_block, 2)
    nAi = np.linalg.norm(op.Ainv_block, 2)
    assert ev.max() <= (nA + 0.25 * 8 * 8 * nAi) ** 2
