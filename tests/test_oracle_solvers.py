"""Pins of the oracle's solvers and guesses.

* MMS-CG against a dense inverse on 2^4 within the appendix A error bound for
  case A, ||e|| <= ||r|| / lambda_min(Q^2 + sigma), and against independent
  single-shift CG;
* the first shifted coefficient zeta_1 = 1/(1 + delta alpha_0) and zeta = 1 for
  delta = 0 (consequences of r_s = zeta_s r);
* Lagrange coefficients: sum l_i = 1 (eq:lagrange_id), exact reproduction of
  polynomials of degree < k, the residual identity eq:residual_interpolation;
* case C, eq:lindif, exactly on dense matrices and through GMRES;
* GMRES against a dense solve.
"""
import numpy as np
import pytest

import synth
from oracle import dense, solvers
from oracle.lattice import Lattice, NDOperator, norm2, rel_residual

K, MB, EB = synth.KAPPA, synth.MUBAR, synth.EPSBAR


def _dense_Q(dims, U):
    D = dense.dense_D_ND(dims, U, K, MB, EB)
    S = dense.dense_schur_odd(D, dims)
    return dense.dense_g5t1(int(np.prod(dims)) // 2) @ S


@pytest.fixture(scope="module")
def small():
    dims = (2, 2, 2, 2)
    U = synth.gauge_field(dims, 11, 0.3)
    lat = Lattice(dims, U)
    op = NDOperator(lat, K, MB, EB)
    b = synth.gaussian_spinor(dims, 21)
    Q = _dense_Q(dims, U)
    return dims, op, b, Q


def test_mms_cg_matches_dense_inverse(small):
    dims, op, b, Q = small
    sig = synth.geometric_shifts(10, 1e-4)
    xs, it, iters = solvers.mms_cg(lambda v: op.Q_hat2(v, sig[-1]), b, sig - sig[-1], tol=1e-10)
    Q2 = Q @ Q
    lmin = np.linalg.eigvalsh(Q2).min()
    for s, x in zip(sig, xs):
        xe = np.linalg.solve(Q2 + s * np.eye(len(Q2)), b.reshape(-1))
        res = rel_residual(op, x, b, s)
        assert res <= 1e-10
        err = np.linalg.norm(x.reshape(-1) - xe)
        assert err <= res * np.sqrt(norm2(b)) / (lmin + s) * (1 + 1e-6) + 1e-14


def test_mms_cg_vs_single_cg():
    dims = (4, 4, 2, 2)
    U = synth.gauge_field(dims, 5, 0.3)
    op = NDOperator(Lattice(dims, U), K, MB, EB)
    b = synth.gaussian_spinor(dims, 6)
    sig = np.array([0.5, 0.05, 0.001])
    xs, it, iters = solvers.mms_cg(lambda v: op.Q_hat2(v, sig[-1]), b, sig - sig[-1], tol=1e-11)
    for s, x in zip(sig, xs):
        xc, _ = solvers.cg(lambda v: op.Q_hat2(v, s), b, tol=1e-11)
        assert rel_residual(op, x, b, s) < 1e-10
        assert rel_residual(op, xc, b, s) < 1e-10
        assert np.linalg.norm(x - xc) <= 1e-8 * np.linalg.norm(xc)
    # larger shifts converge first
    assert iters[0] < iters[1] < iters[2]


def test_mms_zeta_first_step_and_zero_shift(small):
    dims, op, b, Q = small
    deltas = np.array([0.0, 0.3])
    xs, it, iters, log = solvers.mms_cg(lambda v: op.Q_hat2(v, 0.01), b, deltas, tol=1e-6, record=True)
    a0 = log[0]["alpha"]
    assert abs(log[0]["zeta"][1] - 1.0 / (1.0 + 0.3 * a0)) < 1e-14
    assert all(abs(e["zeta"][0] - 1.0) < 1e-14 for e in log)
    # recursive residual |zeta_s| ||r|| equals the true residual of shift s along the way
    xs2, _, it2, log2 = solvers.mms_cg(lambda v: op.Q_hat2(v, 0.01), b, deltas, tol=1e-3, record=True)
    tr = np.sqrt(norm2(b - op.Q_hat2(xs2[1], 0.31)))
    k = it2[1] - 1  # last iteration in which shift 1 was updated
    rec = abs(log2[k]["zeta"][1]) * np.sqrt(log2[k]["rr"])
    assert abs(tr - rec) <= 1e-8 * np.sqrt(norm2(b))


def test_lagrange_identities():
    nodes = synth.geometric_shifts(12, 1e-5)[:9]
    for t in (8.111e-5, 1e-5, 0.2):
        c = solvers.lagrange_coefficients(nodes, t)
        assert abs(c.sum() - 1.0) < 1e-9 * np.abs(c).max()
    # reproduces polynomials of degree < k exactly (up to rounding)
    nodes = np.array([1.0, 0.5, 0.2, 0.1])
    poly = lambda s: 3 - 2 * s + 5 * s ** 3
    c = solvers.lagrange_coefficients(nodes, 0.05)
    assert abs(c @ poly(nodes) - poly(0.05)) < 1e-12
    assert np.allclose(solvers.lagrange_coefficients([0.7], 0.1), [1.0])


def test_lagrange_residual_identity(small):
    """b - (Q^2 + s) sum l_i x_i = sum l_i ((s_i - s) x_i + r_i) for arbitrary x_i (appendix B)."""
    dims, op, b, Q = small
    nodes = np.array([1.0, 0.3, 0.1, 0.02])
    s = 0.004
    xs = [synth.gaussian_spinor(dims, 40 + i) for i in range(4)]
    rs = [b - op.Q_hat2(x, si) for x, si in zip(xs, nodes)]
    l = solvers.lagrange_coefficients(nodes, s)
    lhs = b - op.Q_hat2(sum(li * x for li, x in zip(l, xs)), s)
    rhs = sum(li * ((si - s) * x + r) for li, si, x, r in zip(l, nodes, xs, rs))
    assert np.abs(lhs - rhs).max() < 1e-10 * np.abs(lhs).max()


def test_lebesgue_of_config_shifts():
    """gamma_n(sigma_{n+1}) with all previous nodes, descending order: small (appendix B)."""
    for n_sh, smallest in ((10, 1e-4), (12, 1e-5)):
        sig = synth.geometric_shifts(n_sh, smallest)
        g = [solvers.lebesgue(sig[:n], sig[n]) for n in range(1, n_sh)]
        assert max(g) < 2.5
        assert min(g) >= 1.0


def test_case_c_dense_identity(small):
    dims, op, b, Q = small
    n = len(Q)
    for m2 in (1e-5, 0.3):
        m = np.sqrt(m2)
        sp = lambda c: np.linalg.solve(Q + 1j * m * np.eye(n), c.reshape(-1))
        sm = lambda c: np.linalg.solve(Q - 1j * m * np.eye(n), c.reshape(-1))
        xc = solvers.case_c(sp, sm, b, m)
        xe = np.linalg.solve(Q @ Q + m2 * np.eye(n), b.reshape(-1))
        assert np.linalg.norm(xc - xe) < 1e-11 * np.linalg.norm(xe)


def test_case_c_through_shifted_schur_gmres(small):
    """(Q +- i m) x = b  <=>  (S +- i m Gamma5 tau1) x = Gamma5 tau1 b."""
    dims, op, b, Q = small
    m = np.sqrt(2.8e-5)
    n = len(Q)
    for sgn in (1, -1):
        x, _ = solvers.gmres(lambda v: op.S_shift(v, sgn * m), op.g5t1(b), tol=1e-13, restart=50)
        xe = np.linalg.solve(Q + sgn * 1j * m * np.eye(n), b.reshape(-1))
        assert np.linalg.norm(x.reshape(-1) - xe) < 1e-9 * np.linalg.norm(xe)


def test_case_c_residual_formula(small):
    """r_C = (i/2m)[(Q - i m) r_+ - (Q + i m) r_-] for inexact single solves (appendix A, case C)."""
    dims, op, b, Q = small
    n = len(Q)
    m = 0.05
    bv = b.reshape(-1)
    rng = np.random.default_rng(1)
    xp = np.linalg.solve(Q + 1j * m * np.eye(n), bv) + 1e-3 * rng.standard_normal(n)
    xm = np.linalg.solve(Q - 1j * m * np.eye(n), bv) + 1e-3 * rng.standard_normal(n)
    rp = bv - (Q + 1j * m * np.eye(n)) @ xp
    rm = bv - (Q - 1j * m * np.eye(n)) @ xm
    xc = (1j / (2 * m)) * (xp - xm)
    rc = bv - (Q @ Q + m * m * np.eye(n)) @ xc
    want = (1j / (2 * m)) * ((Q - 1j * m * np.eye(n)) @ rp - (Q + 1j * m * np.eye(n)) @ rm)
    assert np.abs(rc - want).max() < 1e-10 * np.abs(rc).max()


def test_gmres_dense():
    rng = np.random.default_rng(2)
    n = 60
    A = np.eye(n) * 4 + 0.3 * (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    x, it = solvers.gmres(lambda v: A @ v, b, tol=1e-12, restart=15)
    assert np.linalg.norm(A @ x - b) <= 1e-12 * np.linalg.norm(b) * 1.01


def test_projection_guess_pins():
    """K = 1 closed form; the residual is orthogonal to every A_t x_i (first-order
    optimality); it is no larger than the Lagrange guess's and than any perturbed
    combination."""
    dims = (2, 2, 2, 4)
    U = synth.gauge_field(dims, 7, 0.3)
    op = NDOperator(Lattice(dims, U), synth.KAPPA, synth.MUBAR, synth.EPSBAR)
    b = synth.gaussian_spinor(dims, 8)
    nodes = np.array([0.5, 0.1, 0.02, 0.004])
    st = 0.001
    xs = [solvers.cg(lambda v, s=s: op.Q_hat2(v, s), b, tol=1e-13)[0] for s in nodes]
    At = lambda v: op.Q_hat2(v, st)
    # K = 1: c = <A x, b> / <A x, A x>
    x1, c1 = solvers.projection_guess(At, xs[-1:], b)
    y = At(xs[-1])
    assert abs(c1[0] - np.vdot(y, b) / np.vdot(y, y)) < 1e-12 * abs(c1[0])
    x, c = solvers.projection_guess(At, xs, b)
    r = b - At(x)
    for xi in xs:
        assert abs(np.vdot(At(xi), r)) <= 1e-9 * np.linalg.norm(At(xi)) * np.linalg.norm(b)
    xl = solvers.lagrange_guess(xs, nodes, st)
    assert norm2(r) <= norm2(b - At(xl))
    rng = np.random.default_rng(1)
    for _ in range(3):
        dc = 1e-3 * (rng.standard_normal(len(c)) + 1j * rng.standard_normal(len(c)))
        xp = sum((ci + di) * xi for ci, di, xi in zip(c, dc, xs))
        assert norm2(b - At(xp)) >= norm2(r)
