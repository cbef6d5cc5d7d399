"""Rational approximation on the GPU (section "Rational approximation",
eq:rational, eq:zolotarev_shifts, eq:ratapp) against the oracle.

* ndtm_zolotarev (the library's AGM elliptic functions) against the oracle's
  coefficients (scipy's elliptic functions): c_k to 1e-12, a and delta to 1e-13;
* on 2^4, where Q^2 is a dense matrix: ndtm_solve_rational's y lies within delta
  (plus the solve tolerance) of (Q^2)^{-1/2} b from the eigendecomposition, and
  matches the oracle's own rational application with dense solves;
* on the 4^4 config, y matches the oracle's rational application with its own
  CG solves, with the shifts solved as one multi-shift CG;
* argument errors.
"""
import numpy as np
import pytest

import synth
from oracle import solvers
from oracle import zolotarev as oz
from oracle.lattice import Lattice, NDOperator, norm2
from tests.gpu_util import dev, host

pytestmark = pytest.mark.gpu

K, MB, EB = synth.KAPPA, synth.MUBAR, synth.EPSBAR


@pytest.fixture(scope="module")
def nd():
    import paper_1805_09584_amd as nd
    return nd


@pytest.mark.parametrize("n,eps", [(0, 0.01), (1, 0.01), (5, 1e-4), (12, 1e-6), (16, 1e-7)])
def test_coefficients_match_oracle(nd, n, eps):
    c, a, d = nd.zolotarev(n, eps)
    co, ao, do = oz.coefficients(n, eps)
    if n:
        assert np.abs(c / co - 1).max() <= 1e-12
    assert abs(a / ao - 1) <= 1e-13 and abs(d / do - 1) <= 1e-13


def _ctx(nd, dims, seed):
    U = synth.gauge_field(dims, seed, 0.3)
    ctx = nd.Context(dims)
    ctx.ndtm_set_gauge(dev(U))
    ctx.ndtm_set_params(K, MB, EB)
    return ctx, NDOperator(Lattice(dims, U), K, MB, EB)


def test_rational_dense_2x4(nd):
    print("rational approximation 2^4 dense", flush=True)
    dims = (2, 2, 2, 2)
    ctx, op = _ctx(nd, dims, 51)
    nodd = op.lat.V // 2 * 24
    Q = np.zeros((nodd, nodd), dtype=complex)
    for j in range(nodd):
        e = np.zeros(nodd, dtype=complex)
        e[j] = 1
        Q[:, j] = op.Q_hat(e.reshape(-1, 2, 4, 3)).reshape(-1)
    ev, W = np.linalg.eigh(Q @ Q)
    lam, eps = 1.02 * ev.max(), 0.98 * ev.min() / (1.02 * ev.max())
    b = synth.gaussian_spinor(dims, 52)
    bv = b.reshape(-1)
    exact = W @ ((W.conj().T @ bv) / np.sqrt(ev))
    for n in (4, 10):
        d = oz.coefficients(n, eps)[2]
        y, rep = ctx.ndtm_solve_rational(dev(b), n, eps, lam, ctx.solve_params(tol=1e-12))
        y = host(y).reshape(-1)
        err = np.linalg.norm(y - exact) / np.linalg.norm(exact)
        yo = oz.apply(lambda s: np.linalg.solve(Q @ Q + s * np.eye(nodd), bv), bv, n, eps, lam)
        print("n", n, "delta", d, "error vs exact", err, "vs oracle", np.linalg.norm(y - yo) / np.linalg.norm(yo),
              flush=True)
        assert rep["n_shifts"] == n and max(rep["true_res"][:n]) <= 1e-12
        assert err <= d + 1e-9
        assert np.linalg.norm(y - yo) <= 1e-9 * np.linalg.norm(yo)
    ctx.close()


def test_rational_config1(nd):
    print("rational approximation c1", flush=True)
    c = synth.CONFIGS["c1"]
    dims = c["dims"]
    ctx, op = _ctx(nd, dims, c["gauge_seed"])
    b = synth.gaussian_spinor(dims, c["rhs_seed"])
    # spectrum bounds: power iteration for the top, a loose bottom
    v = synth.gaussian_spinor(dims, 7)
    for _ in range(60):
        v = op.Q_hat2(v, 0.0)
        v /= np.sqrt(norm2(v))
    lam = 1.05 * float(np.vdot(v, op.Q_hat2(v, 0.0)).real)
    n, eps = 10, 1e-4
    y, rep = ctx.ndtm_solve_rational(dev(b), n, eps, lam, ctx.solve_params(tol=1e-11))
    yo = oz.apply(lambda s: solvers.cg(lambda u: op.Q_hat2(u, s), b, tol=1e-13)[0], b, n, eps, lam)
    rel = np.sqrt(norm2(host(y) - yo) / norm2(yo))
    print("lambda", lam, "mms iterations", rep["mms_iterations"], "relative difference", rel, flush=True)
    assert rep["method"][:n] == [0] * n
    assert rel <= 1e-9
    ctx.close()


def test_rational_argument_errors(nd):
    ctx, op = _ctx(nd, (2, 2, 2, 2), 53)
    b = dev(synth.gaussian_spinor((2, 2, 2, 2), 54))
    for n, eps, lam in ((0, 0.1, 1.0), (17, 0.1, 1.0), (4, 1.0, 1.0), (4, 0.1, -1.0)):
        with pytest.raises(nd.NdtmError) as e:
            ctx.ndtm_solve_rational(b, n, eps, lam)
        assert e.value.code == -1
    with pytest.raises(nd.NdtmError):
        nd.zolotarev(-1, 0.1)
    ctx.close()
