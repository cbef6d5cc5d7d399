"""Pins of the oracle's Zolotarev rational approximation (section "Rational
approximation", eq:rational, eq:deviation, eq:zolotarev_shifts, eq:ratapp).

* n = 0 reduces to the best constant relative approximation of 1/sqrt(y) on
  [eps, 1]: a = 2/(1 + sqrt(eps)), delta = (1 - sqrt(eps))/(1 + sqrt(eps));
* the error 1 - sqrt(y) R(y) equioscillates: 2n + 2 alternating extrema of size
  delta, endpoints included (the characterisation of the best approximation);
* the partial-fraction form of eq:ratapp equals the product form;
* zeros and poles interlace, c_1 > c_2 > ... > c_2n > 0, and delta falls with n;
* applied to a dense Hermitian positive matrix with spectrum in [eps lam, lam],
  the result is within delta of A^{-1/2} b.
"""
import numpy as np
import pytest

from oracle import zolotarev as z


@pytest.mark.parametrize("eps", [0.3, 1e-2, 1e-5])
def test_order_zero_is_the_best_constant(eps):
    c, a, d = z.coefficients(0, eps)
    assert len(c) == 0
    r = np.sqrt(eps)
    # d^2 = 1 - eps here, so 1 - d^2 loses digits to cancellation for small eps
    assert abs(a - 2.0 / (1.0 + r)) <= 1e-12 * a
    assert abs(d - (1.0 - r) / (1.0 + r)) <= 1e-12


def _extrema(n, eps, pts=200001):
    c, a, d = z.coefficients(n, eps)
    y = np.exp(np.linspace(np.log(eps), 0.0, pts))
    e = 1.0 - np.sqrt(y) * z.evaluate_product(y, c, a)
    idx = [0] + [i for i in range(1, pts - 1) if (e[i] - e[i - 1]) * (e[i + 1] - e[i]) <= 0] + [pts - 1]
    return e[idx], d, np.abs(e).max()


@pytest.mark.parametrize("n,eps", [(1, 0.01), (3, 1e-3), (6, 1e-4), (8, 1e-5)])
def test_equioscillation(n, eps):
    ext, d, emax = _extrema(n, eps)
    assert len(ext) == 2 * n + 2
    assert np.all(np.sign(ext[1:]) == -np.sign(ext[:-1]))
    # every extremum reaches delta (the grid resolves the interior ones to ~1e-8)
    assert np.all(np.abs(np.abs(ext) - d) <= 1e-6 * d)
    assert emax <= d * (1 + 1e-9)


@pytest.mark.parametrize("n,eps", [(1, 0.1), (5, 1e-4), (12, 1e-6)])
def test_partial_fractions_and_ordering(n, eps):
    c, a, d = z.coefficients(n, eps)
    assert np.all(c > 0) and np.all(np.diff(c) < 0)
    y = np.random.default_rng(n).uniform(eps, 1.0, 1000)
    p, s = z.evaluate_product(y, c, a), z.evaluate_sum(y, c, a)
    assert np.abs(s / p - 1).max() <= 1e-13
    m2, q = z.partial_fractions(c)
    assert np.all(q > 0) and np.allclose(m2, c[1::2])


def test_deviation_falls_with_order():
    ds = [z.coefficients(n, 1e-4)[2] for n in range(0, 12)]
    assert all(b < a for a, b in zip(ds, ds[1:]))
    # exponential convergence: the ratio settles
    assert ds[11] < 1e-6 * ds[1]


def test_apply_to_dense_matrix():
    rng = np.random.default_rng(5)
    N = 40
    lam, eps = 7.0, 1e-3
    ev = np.exp(rng.uniform(np.log(eps * lam), np.log(lam), N))
    Q, _ = np.linalg.qr(rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N)))
    A = (Q * ev) @ Q.conj().T
    b = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    exact = (Q * ev ** -0.5) @ (Q.conj().T @ b)
    for n in (4, 8):
        d = z.coefficients(n, eps)[2]
        x = z.apply(lambda s: np.linalg.solve(A + s * np.eye(N), b), b, n, eps, lam)
        err = np.linalg.norm(x - exact)
        # each eigencomponent is off by a factor 1 - sqrt(y) R(y), |.| <= delta
        assert err <= d * np.linalg.norm(exact) * (1 + 1e-8)
        assert err > 1e-3 * d * np.linalg.norm(exact)  # the bound is close to attained
