"""Zolotarev's optimal rational approximation of 1/sqrt(y) (oracle, FP64).

Test infrastructure: only tests/, smoke() and the bench's CPU baseline use the
oracle.

Section "Rational approximation" (eq:rational, eq:deviation, eq:zolotarev_shifts,
eq:ratapp): on eps < y < 1,

    R(y) = a prod_{j=1..n} (y + c_{2j-1}) / (y + c_{2j}),
    c_k = cs^2(k v, k'),  s_k = sn^2(k v, k'),  v = K(k') / (2n + 1),  k' = sqrt(1 - eps),
    d   = (1 - eps)^{(2n+1)/2} prod_{j=1..n} s_{2j-1}^2,
    a   = 2 / (1 + sqrt(1 - d^2)) prod_{j=1..n} s_{2j-1} / s_{2j},

and R(y) = a (1 + sum_i q_i / (y + m_i^2)) with m_i^2 = c_{2i} and
q_i = (c_{2i-1} - c_{2i}) prod_{j != i} (c_{2j-1} - c_{2i}) / (c_{2j} - c_{2i}).

The maximal deviation max |1 - sqrt(y) R(y)| is delta = d^2 / (1 + sqrt(1 - d^2))^2.
The text prints the denominator without the square; the squared form is the one
the approximation attains (for n = 0 it gives the optimal constant's deviation
(1 - sqrt(eps)) / (1 + sqrt(eps)), and the equioscillation test pins it for n >= 1).

The Jacobi elliptic functions and K come from scipy.special (parameter m = k^2).
"""
from __future__ import annotations

import numpy as np
from scipy import special


def coefficients(n: int, eps: float):
    """(c[0..2n-1] = c_1..c_2n, a, delta) for order n on [eps, 1]."""
    if n < 0 or not (0.0 < eps < 1.0):
        raise ValueError("n >= 0 and 0 < eps < 1")
    m = 1.0 - eps  # k'^2
    v = special.ellipk(m) / (2 * n + 1)
    k = np.arange(1, 2 * n + 1)
    sn, cn, _, _ = special.ellipj(k * v, m)
    s = sn ** 2
    c = (cn / sn) ** 2
    d = (1.0 - eps) ** ((2 * n + 1) / 2.0) * np.prod(s[0::2] ** 2)
    a = 2.0 / (1.0 + np.sqrt(1.0 - d * d)) * np.prod(s[0::2] / s[1::2])
    delta = d * d / (1.0 + np.sqrt(1.0 - d * d)) ** 2
    return c, float(a), float(delta)


def evaluate_product(y, c, a):
    """R(y) in the product form of eq:rational."""
    y = np.asarray(y, dtype=np.float64)
    r = np.full_like(y, a)
    for j in range(len(c) // 2):
        r = r * (y + c[2 * j]) / (y + c[2 * j + 1])
    return r


def partial_fractions(c):
    """(shifts m_i^2 = c_{2i}, weights q_i) of eq:ratapp."""
    n = len(c) // 2
    odd, even = c[0::2], c[1::2]
    q = np.empty(n)
    for i in range(n):
        q[i] = odd[i] - even[i]
        for j in range(n):
            if j != i:
                q[i] *= (odd[j] - even[i]) / (even[j] - even[i])
    return even.copy(), q


def evaluate_sum(y, c, a):
    """R(y) = a (1 + sum_i q_i / (y + m_i^2))."""
    y = np.asarray(y, dtype=np.float64)
    m2, q = partial_fractions(c)
    r = np.ones_like(y)
    for mi, qi in zip(m2, q):
        r = r + qi / (y + mi)
    return a * r


def apply(solve_shifted, b, n, eps, lam):
    """x ~ (A)^{-1/2} b for A Hermitian positive with spectrum in [eps lam, lam]:
    A^{-1/2} = lam^{-1/2} (A/lam)^{-1/2}, so with the shifted solves
    x_i = (A + lam m_i^2)^{-1} b,  x = lam^{-1/2} a (b + sum_i q_i lam x_i).
    solve_shifted(sigma) returns (A + sigma)^{-1} b."""
    c, a, _ = coefficients(n, eps)
    m2, q = partial_fractions(c)
    x = b.copy()
    for mi, qi in zip(m2, q):
        x = x + (qi * lam) * solve_shifted(lam * mi)
    return (a / np.sqrt(lam)) * x
