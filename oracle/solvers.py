"""Krylov solvers and initial guesses of the oracle (FP64, NumPy).

* ``cg``        conjugate gradient on a Hermitian positive operator (case A of
                section 3.1 for a single shift).
* ``mms_cg``    multi-mass-shift CG (the "standard" solver of section 1 and the
                MMS-CG subsection of section 4.2): one Krylov space, built for the
                smallest shift, iterates every shifted system.  The shifted
                coefficients are re-derived here from r_s = zeta_s r.
* ``lagrange_coefficients``  l_i(sigma_t) of the Lagrange-interpolation guess
                (section 4.2, appendix B), nodes = the shifts sigma_i.
* ``case_c``    difference of single solves, eq:lindif.
* ``gmres``     restarted GMRES for the single shifted systems.
"""
from __future__ import annotations

import numpy as np


def _dot(a, b):
    return np.vdot(a, b)


def _n2(a):
    return float(np.vdot(a, a).real)


def cg(apply_A, b, tol=1e-10, maxiter=100000, x0=None):
    """Plain CG for A x = b, stop when ||r|| <= tol ||b|| (recursive residual)."""
    x = np.zeros_like(b) if x0 is None else x0.copy()
    r = b - apply_A(x) if x0 is not None else b.copy()
    p = r.copy()
    rr = _n2(r)
    bb = _n2(b)
    it = 0
    while rr > tol * tol * bb and it < maxiter:
        w = apply_A(p)
        alpha = rr / float(_dot(p, w).real)
        x += alpha * p
        r -= alpha * w
        rr_new = _n2(r)
        p = r + (rr_new / rr) * p
        rr = rr_new
        it += 1
    return x, it


def mms_cg(apply_A, b, deltas, tol=1e-10, maxiter=100000, record=False):
    """Multi-shift CG for (A + delta_s) x_s = b, all delta_s >= 0, A Hermitian positive.

    The base CG runs on A (delta = 0, the most ill-conditioned system).  With
    r_s = zeta_s r for every shift, matching the shifted recursion to the base
    one gives, with zeta_{-1} = zeta_0 = 1, alpha_{-1} = 1, beta_{-1} = 0:

        zeta_{k+1} = zeta_k zeta_{k-1} alpha_{k-1} /
                     (alpha_k beta_{k-1} (zeta_{k-1} - zeta_k)
                      + zeta_{k-1} alpha_{k-1} (1 + delta alpha_k))
        alpha_k^s  = alpha_k zeta_{k+1} / zeta_k
        beta_k^s   = beta_k (zeta_{k+1} / zeta_k)^2
        x^s += alpha_k^s p^s ;  p^s = zeta_{k+1} r_{k+1} + beta_k^s p^s.

    A shift is frozen once |zeta_s| ||r|| <= tol ||b||; the loop ends when every
    shift is frozen.  Returns (xs, iterations, per-shift iteration counts[, log]).
    """
    deltas = np.asarray(deltas, dtype=np.float64)
    n = len(deltas)
    xs = [np.zeros_like(b) for _ in range(n)]
    ps = [b.copy() for _ in range(n)]
    r = b.copy()
    p = b.copy()
    rr = _n2(r)
    bb = _n2(b)
    zeta = np.ones(n)
    zeta_prev = np.ones(n)
    alpha_prev = 1.0
    beta_prev = 0.0
    active = np.ones(n, dtype=bool)
    iters = np.zeros(n, dtype=int)
    log = []
    it = 0
    while active.any() and it < maxiter:
        w = apply_A(p)
        alpha = rr / float(_dot(p, w).real)
        zeta_next = zeta.copy()
        for s in range(n):
            if not active[s]:
                continue
            den = (alpha * beta_prev * (zeta_prev[s] - zeta[s])
                   + zeta_prev[s] * alpha_prev * (1.0 + deltas[s] * alpha))
            zeta_next[s] = zeta[s] * zeta_prev[s] * alpha_prev / den
            a_s = alpha * zeta_next[s] / zeta[s]
            xs[s] += a_s * ps[s]
        r = r - alpha * w
        rr_new = _n2(r)
        beta = rr_new / rr
        for s in range(n):
            if not active[s]:
                continue
            b_s = beta * (zeta_next[s] / zeta[s]) ** 2
            ps[s] = zeta_next[s] * r + b_s * ps[s]
        p = r + beta * p
        zeta_prev, zeta = zeta, zeta_next
        alpha_prev, beta_prev = alpha, beta
        rr = rr_new
        it += 1
        iters[active] = it
        if record:
            log.append(dict(alpha=alpha, beta=beta, zeta=zeta.copy(), rr=rr))
        for s in range(n):
            if active[s] and abs(zeta[s]) * np.sqrt(rr) <= tol * np.sqrt(bb):
                active[s] = False
    if record:
        return xs, it, iters, log
    return xs, it, iters


def lagrange_coefficients(nodes, target):
    """l_i(target) = prod_{j != i} (target - node_j)/(node_i - node_j) (section 4.2, appendix B).

    With a single node l_1 = 1 (appendix B's convention)."""
    nodes = np.asarray(nodes, dtype=np.float64)
    k = len(nodes)
    c = np.ones(k)
    for i in range(k):
        for j in range(k):
            if j != i:
                c[i] *= (target - nodes[j]) / (nodes[i] - nodes[j])
    return c


def lebesgue(nodes, target):
    """gamma_k(target) = sum_i |l_i(target)| (appendix B)."""
    return float(np.abs(lagrange_coefficients(nodes, target)).sum())


def lagrange_guess(xs, nodes, target):
    """x_guess = sum_i l_i(target) x_i (interpolation of the converged solutions)."""
    c = lagrange_coefficients(nodes, target)
    out = np.zeros_like(xs[0])
    for ci, xi in zip(c, xs):
        out += ci * xi
    return out


def gmres(apply_A, b, tol=1e-10, restart=30, maxiter=5000, x0=None):
    """Restarted GMRES (modified Gram-Schmidt, Givens rotations) for a general A."""
    x = np.zeros_like(b) if x0 is None else x0.copy()
    bn = np.sqrt(_n2(b))
    total = 0
    shape = b.shape
    while total < maxiter:
        r = b - apply_A(x)
        beta = np.sqrt(_n2(r))
        if beta <= tol * bn:
            break
        Vb = [r / beta]
        H = np.zeros((restart + 1, restart), dtype=np.complex128)
        g = np.zeros(restart + 1, dtype=np.complex128)
        g[0] = beta
        cs = np.zeros(restart, dtype=np.complex128)
        sn = np.zeros(restart, dtype=np.complex128)
        k_done = 0
        for k in range(restart):
            w = apply_A(Vb[k])
            for i in range(k + 1):
                H[i, k] = _dot(Vb[i], w)
                w = w - H[i, k] * Vb[i]
            H[k + 1, k] = np.sqrt(_n2(w))
            Vb.append(w / H[k + 1, k] if H[k + 1, k] != 0 else w)
            # Givens rotation G = [[conj(c), conj(s)], [-s, c]] maps (h_kk, h_k+1,k) to (rho, 0)
            for i in range(k):
                t = np.conj(cs[i]) * H[i, k] + np.conj(sn[i]) * H[i + 1, k]
                H[i + 1, k] = -sn[i] * H[i, k] + cs[i] * H[i + 1, k]
                H[i, k] = t
            den = np.sqrt(abs(H[k, k]) ** 2 + abs(H[k + 1, k]) ** 2)
            cs[k] = H[k, k] / den
            sn[k] = H[k + 1, k] / den
            H[k, k] = den
            H[k + 1, k] = 0
            g[k + 1] = -sn[k] * g[k]
            g[k] = np.conj(cs[k]) * g[k]
            total += 1
            k_done = k + 1
            if abs(g[k + 1]) <= tol * bn or total >= maxiter:
                break
        y = np.linalg.solve(np.triu(H[:k_done, :k_done]), g[:k_done])
        for i in range(k_done):
            x = x + y[i] * Vb[i]
    return x.reshape(shape), total


def case_c(solve_plus, solve_minus, b, m):
    """Difference of single solves, eq:lindif:
    (Q^2 + m^2)^-1 b = (i / 2m) [ (Q + i m)^-1 b - (Q - i m)^-1 b ]."""
    xp = solve_plus(b)
    xm = solve_minus(b)
    return (1j / (2.0 * m)) * (xp - xm)


def projection_guess(apply_At, xs, b):
    """Minimal-residual combination of the converged solutions (generalises the
    interpolated guesses of section 4.2): c = argmin || b - A_t sum_i c_i x_i ||
    over complex c, with the products A_t x_i formed explicitly (the plain
    definition; the appendix B identity is not used here).  Returns (x, c)."""
    Y = np.stack([np.asarray(apply_At(x)).reshape(-1) for x in xs], axis=1)
    c, *_ = np.linalg.lstsq(Y, np.asarray(b).reshape(-1), rcond=None)
    x = sum(ci * xi for ci, xi in zip(c, xs))
    return x, c
