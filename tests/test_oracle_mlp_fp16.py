"""Pins of the oracle's network and FP16 codec.

* backward against central finite differences of the loss;
* the Gram-form loss equals the directly computed ||b - (Q^2 + s) x||^2 /
  ||r_L||^2 on explicit vectors (appendix B identity r = b + sum c_i w_i);
* L(0) = 1 (Lagrange) and c0 is the least-squares optimum over the span;
* FP16 codec: round-trip error <= 2^-11 * scale; NumPy's float16 rounding is
  round-to-nearest-even on exactly representable midpoints.
"""
import numpy as np

import synth
from oracle import fp16, mlp, solvers
from oracle.lattice import Lattice, NDOperator, norm2


def _batch(B=5, seed=0):
    rng = np.random.default_rng(seed)
    F = rng.standard_normal((B, mlp.N_FEAT))
    mask = (rng.random((B, mlp.K_MAX)) < 0.8).astype(float)
    R = rng.standard_normal((B, mlp.K_MAX, mlp.K_MAX))
    q = rng.standard_normal((B, mlp.K_MAX))
    c0 = rng.random(B)
    return F, mask, R, q, c0


def test_backward_finite_differences():
    p = mlp.init_params(1, out_scale=0.3)
    F, mask, R, q, c0 = _batch()

    def L(pp):
        y, _ = mlp.forward(pp, F)
        return mlp.loss(y, mask, R, q, c0)[0]

    y, cache = mlp.forward(p, F)
    _, dy, _ = mlp.loss(y, mask, R, q, c0)
    g = mlp.backward(p, cache, dy)
    rng = np.random.default_rng(3)
    for k in p:
        for _ in range(4):
            idx = tuple(rng.integers(0, s) for s in p[k].shape)
            h = 1e-6
            pp = {kk: vv.copy() for kk, vv in p.items()}
            pp[k][idx] += h
            lp = L(pp)
            pp[k][idx] -= 2 * h
            lm = L(pp)
            fd = (lp - lm) / (2 * h)
            assert abs(fd - g[k][idx]) <= 1e-6 * max(1.0, abs(fd))


def test_gram_loss_matches_direct_residual():
    dims = (2, 2, 2, 2)
    U = synth.gauge_field(dims, 3, 0.3)
    op = NDOperator(Lattice(dims, U), synth.KAPPA, synth.MUBAR, synth.EPSBAR)
    b = synth.gaussian_spinor(dims, 4)
    nodes = np.array([1.0, 0.2, 0.05, 0.01])
    st = 0.003
    xs = [solvers.cg(lambda v: op.Q_hat2(v, s), b, tol=1e-6)[0] for s in nodes]
    rs = [b - op.Q_hat2(x, s) for x, s in zip(xs, nodes)]
    vecs = [b] + xs + rs
    M = np.array([[np.vdot(u, v) for v in vecs] for u in vecs])
    Kn = len(nodes)
    Gw, gb, bb = mlp.w_gram(M, Kn, nodes, st)
    lag = solvers.lagrange_coefficients(nodes, st)
    R, q, c0, rL2 = mlp.quad_form(Gw, gb, bb, lag)
    xL = sum(l * x for l, x in zip(lag, xs))
    assert abs(rL2 - norm2(b - op.Q_hat2(xL, st))) < 1e-8 * rL2
    rng = np.random.default_rng(5)
    for scale in (0.0, 1e-3, 1e-1):
        dc = scale * rng.standard_normal(Kn)
        x = sum((l + d) * xi for l, d, xi in zip(lag, dc, xs))
        direct = norm2(b - op.Q_hat2(x, st)) / rL2
        u = R @ dc + q
        assert abs(c0 + u @ u - direct) < 1e-7 * max(1.0, direct)
    # c0 is the least-squares optimum: no coefficient vector does better
    W = np.stack([(r - b + (s - st) * x).reshape(-1) for x, r, s in zip(xs, rs, nodes)], axis=1)
    rL = (b - op.Q_hat2(xL, st)).reshape(-1)
    dc_opt, *_ = np.linalg.lstsq(W, -rL, rcond=None)
    best = norm2(rL + W @ dc_opt) / rL2
    assert abs(best - c0) < 1e-6


def test_fp16_roundtrip_bound():
    v = synth.gaussian_spinor((2, 2, 2, 4), 8).reshape(-1, 24)
    h, s = fp16.encode_spinor(v)
    d = fp16.decode_spinor(h, s, v.shape)
    err = np.maximum(np.abs(d.real - v.real), np.abs(d.imag - v.imag))
    assert (err <= 2.0 ** -11 * s[:, None] * (1 + 1e-6)).all()
    U = synth.gauge_field((2, 2, 2, 2), 1)
    du = fp16.decode_links(fp16.encode_links(U))
    assert np.abs(du - U).max() <= 2.0 ** -11


def test_fp16_round_to_nearest_even():
    # 1 + 2^-11 is the midpoint between 1 and 1 + 2^-10: ties go to the even mantissa (1.0)
    assert np.float16(1.0 + 2.0 ** -11) == np.float16(1.0)
    assert np.float16(1.0 + 3 * 2.0 ** -11) == np.float16(1.0 + 2 * 2.0 ** -10)
