"""Pins of the oracle's network and FP16 codec.

* backward against central finite differences of the loss;
* the Gram-form loss equals the directly computed ||b - (Q^2 + s) x||^2 /
  ||r_L||^2 on explicit vectors (appendix B identity r = b + sum c_i w_i);
* L(0) = 1 (Lagrange) and c0 is the least-squares optimum over the span;
* BF16 rounding: ties to even on exact midpoints, representable values kept,
  relative error <= 2^-8, and the BF16 forward equals the FP64 forward on
  weights and inputs that are already bfloat16 with activations that are too;
* Adam (Kingma & Ba 2015): the bias-corrected first step is -lr g/(|g| + eps)
  elementwise (m_hat = g, v_hat = g^2), a constant gradient gives that same step
  at every t, and on a 1-D quadratic far from its minimum each step moves
  towards it by between 0.9 lr and lr;
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
    A = rng.standard_normal((B, mlp.K_MAX, mlp.K_MAX))
    G = np.einsum("bij,bkj->bik", A, A)
    h = rng.standard_normal((B, mlp.K_MAX))
    return F, mask, G, h


def test_backward_finite_differences():
    p = mlp.init_params(1, out_scale=0.3)
    F, mask, G, h = _batch()

    def L(pp):
        y, _ = mlp.forward(pp, F)
        return mlp.loss(y, mask, G, h)[0]

    y, cache = mlp.forward(p, F)
    _, dy, _ = mlp.loss(y, mask, G, h)
    g = mlp.backward(p, cache, dy)
    rng = np.random.default_rng(3)
    for k in p:
        for _ in range(4):
            idx = tuple(rng.integers(0, s) for s in p[k].shape)
            eps = 1e-6
            pp = {kk: vv.copy() for kk, vv in p.items()}
            pp[k][idx] += eps
            lp = L(pp)
            pp[k][idx] -= 2 * eps
            lm = L(pp)
            fd = (lp - lm) / (2 * eps)
            assert abs(fd - g[k][idx]) <= 1e-6 * max(1.0, abs(fd))
    assert mlp.flatten(p).size == mlp.N_PARAM
    q = mlp.unflatten(mlp.flatten(p))
    assert all(np.array_equal(q[k], p[k]) for k in p)


def test_loss_form_matches_direct_residual():
    """1 + 2 hh.y + y.Gh.y = ||b - (Q^2+s)(x_L + tau sum y x)||^2 / ||r_L||^2 (appendix B identity)."""
    dims = (2, 2, 2, 4)
    U = synth.gauge_field(dims, 3, 0.3)
    op = NDOperator(Lattice(dims, U), synth.KAPPA, synth.MUBAR, synth.EPSBAR)
    b = synth.gaussian_spinor(dims, 4)
    nodes = np.array([1.0, 0.2, 0.05, 0.01])
    st = 0.003
    xs = [solvers.cg(lambda v: op.Q_hat2(v, s), b, tol=1e-13)[0] for s in nodes]
    lag = solvers.lagrange_coefficients(nodes, st)
    xL = sum(l * x for l, x in zip(lag, xs))
    rL = b - op.Q_hat2(xL, st)
    M = mlp.gram_of([b] + xs)
    hv = np.array([np.vdot(v, rL) for v in [b] + xs])
    f, mask, G, h, slot, lag2, tau = mlp.sample(M, hv, norm2(rL), nodes, st)
    assert np.allclose(lag2, lag)
    assert abs(tau - np.sqrt(norm2(rL) / norm2(b))) < 1e-15
    rng = np.random.default_rng(5)
    for scale in (0.0, 0.1, 1.0):
        y = scale * rng.standard_normal(mlp.K_MAX) * mask
        x = xL + tau * sum(y[slot[i]] * xs[i] for i in range(len(nodes)))
        direct = norm2(b - op.Q_hat2(x, st)) / norm2(rL)
        form = 1.0 + 2.0 * h @ y + y @ G @ y
        assert abs(form - direct) < 1e-6 * max(1.0, direct)
    # the least-squares optimum is no worse than any other proposal
    Ls, ys = mlp.ls_optimum(G, h, mask)
    assert Ls <= 1.0 + 1e-12
    W = np.stack([(-b + (s - st) * x).reshape(-1) for x, s in zip(xs, nodes)], axis=1)
    dc, *_ = np.linalg.lstsq(W, -rL.reshape(-1), rcond=None)
    assert abs(norm2(rL.reshape(-1) + W @ dc) / norm2(rL) - Ls) < 1e-6


def test_features_slots_and_mask():
    nodes = synth.geometric_shifts(12, 1e-5)[:9]
    rng = np.random.default_rng(2)
    V = [rng.standard_normal(40) + 1j * rng.standard_normal(40) for _ in range(10)]
    M = mlp.gram_of(V)
    f, mask, G, h, slot, lag, tau = mlp.sample(M, np.ones(10, complex), 1e-6, nodes, 8.111e-5)
    assert mask.sum() == 9 and mask[9:].sum() == 0
    assert slot[-1] == 0 and slot[0] == 8  # nearest node in slot 0
    assert f[0 * mlp.N_FEAT_SLOT + 2] == 1.0  # |x_K| / |x_K|
    assert np.allclose(G, G.T)


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


def test_bf16_round():
    # ulp of bfloat16 at 1 is 2^-7: 1 + 2^-8 is a midpoint -> 1 (even), 1 + 3*2^-8 -> 1 + 2^-6 (even)
    assert mlp.bf16_round(1.0 + 2.0 ** -8) == 1.0
    assert mlp.bf16_round(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6
    assert mlp.bf16_round(1.0 + 2.0 ** -8 + 2.0 ** -20) == 1.0 + 2.0 ** -7
    assert mlp.bf16_round(-(1.0 + 3 * 2.0 ** -8)) == -(1.0 + 2.0 ** -6)
    for v in (0.0, 1.0, -2.5, 2.0 ** -30, 3.0 * 2.0 ** 20):
        assert mlp.bf16_round(v) == v
    x = np.random.default_rng(0).standard_normal(10000) * 10.0 ** np.random.default_rng(1).uniform(-5, 5, 10000)
    r = mlp.bf16_round(x)
    assert (np.abs(r - x) <= 2.0 ** -8 * np.abs(x)).all()
    assert np.array_equal(mlp.bf16_round(r), r)


def test_forward_bf16_reduces_to_fp64_on_bf16_values():
    # weights/inputs already bf16 and a single-neuron net whose activations are bf16 exactly
    p = mlp.init_params(2, out_scale=0.5)
    p = {k: mlp.bf16_round(v) for k, v in p.items()}
    F = mlp.bf16_round(np.random.default_rng(3).standard_normal((4, mlp.N_FEAT)))
    y16 = mlp.forward_bf16(p, F)
    y64, (_, h1, h2) = mlp.forward(p, F)
    # the only differences come from rounding h1, h2: bounded by 2^-8 |h| propagated
    bound = 2.0 ** -8 * (np.abs(p["W3"]) @ (np.abs(h2).T + np.abs(p["W2"]) @ np.abs(h1).T)).T
    assert (np.abs(y16 - y64) <= bound + 1e-15).all()


def _adam_params(seed=3):
    rng = np.random.default_rng(seed)
    return {"W": rng.standard_normal((4, 3)), "b": rng.standard_normal(3)}


def test_adam_first_step_is_signed_lr():
    p = _adam_params()
    g = {k: np.random.default_rng(7).standard_normal(v.shape) * 10.0 ** np.arange(v.size).reshape(v.shape) % 5 - 2.5
         for k, v in p.items()}
    lr, eps = 1e-2, 1e-8
    p0 = {k: v.copy() for k, v in p.items()}
    mlp.adam_step(p, g, {}, lr, eps=eps)
    for k in p:
        want = p0[k] - lr * g[k] / (np.abs(g[k]) + eps)
        assert np.abs(p[k] - want).max() < 1e-15
        # magnitude lr in every component whose gradient is not tiny
        big = np.abs(g[k]) > 1e-3
        assert np.allclose(np.abs(p[k] - p0[k])[big], lr, rtol=1e-5)


def test_adam_constant_gradient_same_step_every_t():
    # with bias correction m_hat = g and v_hat = g^2 at every t for a constant g; a wrong
    # correction exponent (t+1, or none) changes the early steps by tens of percent
    p = _adam_params()
    g = {k: np.full(v.shape, -0.3) for k, v in p.items()}
    state, lr = {}, 5e-3
    for t in range(1, 8):
        before = {k: v.copy() for k, v in p.items()}
        mlp.adam_step(p, g, state, lr)
        for k in p:
            step = p[k] - before[k]
            assert np.abs(step - lr * 0.3 / (0.3 + 1e-8)).max() < 1e-15, (t, k)
    assert state["t"] == 7


def test_adam_walks_down_a_quadratic_at_rate_lr():
    # f(w) = (w - 5)^2 / 2 from w = 0: the gradient keeps its sign and changes slowly,
    # so every step moves towards the minimum by a little less than lr (|m_hat| / sqrt(v_hat)
    # <= 1 while |g| shrinks, since v_hat remembers the larger past gradients)
    p = {"w": np.zeros(1)}
    state, lr = {}, 1e-2
    prev = 0.0
    for _ in range(100):
        mlp.adam_step(p, {"w": p["w"] - 5.0}, state, lr)
        step = p["w"][0] - prev
        assert 0.9 * lr < step <= lr * (1 + 1e-12)
        prev = p["w"][0]
