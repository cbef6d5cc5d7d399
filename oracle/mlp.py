"""FP64 reference of the learned initial-guess proposer.

The paper builds the guess for the next shifted system as a Lagrange
interpolation of the converged solutions, x_L = sum_i l_i(sigma_t) x_i
(section 4.2), and appendix B shows that the residual of any combination of
converged solutions is the same combination of w_i = r_i - b + (sigma_i -
sigma_t) x_i added to b.  The learned form keeps that structure: a small
network proposes a correction to the Lagrange coefficients, c = l + tau * y,
tau = ||r_L|| / ||b||, so the proposal is still a mix of converged solutions
and y is O(1).  With w_i = -b + (sigma_i - sigma_t) x_i (node residuals below
the solver tolerance neglected) the exact relative loss is

    L(y) = ||r_L + W tau y||^2 / ||r_L||^2 = 1 + 2 hh.y + y.Gh.y,
    Gh_ij = Re<w_i, w_j> / ||b||^2,  hh_i = Re<w_i, r_L> / (||r_L|| ||b||),

computed from the Gram matrix of [b, x_1..x_K], the vector r_L = b - (Q^2 +
sigma_t) x_L and its overlaps with b and the x_i.  L = 1 is the Lagrange guess;
the least-squares optimum over the span is 1 - hh.Gh^+.hh.

Network: 3 dense layers, tanh after the first two, width 64:
    h1 = tanh(W1 f + b1), h2 = tanh(W2 h1 + b2), y = W3 h2 + b3, masked to the
    filled slots.  Trained in FP32 with Adam; inference stores weights and
    activations in BF16 with FP32 accumulation.
"""
from __future__ import annotations

import numpy as np

WIDTH = 64
K_MAX = 11
N_FEAT_SLOT = 5
N_FEAT_GLOBAL = 4
N_FEAT = K_MAX * N_FEAT_SLOT + N_FEAT_GLOBAL  # 59
N_PARAM = WIDTH * N_FEAT + WIDTH + WIDTH * WIDTH + WIDTH + K_MAX * WIDTH + K_MAX


def init_params(seed, n_in=N_FEAT, width=WIDTH, n_out=K_MAX, out_scale=1e-3):
    rng = np.random.default_rng(seed)
    W1 = rng.standard_normal((width, n_in)) / np.sqrt(n_in)
    W2 = rng.standard_normal((width, width)) / np.sqrt(width)
    W3 = rng.standard_normal((n_out, width)) * out_scale
    return dict(W1=W1, b1=np.zeros(width), W2=W2, b2=np.zeros(width), W3=W3, b3=np.zeros(n_out))


def forward(p, F):
    """F: (B, n_in) -> y (B, n_out) and the activations needed by backward."""
    z1 = F @ p["W1"].T + p["b1"]
    h1 = np.tanh(z1)
    z2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.tanh(z2)
    y = h2 @ p["W3"].T + p["b3"]
    return y, (F, h1, h2)


def loss(y, mask, G, h):
    """Mean over the batch of 1 + 2 h.(m*y) + (m*y).G.(m*y); returns (loss, dL/dy, per-sample L)."""
    ym = mask * y
    u = h + np.einsum("bij,bj->bi", G, ym)
    L = 1.0 + np.einsum("bi,bi->b", 2.0 * h + np.einsum("bij,bj->bi", G, ym), ym)
    B = y.shape[0]
    dy = mask * (2.0 * u) / B
    return float(L.mean()), dy, L


def backward(p, cache, dy):
    F, h1, h2 = cache
    g = {}
    g["W3"] = dy.T @ h2
    g["b3"] = dy.sum(axis=0)
    dh2 = dy @ p["W3"]
    dz2 = dh2 * (1.0 - h2 * h2)
    g["W2"] = dz2.T @ h1
    g["b2"] = dz2.sum(axis=0)
    dh1 = dz2 @ p["W2"]
    dz1 = dh1 * (1.0 - h1 * h1)
    g["W1"] = dz1.T @ F
    g["b1"] = dz1.sum(axis=0)
    return g


def adam_step(p, g, state, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015) with bias correction; state holds m, v, t."""
    state["t"] = state.get("t", 0) + 1
    t = state["t"]
    for k in p:
        m = state.setdefault("m_" + k, np.zeros_like(p[k]))
        v = state.setdefault("v_" + k, np.zeros_like(p[k]))
        m[:] = beta1 * m + (1 - beta1) * g[k]
        v[:] = beta2 * v + (1 - beta2) * g[k] * g[k]
        mh = m / (1 - beta1 ** t)
        vh = v / (1 - beta2 ** t)
        p[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)
    return p


def bf16_round(x):
    """Round to bfloat16 (8 significant bits, round to nearest, ties to even), returned as float64.

    bfloat16 is the upper half of an IEEE binary32: the value is first rounded to
    binary32, then its low 16 bits are rounded away.
    """
    u = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    low = u & 0xFFFF
    hi = u >> 16
    up = (low > 0x8000) | ((low == 0x8000) & ((hi & 1) == 1))
    hi = hi + up.astype(np.uint64)
    return (hi << 16).astype(np.uint32).view(np.float32).astype(np.float64)


def forward_bf16(p, F):
    """Inference as the BF16 form defines it: weights, inputs and the two hidden
    activations rounded to bfloat16, sums and tanh exact (FP64 here)."""
    q = {k: bf16_round(v) for k, v in p.items()}
    h1 = bf16_round(np.tanh(bf16_round(F) @ q["W1"].T + q["b1"]))
    h2 = bf16_round(np.tanh(h1 @ q["W2"].T + q["b2"]))
    return h2 @ q["W3"].T + q["b3"]


def flatten(p):
    """Parameter dict -> flat vector in the order W1, b1, W2, b2, W3, b3 (row-major)."""
    return np.concatenate([p[k].reshape(-1) for k in ("W1", "b1", "W2", "b2", "W3", "b3")])


def unflatten(v, n_in=N_FEAT, width=WIDTH, n_out=K_MAX):
    shapes = (("W1", (width, n_in)), ("b1", (width,)), ("W2", (width, width)), ("b2", (width,)),
              ("W3", (n_out, width)), ("b3", (n_out,)))
    out, o = {}, 0
    for k, sh in shapes:
        n = int(np.prod(sh))
        out[k] = np.asarray(v[o:o + n], dtype=np.float64).reshape(sh)
        o += n
    return out


# ---- sample preparation: features and loss form for one target shift ----------
#
# Nodes are the converged shifts sigma_1 > ... > sigma_K (K <= K_MAX) with
# solutions x_i; the target is sigma_t < sigma_K.  Slots are filled from the
# nearest node outwards (slot 0 = sigma_K, the last solved), so a slot means the
# same thing for every K.
#
# Per slot j (node i): [log10(sigma_i/sigma_t)/5, l_i/gamma, |x_i|/|x_K|,
#                       log10(max(1 - cos(x_i, x_K), 1e-12))/12, 1]
# Global: [log10(sigma_t)/5, K/K_MAX, log10(gamma), log10(||r_L||/||b||)/10],
# gamma = sum |l_i|.

def sample(M, hv, rL2, nodes, sig_t):
    """Features, mask, Gh, hh (slot order), the slot of each node, l and tau.

    M: Gram of [b, x_1..x_K] (complex, (K+1)^2); hv: [<b, r_L>, <x_1, r_L>, ..]
    (complex, K+1); rL2 = ||r_L||^2.
    """
    from .solvers import lagrange_coefficients

    nodes = np.asarray(nodes, dtype=np.float64)
    K = len(nodes)
    lag = lagrange_coefficients(nodes, sig_t)
    gamma = float(np.abs(lag).sum())
    bb = float(M[0, 0].real)
    tau = np.sqrt(rL2 / bb)
    G = M.real
    nx = np.sqrt(np.maximum(np.diag(G)[1:], 0.0))
    near = K - 1
    f = np.zeros(N_FEAT)
    mask = np.zeros(K_MAX)
    slot = np.zeros(K, dtype=int)
    d = nodes - sig_t
    for i in range(K):
        j = near - i
        slot[i] = j
        cosv = G[1 + i, 1 + near] / (nx[i] * nx[near])
        f[j * N_FEAT_SLOT + 0] = np.log10(nodes[i] / sig_t) / 5.0
        f[j * N_FEAT_SLOT + 1] = lag[i] / gamma
        f[j * N_FEAT_SLOT + 2] = nx[i] / nx[near]
        f[j * N_FEAT_SLOT + 3] = np.log10(max(1.0 - cosv, 1e-12)) / 12.0
        f[j * N_FEAT_SLOT + 4] = 1.0
        mask[j] = 1.0
    g0 = K_MAX * N_FEAT_SLOT
    f[g0 + 0] = np.log10(sig_t) / 5.0
    f[g0 + 1] = K / K_MAX
    f[g0 + 2] = np.log10(gamma)
    f[g0 + 3] = np.log10(tau) / 10.0
    # w_i = -b + d_i x_i
    Gw = np.zeros((K, K))
    hw = np.zeros(K)
    for i in range(K):
        hw[i] = (-hv[0] + d[i] * hv[1 + i]).real
        for j in range(K):
            Gw[i, j] = (M[0, 0] - d[j] * M[0, 1 + j] - d[i] * M[1 + i, 0] + d[i] * d[j] * M[1 + i, 1 + j]).real
    Gs = np.zeros((K_MAX, K_MAX))
    hs = np.zeros(K_MAX)
    Gs[np.ix_(slot, slot)] = Gw / bb
    hs[slot] = hw / np.sqrt(rL2 * bb)
    return f, mask, Gs, hs, slot, lag, tau


def ls_optimum(Gs, hs, mask):
    """Least-squares optimum of the loss over the span: returns (L*, y*)."""
    idx = np.nonzero(mask)[0]
    G = Gs[np.ix_(idx, idx)]
    h = hs[idx]
    y, *_ = np.linalg.lstsq(G, -h, rcond=1e-13)
    yf = np.zeros(K_MAX)
    yf[idx] = y
    return float(1.0 + 2.0 * h @ y + y @ G @ y), yf


def gram_of(vectors):
    """Gram matrix <v_i, v_j> of a list of arrays (complex)."""
    V = [np.asarray(v).reshape(-1) for v in vectors]
    n = len(V)
    M = np.zeros((n, n), dtype=np.complex128)
    for i in range(n):
        for j in range(n):
            M[i, j] = np.vdot(V[i], V[j])
    return M
