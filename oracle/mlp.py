"""FP64 reference of the learned initial-guess proposer.

The paper builds the guess for the next shifted system as a Lagrange
interpolation of the converged solutions, x_t = sum_i l_i(sigma_t) x_i
(section 4.2), and appendix B shows that its residual is the same
combination of w_i = r_i - b + (sigma_i - sigma_t) x_i added to b:
r_t = b + sum_i c_i w_i for any real coefficients c.  The learned form keeps
that structure and lets a small network propose a correction dc to the
Lagrange coefficients, c = l(sigma_t) + dc, so the proposal is still a mix of
converged solutions.

Network: 3 dense layers, tanh after the first two, width 64:
    h1 = tanh(W1 f + b1), h2 = tanh(W2 h1 + b2), y = W3 h2 + b3, dc = mask * y.
Loss per sample (exact, from the Gram matrix of the w_i, relative to the
Lagrange residual r_L = b + W l):
    L(dc) = ||r_L + W dc||^2 / ||r_L||^2 = c0 + ||R dc + q||^2,
with G = W^T W / ||r_L||^2 = V diag(lam) V^T, R = diag(sqrt(lam)) V^T,
q = diag(1/sqrt(lam)) V^T h, h = W^T r_L / ||r_L||^2 (real parts),
c0 = 1 - ||q||^2 (eigen-directions with lam <= 1e-12 lam_max are dropped).
L = 1 at dc = 0 (Lagrange) and c0 is the least-squares optimum over the span.
"""
from __future__ import annotations

import numpy as np

WIDTH = 64
K_MAX = 11
N_FEAT_SLOT = 5
N_FEAT_GLOBAL = 3
N_FEAT = K_MAX * N_FEAT_SLOT + N_FEAT_GLOBAL  # 58


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


def loss(y, mask, R, q, c0):
    """Mean over the batch of c0 + ||R (mask*y) + q||^2; returns (loss, dL/dy)."""
    dc = mask * y
    u = np.einsum("bij,bj->bi", R, dc) + q
    L = c0 + np.einsum("bi,bi->b", u, u)
    B = y.shape[0]
    dy = mask * (2.0 * np.einsum("bij,bi->bj", R, u)) / B
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


def w_gram(M, K, sig_nodes, sig_t):
    """Gram of w_i = r_i - b + (sigma_i - sigma_t) x_i from the Gram M of the vector set
    [b, x_1..x_K, r_1..r_K] (Hermitian, complex).  Returns (Gw (K,K) real, gb (K,) real, bb)."""
    n = 1 + 2 * K
    assert M.shape == (n, n)
    # coefficient matrix expressing w_i in the basis [b, x, r]
    C = np.zeros((K, n))
    for i in range(K):
        C[i, 0] = -1.0
        C[i, 1 + i] = sig_nodes[i] - sig_t
        C[i, 1 + K + i] = 1.0
    Gw = (C @ M @ C.T).real
    gb = (M[0, :] @ C.T).real  # <b, w_i>
    bb = float(M[0, 0].real)
    return Gw, gb, bb


def quad_form(Gw, gb, bb, lag, drop=1e-12):
    """(R, q, c0, rL2) of the loss above from the w-Gram and the Lagrange coefficients."""
    K = len(lag)
    rL2 = bb + 2.0 * gb @ lag + lag @ Gw @ lag
    h = (gb + Gw @ lag) / rL2
    G = Gw / rL2
    lam, Vm = np.linalg.eigh(G)
    keep = lam > drop * max(lam.max(), 0.0)
    R = np.zeros((K, K))
    q = np.zeros(K)
    nk = int(keep.sum())
    R[:nk] = (np.sqrt(lam[keep])[:, None] * Vm[:, keep].T)
    q[:nk] = (Vm[:, keep].T @ h) / np.sqrt(lam[keep])
    c0 = 1.0 - float(q @ q)
    return R, q, c0, rL2
