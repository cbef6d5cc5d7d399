"""Helpers for the GPU parity tests (inputs from synth, expected values from the oracle)."""
import numpy as np
import torch

import synth


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(t):
    return t.detach().cpu().numpy()


def rel_err(got, want):
    return float(np.linalg.norm((got - want).ravel()) / np.linalg.norm(want.ravel()))


def site_err(got, want):
    """max over sites of |got - want|_site / max_site |want|_site."""
    g = got.reshape(got.shape[0], -1)
    w = want.reshape(want.shape[0], -1)
    return float(np.abs(g - w).max() / np.abs(w).max())


# Q^2 is local (its value at a site depends on sites at most four hops away), so the
# oracle can recompute it at sampled sites from a box of the lattice: a box^4 piece
# with an even-parity origin (odd sites stay odd), treated as a periodic lattice of
# its own, is exact at the 2^4 sites of its centre, which no path of four hops joins
# to the box's wrap.
def box_fields(U, v_odd, dims, origin, box):
    """Box of the links (box^4, 4, 3, 3) and of an odd-site field, in the box's own layout."""
    T, Z, Y, X = dims
    c = np.meshgrid(*[(o + np.arange(box)) % n for o, n in zip(origin, dims)], indexing="ij")
    s = ((c[0] * Z + c[1]) * Y + c[2]) * X + c[3]
    Ub = U[s.reshape(-1)]
    cb = np.meshgrid(*[np.arange(box)] * 4, indexing="ij")
    odd = ((cb[0] + cb[1] + cb[2] + cb[3]) % 2 == 1).reshape(-1)
    vb = v_odd[(s.reshape(-1)[odd]) >> 1]
    return Ub, vb


def box_centre_mask(box):
    cb = np.meshgrid(*[np.arange(box)] * 4, indexing="ij")
    odd = ((cb[0] + cb[1] + cb[2] + cb[3]) % 2 == 1).reshape(-1)
    inner = np.ones_like(cb[0], dtype=bool)
    for a in cb:
        inner &= (a >= 4) & (a < box - 4)
    return inner.reshape(-1)[odd]




def sampled_residual_check(U, dims, x, b, r_gpu, sigma, origins, box=10):
    """At the centre sites of each box: the oracle's b - (Q^2 + sigma) x against the
    GPU's residual r_gpu (FP64 rounding of b - A x); returns the largest relative
    local residual seen."""
    from oracle.lattice import Lattice, NDOperator
    mask = box_centre_mask(box)
    worst = 0.0
    for o in origins:
        Ub, xb = box_fields(U, x, dims, o, box)
        _, bb = box_fields(U, b, dims, o, box)
        _, rgb = box_fields(U, r_gpu, dims, o, box)
        opb = NDOperator(Lattice((box,) * 4, Ub), synth.KAPPA, synth.MUBAR, synth.EPSBAR)
        rb = (bb - opb.Q_hat2(xb, float(sigma)))[mask]
        assert np.abs(rb - rgb[mask]).max() <= 1e-13 * np.abs(bb[mask]).max()
        worst = max(worst, float(np.linalg.norm(rb) / np.linalg.norm(bb[mask])))
    return worst


def even_origins(dims, n, seed):
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < n:
        o = [int(rng.integers(0, d)) for d in dims]
        if sum(o) % 2 == 0:
            out.append(o)
    return out
