"""Smoothers of the multigrid cycle, on the full-lattice operator D'(m) = D_ND +- i m Gamma5 tau1 P_odd.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The cycle's error propagation (eq:error_propagation) applies the smoother M after the
coarse-grid correction, with no pre-smoothing.  Section 3 names the Schwarz alternating
procedure (SAP, Luescher 2003) as M; the library also offers plain minimal-residual (MR)
steps on the whole lattice.  Both start from the coarse correction z and work on the
residual r - D' z.

SAP as written here (the multiplicative Schwarz method on two colours of blocks):

* The lattice is cut into blocks of ``block = (bt, bz, by, bx)`` sites; block (Bt, Bz,
  By, Bx) has colour (Bt + Bz + By + Bx) mod 2.  Every block extent of the block grid
  is even, so neighbouring blocks always differ in colour and the blocks of one colour
  are decoupled.
* One sweep: for colour 0, then colour 1, every block B of that colour solves
  D'_B e_B = s_B, where s = r - D' z is the current residual and D'_B the operator
  restricted to B (hops that leave B dropped), and z += e.  The residual is formed
  again before the next colour.
* The block systems are solved approximately by ``mr_iters`` minimal-residual steps from
  e_B = 0: q = D'_B s_B, w = <q, s_B> / <q, q>, e_B += w s_B, s_B -= w q.
"""
from __future__ import annotations

import numpy as np

from .lattice import NDOperator


def _vdot(a, b):
    """<a, b> = sum conj(a) b over every axis."""
    return np.vdot(a.reshape(-1), b.reshape(-1))


def mr_smooth(op: NDOperator, m, r, z, steps):
    """z after `steps` minimal-residual steps on D'(m) z = r, started from z."""
    z = np.array(z, dtype=np.complex128, copy=True)
    s = r - op.D_full(z, m)
    for _ in range(steps):
        q = op.D_full(s, m)
        qq = _vdot(q, q).real
        if not qq > 0.0:
            break
        w = _vdot(q, s) / qq
        z = z + w * s
        s = s - w * q
    return z


def block_labels(dims, block):
    """(label, colour): the block index of every site (lexicographic over the block grid,
    shape dims) and the colour of every block."""
    T, Z, Y, X = dims
    bt, bz, by, bx = block
    nb = (T // bt, Z // bz, Y // by, X // bx)
    for d, b, n in zip(dims, block, nb):
        if d % b or n % 2:
            raise ValueError("blocks must tile the lattice with an even number per direction")
    t, z, y, x = np.meshgrid(np.arange(T), np.arange(Z), np.arange(Y), np.arange(X), indexing="ij")
    Bt, Bz, By, Bx = t // bt, z // bz, y // by, x // bx
    label = ((Bt * nb[1] + Bz) * nb[2] + By) * nb[3] + Bx
    g = np.meshgrid(*[np.arange(n) for n in nb], indexing="ij")
    colour = (sum(g) % 2).reshape(-1)
    return label, colour


def block_mr(op: NDOperator, m, s, mask, mr_iters):
    """Approximate solution of D'_B e = s_B on the sites where `mask` holds (one block):
    `mr_iters` minimal-residual steps from e = 0, e zero off the block."""
    sel = mask[..., None, None, None]
    r = np.where(sel, s, 0)
    e = np.zeros_like(r)
    for _ in range(mr_iters):
        q = np.where(sel, op.D_full(r, m), 0)
        qq = _vdot(q, q).real
        if not qq > 0.0:
            break
        w = _vdot(q, r) / qq
        e = e + w * r
        r = r - w * q
    return e


def sap_smooth(op: NDOperator, m, r, z, block, sweeps, mr_iters):
    """z after `sweeps` SAP sweeps on D'(m) z = r, started from z (block by block)."""
    label, colour = block_labels(op.lat.dims, block)
    z = np.array(z, dtype=np.complex128, copy=True)
    for _ in range(sweeps):
        for c in (0, 1):
            s = r - op.D_full(z, m)
            for B in np.nonzero(colour == c)[0]:
                z = z + block_mr(op, m, s, label == B, mr_iters)
    return z


def sap_smooth_colour(op: NDOperator, m, r, z, block, sweeps, mr_iters):
    """The same sweeps with all blocks of one colour stepped together: one operator
    application per minimal-residual step, each block with its own step length (the
    blocks of one colour do not couple, so this equals `sap_smooth`)."""
    label, colour = block_labels(op.lat.dims, block)
    nblk = len(colour)
    z = np.array(z, dtype=np.complex128, copy=True)

    def per_block(v):  # sum over the sites of each block, v of shape dims
        return np.bincount(label.reshape(-1), weights=v.reshape(-1).real, minlength=nblk) + \
            1j * np.bincount(label.reshape(-1), weights=v.reshape(-1).imag, minlength=nblk)

    for _ in range(sweeps):
        for c in (0, 1):
            on = (colour[label] == c)
            sel = on[..., None, None, None]
            rr = np.where(sel, r - op.D_full(z, m), 0)
            e = np.zeros_like(rr)
            for _k in range(mr_iters):
                q = np.where(sel, op.D_full(rr, m), 0)
                qs = per_block(np.sum(np.conj(q) * rr, axis=(-3, -2, -1)))
                qq = per_block(np.sum(np.abs(q) ** 2, axis=(-3, -2, -1))).real
                w = np.where(qq > 0, qs / np.where(qq > 0, qq, 1.0), 0.0)
                ws = w[label][..., None, None, None]
                e = e + ws * rr
                rr = rr - ws * q
            z = z + e
    return z
