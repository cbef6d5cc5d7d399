"""Pins of the oracle's smoothers (oracle/smoothers.py) against dense linear algebra.

* Block solves: minimal-residual steps on one block converge to the solution of the
  block-restricted dense system D'_BB e = s_B (rows and columns of the dense D' on the
  block's sites, built site by site in oracle/dense.py), and e vanishes off the block.
* SAP with exact block solves is the multiplicative Schwarz method: one sweep equals
  z1 = z0 + M_0 (r - D' z0), z2 = z1 + M_1 (r - D' z1) with M_c the sum over the blocks B of
  colour c of I_B D'_BB^-1 I_B^T, assembled from dense inverses; after it the residual
  vanishes on the colour-1 blocks (the last solved).
* The colour-at-once form equals the block-by-block form to rounding, for few MR steps.
* Minimal-residual steps: each step's residual equals the closed form
  |s|^2 - |<q, s>|^2 / |q|^2.
"""
import numpy as np
import pytest

import synth
from oracle import dense
from oracle import smoothers as sm
from oracle.lattice import Lattice, NDOperator

K, MB, EB = synth.KAPPA, synth.MUBAR, synth.EPSBAR


def _setup(dims, seed=5, m=0.07):
    U = synth.gauge_field(dims, seed, 0.3)
    lat = Lattice(dims, U)
    op = NDOperator(lat, K, MB, EB)
    D = dense.dense_D_ND(dims, U, K, MB, EB, odd_shift=m)
    return op, D, m


def _block_index(dims, block, B):
    label, _ = sm.block_labels(dims, block)
    sites = np.nonzero(label.reshape(-1) == B)[0]
    return (sites[:, None] * 24 + np.arange(24)[None, :]).reshape(-1), label


def test_block_labels_colouring():
    dims, block = (4, 4, 2, 2), (2, 2, 1, 1)
    label, colour = sm.block_labels(dims, block)
    assert label.shape == dims and len(colour) == 16
    # every hop between different blocks joins opposite colours
    for mu in range(4):
        nb = np.roll(label, -1, axis=mu)
        diff = nb != label
        assert np.all(colour[label[diff]] != colour[nb[diff]])
    with pytest.raises(ValueError):
        sm.block_labels((4, 4, 2, 2), (4, 2, 1, 1))  # one block in t


@pytest.mark.parametrize("dims,block", [((4, 4, 2, 2), (2, 2, 1, 1)), ((4, 4, 4, 2), (2, 2, 2, 1))])
def test_block_mr_converges_to_dense_block_solve(dims, block):
    op, D, m = _setup(dims)
    s = synth.gaussian_vectors(dims + (2, 4, 3), 11)
    for B in (0, 3):
        idx, label = _block_index(dims, block, B)
        e = sm.block_mr(op, m, s, label == B, 120)
        ref = np.linalg.solve(D[np.ix_(idx, idx)], s.reshape(-1)[idx])
        flat = e.reshape(-1)
        assert np.max(np.abs(flat[idx] - ref)) <= 1e-10 * np.max(np.abs(ref))
        off = np.ones(flat.size, bool)
        off[idx] = False
        assert np.all(flat[off] == 0)


def test_sap_exact_blocks_is_multiplicative_schwarz():
    dims, block = (4, 4, 2, 2), (2, 2, 1, 1)
    op, D, m = _setup(dims)
    r = synth.gaussian_vectors(dims + (2, 4, 3), 12)
    z0 = synth.gaussian_vectors(dims + (2, 4, 3), 13)
    label, colour = sm.block_labels(dims, block)
    n = D.shape[0]
    Mc = [np.zeros((n, n), complex), np.zeros((n, n), complex)]
    for B in range(len(colour)):
        idx, _ = _block_index(dims, block, B)
        Mc[colour[B]][np.ix_(idx, idx)] = np.linalg.inv(D[np.ix_(idx, idx)])
    rv, z = r.reshape(-1), z0.reshape(-1)
    for c in (0, 1):
        z = z + Mc[c] @ (rv - D @ z)
    got = sm.sap_smooth(op, m, r, z0, block, 1, 120).reshape(-1)
    assert np.max(np.abs(got - z)) <= 1e-9 * np.max(np.abs(z))
    res = rv - D @ got
    on1 = np.repeat(colour[label.reshape(-1)] == 1, 24)
    assert np.max(np.abs(res[on1])) <= 1e-9 * np.max(np.abs(rv))
    assert np.max(np.abs(res[~on1])) > 1e-3 * np.max(np.abs(rv))


@pytest.mark.parametrize("sweeps,mr", [(1, 1), (2, 3), (2, 4)])
def test_sap_colour_form_equals_block_form(sweeps, mr):
    dims, block = (4, 4, 4, 2), (2, 2, 2, 1)
    op, _, m = _setup(dims, seed=8, m=-0.04)
    r = synth.gaussian_vectors(dims + (2, 4, 3), 21)
    z0 = synth.gaussian_vectors(dims + (2, 4, 3), 22)
    a = sm.sap_smooth(op, m, r, z0, block, sweeps, mr)
    b = sm.sap_smooth_colour(op, m, r, z0, block, sweeps, mr)
    assert np.max(np.abs(a - b)) <= 1e-13 * np.max(np.abs(a))


def test_mr_steps_closed_form():
    dims = (4, 4, 2, 2)
    op, D, m = _setup(dims)
    r = synth.gaussian_vectors(dims + (2, 4, 3), 31)
    z = np.zeros_like(r)
    s = r.reshape(-1).copy()
    for k in range(1, 6):
        q = D @ s
        expect = np.vdot(s, s).real - abs(np.vdot(q, s)) ** 2 / np.vdot(q, q).real
        zk = sm.mr_smooth(op, m, r, z, k)
        s = r.reshape(-1) - D @ zk.reshape(-1)
        assert abs(np.vdot(s, s).real - expect) <= 1e-10 * expect


def test_two_grid_coarse_correction_is_galerkin_projection():
    """With no smoothing the cycle's output z satisfies (P x I2)^dag (r - D'z) = 0 (the coarse
    operator is the Galerkin product of D' including the odd-site shift), and applying the
    coarse correction to the new residual changes nothing (a projection)."""
    from oracle import mg as omg
    dims, block, Nv = (4, 4, 2, 2), (2, 2, 1, 1), 4
    U = synth.gauge_field(dims, 9, 0.3)
    op = NDOperator(Lattice(dims, U), K, MB, EB)
    V = int(np.prod(dims))
    tv = synth.gaussian_vectors((Nv, V, 4, 3), 41)
    P = omg.build_prolongator(tv, dims, block)
    agg = omg.aggregate_of_site(dims, block)
    Vc = int(np.prod(omg.coarse_dims(dims, block)))
    m = 0.06
    r = synth.gaussian_vectors(dims + (2, 4, 3), 42)
    z = omg.two_grid_cycle(op, m, r, P, agg, Vc)
    res = r - op.D_full(z, m)
    rc = omg.restrict(P, res.reshape(V, 2, 4, 3), agg, Vc)
    assert np.max(np.abs(rc)) <= 1e-12 * np.max(np.abs(r))
    z2 = omg.two_grid_cycle(op, m, res, P, agg, Vc)
    assert np.max(np.abs(z2)) <= 1e-12 * np.max(np.abs(z))
    # with post-smoothing the output is the smoother started from the coarse correction
    zs = omg.two_grid_cycle(op, m, r, P, agg, Vc, smoother="sap", steps=1, block=block, mr_iters=2)
    assert np.max(np.abs(zs - sm.sap_smooth(op, m, r, z, block, 1, 2))) <= 1e-13 * np.max(np.abs(zs))
