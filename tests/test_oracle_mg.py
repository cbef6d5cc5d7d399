"""Pins of the oracle's multigrid pieces (section 3, eq:g5-t1-compatible,
eq:g5-t1-hermiticity, eq:non-degenerate_coarse).

* P^dag P = I and P P^dag reproduces every test vector on its aggregate;
* Gamma5-compatibility Gamma5 P = P Gamma5_c;
* the structured coarse operator equals the dense Galerkin product
  P_ND^dag D'_+- P_ND (dense matrices built site by site), including the
  odd-site shift term that becomes i m C_o x tau1 on the coarse grid;
* (Gamma5_c x tau1)-hermiticity of the coarse doublet operator;
* Galerkin orthogonality P^dag D (I - P D_c^-1 P^dag D) = 0.
"""
import numpy as np
import pytest

import synth
from oracle import dense, mg
from oracle.lattice import GAMMA5, Lattice, NDOperator

K, MB, EB = synth.KAPPA, synth.MUBAR, synth.EPSBAR


@pytest.fixture(scope="module")
def setup():
    dims = (4, 2, 2, 4)
    block = (2, 2, 2, 2)
    Nv = 4
    U = synth.gauge_field(dims, 31, 0.3)
    lat = Lattice(dims, U)
    tv = synth.gaussian_vectors((Nv, lat.V, 4, 3), 32)
    P = mg.build_prolongator(tv, dims, block)
    agg = mg.aggregate_of_site(dims, block)
    Vc = int(np.prod(mg.coarse_dims(dims, block)))
    return dims, block, Nv, U, lat, tv, P, agg, Vc


def test_orthonormal_and_spans_test_vectors(setup):
    dims, block, Nv, U, lat, tv, P, agg, Vc = setup
    Pd = mg.dense_prolongator(P, agg, Vc)
    assert np.abs(Pd.conj().T @ Pd - np.eye(Pd.shape[1])).max() < 1e-13
    for k in range(Nv):
        v = tv[k].reshape(-1)
        assert np.abs(Pd @ (Pd.conj().T @ v) - v).max() < 1e-12 * np.abs(v).max()


def test_gamma5_compatible(setup):
    dims, block, Nv, U, lat, tv, P, agg, Vc = setup
    g5 = np.kron(GAMMA5, np.eye(3))
    g5c = mg.gamma5_coarse(Nv)
    lhs = np.einsum("ij,xjk->xik", g5, P)
    rhs = P * g5c[None, None, :]
    assert np.abs(lhs - rhs).max() < 1e-14


@pytest.mark.parametrize("m", [0.0, 0.0316])
def test_coarse_operator_is_galerkin_product(setup, m):
    dims, block, Nv, U, lat, tv, P, agg, Vc = setup
    op = NDOperator(lat, K, MB, EB)
    Dc = mg.coarse_wilson_dense(lat, op.a, P, agg, Vc)
    Bo = mg.odd_projector_coarse(lat, P, agg, Vc)
    Dfine = dense.dense_D_ND(dims, U, K, MB, EB, odd_shift=m)
    Pd1 = mg.dense_prolongator(P, agg, Vc)  # single flavour, rows (site, spin, colour)
    V = lat.V
    n2 = 2 * Nv
    # P_ND = P x I_2 in the dense orderings: fine ((s*2+f)*12 + sc), coarse ((X*2+f)*n2 + j)
    Pnd = np.zeros((V * 24, Vc * 2 * n2), dtype=complex)
    for f in range(2):
        rows = (np.arange(V)[:, None] * 24 + f * 12 + np.arange(12)[None, :]).reshape(-1)
        cols = (np.arange(Vc)[:, None] * 2 * n2 + f * n2 + np.arange(n2)[None, :]).reshape(-1)
        Pnd[np.ix_(rows, cols)] = Pd1
    Dc_nd = Pnd.conj().T @ Dfine @ Pnd
    vc = synth.gaussian_vectors((Vc, 2, n2), 77)
    got = mg.coarse_nd_apply(Dc, Bo, vc, Nv, MB, EB, m=m)
    want = (Dc_nd @ vc.reshape(-1)).reshape(Vc, 2, n2)
    assert np.abs(got - want).max() < 1e-12 * np.abs(want).max()


def test_coarse_g5t1_hermiticity(setup):
    dims, block, Nv, U, lat, tv, P, agg, Vc = setup
    op = NDOperator(lat, K, MB, EB)
    Dc = mg.coarse_wilson_dense(lat, op.a, P, agg, Vc)
    Bo = mg.odd_projector_coarse(lat, P, agg, Vc)
    g5c = mg.gamma5_coarse(Nv)
    G = lambda v: (g5c[None, None, :] * v)[:, ::-1, :]
    x = synth.gaussian_vectors((Vc, 2, 2 * Nv), 1)
    y = synth.gaussian_vectors((Vc, 2, 2 * Nv), 2)
    A = lambda v: G(mg.coarse_nd_apply(Dc, Bo, v, Nv, MB, EB))
    lhs = np.vdot(y, A(x))
    rhs = np.vdot(A(y), x)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_galerkin_orthogonality(setup):
    dims, block, Nv, U, lat, tv, P, agg, Vc = setup
    op = NDOperator(lat, K, MB, EB)
    Dc = mg.coarse_wilson_dense(lat, op.a, P, agg, Vc)
    Bo = mg.odd_projector_coarse(lat, P, agg, Vc)
    n2 = 2 * Nv
    # dense coarse doublet matrix from the structured apply
    N = Vc * 2 * n2
    M = np.zeros((N, N), dtype=complex)
    for j in range(N):
        e = np.zeros(N, dtype=complex)
        e[j] = 1
        M[:, j] = mg.coarse_nd_apply(Dc, Bo, e.reshape(Vc, 2, n2), Nv, MB, EB, m=0.02).reshape(-1)
    v = synth.gaussian_spinor(dims, 9, "full")
    D = lambda f: op.D_full(f.reshape(dims + (2, 4, 3)), odd_shift=0.02).reshape(lat.V, 2, 4, 3)
    Dv = D(v)
    ec = np.linalg.solve(M, mg.restrict(P, Dv, agg, Vc).reshape(-1)).reshape(Vc, 2, n2)
    e = v - mg.prolong(P, ec, agg)
    res = mg.restrict(P, D(e), agg, Vc)
    assert np.abs(res).max() < 1e-11 * np.abs(mg.restrict(P, Dv, agg, Vc)).max()
