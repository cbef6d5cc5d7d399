"""GPU parity of the stencil operators against the FP64 oracle (through the C-ABI).

Bar: FP64 applications match to 1e-12 relative (norm-wise and per-site max);
FP32 to 2e-6; FP16 storage (per-site scale, FP32 arithmetic) to 5e-3.
Lattices: 2^4 (neighbours alias), a ragged one (V/2 not a multiple of the
128-site block), the 4^4 config and the 16^3x32 config (several hundred blocks).
Traversal tiles: every operator (all site epilogues) with (z, y) tiles smaller than
the lattice in both directions, so that tile edges, t-marching and the XCD block
order are all exercised element by element.
"""
import numpy as np
import pytest

import synth
from oracle.lattice import Lattice, NDOperator
from tests.gpu_util import dev, host, rel_err, site_err

pytestmark = pytest.mark.gpu

K, MB, EB = synth.KAPPA, synth.MUBAR, synth.EPSBAR
# FP64; FP32; FP16 (2^-11 per component over 8 hops); FP32 fields on FP16 links
TOL = {0: 1e-12, 1: 2e-6, 2: 5e-3, 3: 5e-3}

CASES = [((2, 2, 2, 2), False), ((2, 2, 2, 2), True), ((6, 4, 2, 10), True), ((4, 4, 4, 4), False),
         ((32, 16, 16, 16), False)]


@pytest.fixture(scope="module")
def nd():
    import paper_1805_09584_amd as nd
    return nd


def _setup(nd, dims, ap, seed=11):
    U = synth.gauge_field(dims, seed, 0.3)
    lat = Lattice(dims, U, antiperiodic_t=ap)
    op = NDOperator(lat, K, MB, EB)
    ctx = nd.Context(dims, bc_flags=1 if ap else 0)
    ctx.ndtm_set_gauge(dev(U))
    ctx.ndtm_set_params(K, MB, EB)
    return lat, op, ctx


@pytest.mark.parametrize("dims,ap", CASES)
def test_hop_and_qhat_fp64(nd, dims, ap):
    print(f"case dims={dims} antiperiodic={ap}", flush=True)
    lat, op, ctx = _setup(nd, dims, ap)
    x = synth.gaussian_spinor(dims, 5)
    xd = dev(x)
    got = host(ctx.ndtm_apply(nd.NDTM_OP_HOP_EO, xd))
    want = op.H_eo(x)
    assert rel_err(got, want) < 1e-12 and site_err(got, want) < 1e-12
    got = host(ctx.ndtm_apply(nd.NDTM_OP_HOP_OE, xd))
    want = op.H_oe(x)
    assert rel_err(got, want) < 1e-12 and site_err(got, want) < 1e-12
    got = host(ctx.ndtm_apply(nd.NDTM_OP_QHAT, xd))
    want = op.Q_hat(x)
    assert rel_err(got, want) < 1e-12 and site_err(got, want) < 1e-12
    if True:
        got = host(ctx.ndtm_apply(nd.NDTM_OP_QHAT2, xd, 0.0123))
        want = op.Q_hat2(x, 0.0123)
        assert rel_err(got, want) < 1e-12
        got = host(ctx.ndtm_apply(nd.NDTM_OP_SHAT_SHIFT, xd, -0.0316))
        want = op.S_shift(x, -0.0316)
        assert rel_err(got, want) < 1e-12
        xf = synth.gaussian_spinor(dims, 6, "full")
        got = host(ctx.ndtm_apply(nd.NDTM_OP_DFULL, dev(xf), 0.05))
        want = op.D_full(xf.reshape(dims + (2, 4, 3)), odd_shift=0.05).reshape(xf.shape)
        assert rel_err(got, want) < 1e-12 and site_err(got, want) < 1e-12
    ctx.close()


TILES = [((8, 8, 4, 8), (2, 2), False), ((8, 8, 4, 8), (4, 1), True), ((8, 12, 6, 4), (3, 2), False),
         ((16, 8, 8, 8), (2, 4), True)]


@pytest.mark.parametrize("dims,tile,ap", TILES)
def test_tiled_traversal_every_operator(nd, dims, tile, ap):
    print(f"case tiled dims={dims} tile={tile} antiperiodic={ap}", flush=True)
    lat, op, ctx = _setup(nd, dims, ap, seed=17)
    ctx.ndtm_set_stencil_tile(*tile)
    x = synth.gaussian_spinor(dims, 9)
    xf = synth.gaussian_spinor(dims, 10, "full")
    xd, xfd = dev(x), dev(xf)
    refs = [(nd.NDTM_OP_HOP_EO, xd, 0.0, op.H_eo(x)), (nd.NDTM_OP_HOP_OE, xd, 0.0, op.H_oe(x)),
            (nd.NDTM_OP_QHAT, xd, 0.0, op.Q_hat(x)), (nd.NDTM_OP_QHAT2, xd, 0.031, op.Q_hat2(x, 0.031)),
            (nd.NDTM_OP_SHAT_SHIFT, xd, 0.17, op.S_shift(x, 0.17)),
            (nd.NDTM_OP_DFULL, xfd, -0.09, op.D_full(xf.reshape(dims + (2, 4, 3)), odd_shift=-0.09).reshape(xf.shape))]
    for prec in (0, 1, 2):
        for opc, xin, par, want in refs:
            got = host(ctx.ndtm_apply(opc, xin, par, prec=prec))
            e = rel_err(got, want)
            assert e < TOL[prec], (prec, opc, e)
            if prec == 0:
                assert site_err(got, want) < 1e-12, (opc, site_err(got, want))
    # the same results bit for bit as the whole-plane traversal
    got = host(ctx.ndtm_apply(nd.NDTM_OP_QHAT2, xd, 0.031))
    ctx.ndtm_set_stencil_tile(0, 0)
    assert np.array_equal(got, host(ctx.ndtm_apply(nd.NDTM_OP_QHAT2, xd, 0.031)))
    with pytest.raises(nd.NdtmError):
        ctx.ndtm_set_stencil_tile(dims[1] + 1, 0)
    ctx.close()


@pytest.mark.parametrize("prec", [1, 2, 3])
@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (6, 4, 2, 10)])
def test_low_precision_operators(nd, dims, prec):
    print(f"case dims={dims} prec={prec}", flush=True)
    lat, op, ctx = _setup(nd, dims, False)
    x = synth.gaussian_spinor(dims, 7)
    xd = dev(x)
    for opcode, ref, par in ((nd.NDTM_OP_QHAT, lambda v: op.Q_hat(v), 0.0),
                             (nd.NDTM_OP_SHAT_SHIFT, lambda v: op.S_shift(v, 0.02), 0.02),
                             (nd.NDTM_OP_HOP_EO, lambda v: op.H_eo(v), 0.0)):
        got = host(ctx.ndtm_apply(opcode, xd, par, prec=prec))
        want = ref(x)
        assert rel_err(got, want) < TOL[prec], (opcode, rel_err(got, want))
        if prec == 3:  # the FP16 links are really read (their rounding is visible)
            assert rel_err(got, want) > 1e-6
    xf = synth.gaussian_spinor(dims, 8, "full")
    got = host(ctx.ndtm_apply(nd.NDTM_OP_DFULL, dev(xf), 0.03, prec=prec))
    want = op.D_full(xf.reshape(dims + (2, 4, 3)), odd_shift=0.03).reshape(xf.shape)
    assert rel_err(got, want) < TOL[prec]
    ctx.close()


def test_errors_and_state(nd):
    ctx = nd.Context((4, 4, 4, 4))
    x = dev(synth.gaussian_spinor((4, 4, 4, 4), 1))
    with pytest.raises(nd.NdtmError) as e:
        ctx.ndtm_apply(nd.NDTM_OP_QHAT, x)
    assert e.value.code == -5  # ESTATE before set_gauge
    with pytest.raises(nd.NdtmError):
        ctx.ndtm_set_params(-1.0, MB, EB)
    with pytest.raises(nd.NdtmError):
        ctx.ndtm_set_shifts([0.1, 0.1])
    with pytest.raises(nd.NdtmError):
        nd.Context((3, 4, 4, 4))
    ctx.close()


@pytest.mark.parametrize("prec", [0, 1, 2, 3])
def test_non_su3_links_use_all_rows(nd, prec):
    """Links multiplied by a random U(1) phase per link are unitary but not SU(3):
    their third row is not conj(row 0 x row 1), so the stencil must load all
    three rows.  Parity with the oracle at each precision's bar, and the same
    field without the phases still passes (the two-row path)."""
    print(f"non-SU(3) links prec={prec}", flush=True)
    dims = (4, 4, 4, 4)
    U = synth.gauge_field(dims, 23, 0.3)
    ph = np.exp(1j * np.random.default_rng(3).uniform(-np.pi, np.pi, U.shape[:2]))
    x = synth.gaussian_spinor(dims, 6)
    for links in (U * ph[:, :, None, None], U):
        op = NDOperator(Lattice(dims, links), K, MB, EB)
        ctx = nd.Context(dims)
        ctx.ndtm_set_gauge(dev(links))
        ctx.ndtm_set_params(K, MB, EB)
        got = host(ctx.ndtm_apply(nd.NDTM_OP_QHAT, dev(x), prec=prec))
        want = op.Q_hat(x)
        assert rel_err(got, want) < TOL[prec], (prec, rel_err(got, want))
        ctx.close()


def test_unit_links_and_near_unit_links(nd):
    """The FP64 stencil reads SU(3) links in eight parameters unless some link's first
    row is (u, 0, 0) to rounding (unit links): then it keeps the two-row form.  Both
    paths against the oracle at 1e-12: unit links, and a field whose links are unit
    except for one random SU(3) matrix per direction pattern (first rows far from
    (u, 0, 0) only there)."""
    dims = (4, 4, 2, 6)
    print("unit and near-unit links", flush=True)
    U1 = synth.unit_gauge(dims)
    Ur = synth.gauge_field(dims, 29, 0.3)
    mask = (np.arange(U1.shape[0]) % 3 == 0)
    Um = np.where(mask[:, None, None, None], Ur, U1)
    x = synth.gaussian_spinor(dims, 31)
    for links in (U1, Um, Ur):
        op = NDOperator(Lattice(dims, links), K, MB, EB)
        ctx = nd.Context(dims)
        ctx.ndtm_set_gauge(dev(links))
        ctx.ndtm_set_params(K, MB, EB)
        for opc, ref in ((nd.NDTM_OP_QHAT, op.Q_hat), (nd.NDTM_OP_HOP_EO, op.H_eo)):
            got = host(ctx.ndtm_apply(opc, dev(x)))
            assert rel_err(got, ref(x)) < 1e-12
            assert site_err(got, ref(x)) < 1e-12
        ctx.close()
