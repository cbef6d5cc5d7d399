"""ndtm_apply_noalloc (fixed scratch array, no device allocation) against ndtm_apply.

Every operator, FP64, through the C ABI: the same results bit for bit on two
calls in a row, the second on a smaller lattice (another context) whose fields
reuse the same device array; a lattice above the array's size is refused with
NDTM_EINVAL; the call makes no device allocation (the context's count of
hipMalloc calls for lattice storage does not move, and its storage is untouched).
"""
import numpy as np
import pytest
import torch

import synth
from tests.gpu_util import dev, host

pytestmark = pytest.mark.gpu

K, MB, EB = synth.KAPPA, synth.MUBAR, synth.EPSBAR


@pytest.fixture(scope="module")
def nd():
    import paper_1805_09584_amd as nd
    return nd


def _ctx(nd, dims, seed):
    ctx = nd.Context(dims)
    ctx.ndtm_set_gauge(dev(synth.gauge_field(dims, seed, 0.3)))
    ctx.ndtm_set_params(K, MB, EB)
    return ctx


def _check_all_ops(nd, ctx, dims, seed):
    half = dev(synth.gaussian_spinor(dims, seed))
    full = dev(synth.gaussian_spinor(dims, seed + 1, "full"))
    for op, x, param in ((nd.NDTM_OP_QHAT, half, 0.0), (nd.NDTM_OP_QHAT2, half, 0.0123),
                         (nd.NDTM_OP_SHAT_SHIFT, half, 0.21), (nd.NDTM_OP_DFULL, full, -0.17),
                         (nd.NDTM_OP_HOP_EO, half, 0.0), (nd.NDTM_OP_HOP_OE, half, 0.0)):
        print(f"case noalloc dims={dims} op={op}", flush=True)
        before = ctx.ndtm_workspace_stats()
        got = ctx.ndtm_apply_noalloc(op, x, param)
        torch.cuda.synchronize()
        after = ctx.ndtm_workspace_stats()
        assert after["device_allocs"] == before["device_allocs"]
        assert after["live"] == before["live"]
        want = ctx.ndtm_apply(op, x, param)
        g, w = host(got), host(want)
        assert np.array_equal(g, w), (op, np.abs(g - w).max())


def test_noalloc_matches_apply_on_two_lattices_in_a_row(nd):
    big, small = (8, 8, 8, 8), (4, 4, 4, 4)
    a = _ctx(nd, big, 51)
    _check_all_ops(nd, a, big, 61)
    b = _ctx(nd, small, 52)
    _check_all_ops(nd, b, small, 62)
    # and the larger lattice again, after the smaller one has used the array
    _check_all_ops(nd, a, big, 63)
    a.close()
    b.close()


def test_noalloc_refuses_a_lattice_above_its_array(nd):
    dims = (32, 16, 16, 24)  # V/2 = 98304: 4 FP64 half fields exceed 128 MiB
    ctx = nd.Context(dims)
    ctx.ndtm_set_gauge(dev(synth.unit_gauge(dims)))
    ctx.ndtm_set_params(K, MB, EB)
    x = dev(np.zeros((ctx.vh, 2, 4, 3), dtype=complex))
    with pytest.raises(nd.NdtmError) as e:
        ctx.ndtm_apply_noalloc(nd.NDTM_OP_QHAT, x)
    assert e.value.code == -1 and "scratch" in str(e.value)
    assert nd.load_library().ndtm_apply_noalloc_max_bytes() == 128 << 20
    ctx.close()
