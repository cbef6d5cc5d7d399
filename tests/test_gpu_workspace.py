"""Caller-owned device storage (ndtm_workspace_bytes / ndtm_set_workspace).

* The bound of ndtm_workspace_bytes covers what the same calls take from
  hipMalloc (peak live bytes in the library's own accounting), for the FP64
  hybrid with projection guesses, the mixed form and plain multi-shift CG.
* A context given a region of exactly that bound runs the same calls without one
  device allocation and returns the same solutions as the hipMalloc context; every
  shift meets 1e-10 by the oracle's residual.
* A region a quarter of the bound makes a call fail with NDTM_ENOMEM (not a fault),
  and set_workspace after set_gauge is refused with NDTM_ESTATE.
"""
import numpy as np
import pytest
import torch

import synth
from oracle.lattice import Lattice, NDOperator, rel_residual
from tests.gpu_util import dev, host

pytestmark = pytest.mark.gpu

K, MB, EB = synth.KAPPA, synth.MUBAR, synth.EPSBAR
DIMS = (8, 4, 4, 8)


@pytest.fixture(scope="module")
def nd():
    import paper_1805_09584_amd as nd
    return nd


@pytest.fixture(scope="module")
def inputs():
    U = synth.gauge_field(DIMS, 41, 0.3)
    b = synth.gaussian_spinor(DIMS, 42)
    shifts = list(synth.geometric_shifts(8, 1e-4))
    op = NDOperator(Lattice(DIMS, U), K, MB, EB)
    return U, b, shifts, op


FORMS = {
    "hybrid_projection": dict(n_mmscg=5, guess=3, mms_predict=1, use_graphs=0),
    "mixed": dict(n_mmscg=5, guess=1, precision=2, use_graphs=0),
    "plain": dict(),
}


def _run(nd, inputs, form, region=None):
    U, b, shifts, op = inputs
    ctx = nd.Context(DIMS)
    if region is not None:
        ctx.ndtm_set_workspace(region)
    ctx.ndtm_set_gauge(dev(U))
    ctx.ndtm_set_params(K, MB, EB)
    ctx.ndtm_set_shifts(shifts)
    x = dev(b)
    for prec in (0, 1, 2):
        for opc in (0, 1, 2, 4, 5):
            ctx.ndtm_apply(opc, x, 0.3, prec=prec)
        ctx.ndtm_apply(3, dev(synth.gaussian_spinor(DIMS, 5, "full")), 0.3, prec=prec)
    mgp = ctx.mg_params(block=(2, 2, 2, 2), n_vec=8)
    sp = ctx.solve_params(**FORMS[form])
    if form != "plain":
        ctx.ndtm_mg_setup(mgp)
    xs, rep = ctx.ndtm_solve(x, sp)
    torch.cuda.synchronize()
    out = [host(v) for v in xs]
    stats = ctx.ndtm_workspace_stats()
    bound = ctx.ndtm_workspace_bytes(len(shifts), mgp if form != "plain" else None, sp)
    ctx.close()
    return out, rep, stats, bound


@pytest.mark.parametrize("form", list(FORMS))
def test_bound_covers_managed_peak_and_region_runs_without_allocation(nd, inputs, form):
    print(f"case workspace form={form}", flush=True)
    U, b, shifts, op = inputs
    xs0, rep0, st0, bound = _run(nd, inputs, form)
    assert st0["device_allocs"] > 0
    assert st0["peak"] <= bound, (st0, bound)
    region = torch.empty(bound, dtype=torch.uint8, device="cuda")
    xs1, rep1, st1, bound1 = _run(nd, inputs, form, region)
    assert bound1 == bound
    assert st1["device_allocs"] == 0
    assert st1["peak"] <= bound
    assert rep1["mms_iterations"] == rep0["mms_iterations"]
    for x0, x1, s in zip(xs0, xs1, shifts):
        assert np.array_equal(x0, x1)
        assert rel_residual(op, x1, b, s) <= 1e-10


def test_small_region_reports_enomem_and_late_region_is_refused(nd, inputs):
    U, b, shifts, op = inputs
    ctx = nd.Context(DIMS)
    mgp = ctx.mg_params(block=(2, 2, 2, 2), n_vec=8)
    sp = ctx.solve_params(**FORMS["hybrid_projection"])
    bound = ctx.ndtm_workspace_bytes(len(shifts), mgp, sp)
    region = torch.empty(bound // 4, dtype=torch.uint8, device="cuda")
    ctx.ndtm_set_workspace(region)
    with pytest.raises(nd.NdtmError) as e:
        ctx.ndtm_set_gauge(dev(U))
        ctx.ndtm_set_params(K, MB, EB)
        ctx.ndtm_set_shifts(shifts)
        ctx.ndtm_mg_setup(mgp)
        ctx.ndtm_solve(dev(b), sp)
    assert e.value.code == -2  # NDTM_ENOMEM
    assert ctx.ndtm_workspace_stats()["device_allocs"] == 0
    ctx.close()
    ctx = nd.Context(DIMS)
    ctx.ndtm_set_gauge(dev(U))
    with pytest.raises(nd.NdtmError) as e:
        ctx.ndtm_set_workspace(torch.empty(bound, dtype=torch.uint8, device="cuda"))
    assert e.value.code == -5  # NDTM_ESTATE
    ctx.close()
