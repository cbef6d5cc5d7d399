"""Multigrid cycle in its FP16-storage form (mg precision NDTM_PREC_F16) against the
FP64 oracle.

* Transfers as the cycle runs them (ndtm_mg_transfer_cycle), with P from the same
  seeded test vectors as the oracle's: the FP32 cycle within FP32 rounding (2e-6); the
  FP16 cycle, whose P entries are rounded to 11 bits relative to the largest entry of
  their site, within 3e-3 and visibly above FP32 rounding (the FP16 copy is what is read).
* Hybrid solve on the 16^3x32 configuration without predicted guesses, so that the
  multigrid runs: every shift's true residual (oracle) <= 1e-10 with the FP16 cycle, and
  its outer iteration counts stay within 25% (+2) of the FP32 cycle's.
"""
import numpy as np
import pytest

import synth
from oracle import mg as omg
from oracle.lattice import Lattice, NDOperator, rel_residual
from tests.gpu_util import dev, host, rel_err

pytestmark = pytest.mark.gpu

K, MB, EB = synth.KAPPA, synth.MUBAR, synth.EPSBAR


@pytest.fixture(scope="module")
def nd():
    import paper_1805_09584_amd as nd
    return nd


@pytest.mark.parametrize("prec", [1, 2])
def test_cycle_transfers(nd, prec):
    dims, block, Nv = (8, 8, 8, 8), (4, 4, 4, 4), 8
    print(f"case cycle transfers prec={prec}", flush=True)
    U = synth.gauge_field(dims, 31, 0.3)
    tv = synth.gaussian_vectors((Nv, int(np.prod(dims)), 4, 3), 32)
    ctx = nd.Context(dims)
    ctx.ndtm_set_gauge(dev(U))
    ctx.ndtm_set_params(K, MB, EB)
    ctx.ndtm_mg_setup(ctx.mg_params(block=block, n_vec=Nv, precision=prec, keep_f64=0), test_vectors=dev(tv))
    P = omg.build_prolongator(tv, dims, block)
    agg = omg.aggregate_of_site(dims, block)
    Vc = int(np.prod(omg.coarse_dims(dims, block)))
    v = synth.gaussian_spinor(dims, 3, "full")
    vc = synth.gaussian_vectors((Vc, 2, 2 * Nv), 4)
    e_r = rel_err(host(ctx.ndtm_mg_transfer_cycle(0, dev(v))), omg.restrict(P, v, agg, Vc))
    e_p = rel_err(host(ctx.ndtm_mg_transfer_cycle(1, dev(vc))), omg.prolong(P, vc, agg))
    print(f"restrict {e_r:.2e} prolong {e_p:.2e}", flush=True)
    if prec == 1:
        assert e_r < 2e-6 and e_p < 2e-6
    else:
        assert 1e-6 < e_r < 3e-3 and 1e-6 < e_p < 3e-3
    ctx.close()


def _hybrid(nd, prec):
    c = synth.CONFIGS["c2"]
    dims = c["dims"]
    U = synth.gauge_field(dims, c["gauge_seed"], c["amp"])
    b = synth.gaussian_spinor(dims, c["rhs_seed"])
    ctx = nd.Context(dims)
    ctx.ndtm_set_gauge(dev(U))
    ctx.ndtm_set_params(K, MB, EB)
    ctx.ndtm_set_shifts(list(c["shifts"]))
    ctx.ndtm_mg_setup(ctx.mg_params(precision=prec))
    xs, rep = ctx.ndtm_solve(dev(b), ctx.solve_params(n_mmscg=9, guess=1, mms_predict=0))
    out = [host(x) for x in xs]
    ctx.close()
    return U, b, c, out, rep


def test_hybrid_fp16_cycle_config2(nd):
    print("case c2 hybrid, FP32 and FP16 cycles", flush=True)
    _, _, _, _, rep32 = _hybrid(nd, 1)
    U, b, c, xs, rep16 = _hybrid(nd, 2)
    print("FP32 cycle", rep32["iterations"][9:], rep32["t_mg_ms"], "FP16 cycle", rep16["iterations"][9:],
          rep16["t_mg_ms"], flush=True)
    op = NDOperator(Lattice(c["dims"], U), K, MB, EB)
    for i, s in enumerate(c["shifts"]):
        assert rel_residual(op, xs[i], b, s) <= 1e-10, i
    for i in range(9, 12):
        assert rep16["method"][i] == 1, rep16["method"]
        assert rep16["iterations"][i] <= 1.25 * rep32["iterations"][i] + 2, (rep16["iterations"], rep32["iterations"])


def test_fp32_setup_config2(nd):
    """The inverse iteration's CG in FP32 (setup_prec F32): every shift still meets the
    tolerance by the oracle's residual, and the multigrid's outer iteration counts stay
    within 25% (+2) of those with the FP64 setup."""
    print("case c2 hybrid, FP32 and FP64 setup", flush=True)
    c = synth.CONFIGS["c2"]
    dims = c["dims"]
    U = synth.gauge_field(dims, c["gauge_seed"], c["amp"])
    b = synth.gaussian_spinor(dims, c["rhs_seed"])
    reps, outs = [], []
    for sp in (0, 1):
        ctx = nd.Context(dims)
        ctx.ndtm_set_gauge(dev(U))
        ctx.ndtm_set_params(K, MB, EB)
        ctx.ndtm_set_shifts(list(c["shifts"]))
        ctx.ndtm_mg_setup(ctx.mg_params(precision=2, setup_prec=sp))
        xs, rep = ctx.ndtm_solve(dev(b), ctx.solve_params(n_mmscg=9, guess=1, mms_predict=0))
        outs.append([host(x) for x in xs])
        reps.append(rep)
        ctx.close()
    print("FP64 setup", reps[0]["iterations"][9:], "FP32 setup", reps[1]["iterations"][9:], flush=True)
    op = NDOperator(Lattice(dims, U), K, MB, EB)
    for i, s in enumerate(c["shifts"]):
        assert rel_residual(op, outs[1][i], b, s) <= 1e-10, i
    for i in range(9, 12):
        assert reps[1]["method"][i] == 1, reps[1]["method"]
        assert reps[1]["iterations"][i] <= 1.25 * reps[0]["iterations"][i] + 2, (reps[1]["iterations"], reps[0]["iterations"])
