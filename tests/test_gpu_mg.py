"""GPU multigrid against the FP64 oracle.

* With the same seeded test vectors on both sides, the GPU's restriction,
  prolongation and coarse doublet operator match the oracle's (P is the unique
  positive-diagonal QR factor per aggregate and chirality) to 1e-12, on a
  lattice with coarse extents 1 and 2 (periodic self-neighbours) and on 8^4.
* At the 16^3x32 shape (4^4 aggregates, 24 vectors, 512 coarse sites): the
  Galerkin identity D'_c x_c = P^+ D' P x_c (oracle's D' between the GPU's own
  prolongation and restriction is not used: both sides come from the oracle's P)
  is checked on a random coarse vector, plus P^+ P = I through restrict(prolong(x)) = x.
* Hybrid solves (multi-shift CG for the larger shifts, multigrid case C for the
  smallest): every shift's true residual, recomputed by the oracle, <= 1e-10.
"""
import numpy as np
import pytest

import synth
from oracle import mg as omg
from oracle import solvers
from oracle.lattice import Lattice, NDOperator, norm2, rel_residual
from tests.gpu_util import dev, host, rel_err

pytestmark = pytest.mark.gpu

K, MB, EB = synth.KAPPA, synth.MUBAR, synth.EPSBAR


@pytest.fixture(scope="module")
def nd():
    import paper_1805_09584_amd as nd
    return nd


def _setup(nd, dims, block, Nv, seed=31):
    U = synth.gauge_field(dims, seed, 0.3)
    lat = Lattice(dims, U)
    op = NDOperator(lat, K, MB, EB)
    tv = synth.gaussian_vectors((Nv, lat.V, 4, 3), seed + 1)
    ctx = nd.Context(dims)
    ctx.ndtm_set_gauge(dev(U))
    ctx.ndtm_set_params(K, MB, EB)
    ctx.ndtm_mg_setup(ctx.mg_params(block=block, n_vec=Nv, precision=0), test_vectors=dev(tv))
    P = omg.build_prolongator(tv, dims, block)
    agg = omg.aggregate_of_site(dims, block)
    Vc = int(np.prod(omg.coarse_dims(dims, block)))
    return lat, op, ctx, P, agg, Vc


@pytest.mark.parametrize("dims,block,Nv", [((4, 2, 2, 4), (2, 2, 2, 2), 4), ((8, 8, 8, 8), (4, 4, 4, 4), 8)])
def test_restrict_prolong_coarse_parity(nd, dims, block, Nv):
    print(f"case dims={dims} block={block} Nv={Nv}", flush=True)
    lat, op, ctx, P, agg, Vc = _setup(nd, dims, block, Nv)
    assert ctx.Vc == Vc
    v = synth.gaussian_spinor(dims, 3, "full")
    got = host(ctx.ndtm_mg_restrict(dev(v)))
    want = omg.restrict(P, v, agg, Vc)
    assert rel_err(got, want) < 1e-12
    vc = synth.gaussian_vectors((Vc, 2, 2 * Nv), 4)
    got = host(ctx.ndtm_mg_prolong(dev(vc)))
    want = omg.prolong(P, vc, agg)
    assert rel_err(got, want) < 1e-12
    Bo = omg.odd_projector_coarse(lat, P, agg, Vc)
    if Vc * 2 * Nv <= 512:
        Dc = omg.coarse_wilson_dense(lat, op.a, P, agg, Vc)
        for m in (0.0, 0.0316):
            got = host(ctx.ndtm_mg_coarse_apply(dev(vc), m))
            want = omg.coarse_nd_apply(Dc, Bo, vc, Nv, MB, EB, m=m)
            assert rel_err(got, want) < 1e-12, m
    for m in (0.0, -0.05):
        # Galerkin identity through the oracle's own operators
        got = host(ctx.ndtm_mg_coarse_apply(dev(vc), m))
        f = omg.prolong(P, vc, agg).reshape(dims + (2, 4, 3))
        want = omg.restrict(P, op.D_full(f, odd_shift=m).reshape(lat.V, 2, 4, 3), agg, Vc)
        assert rel_err(got, want) < 1e-12, m
    ctx.close()


def test_galerkin_identity_config2_shape(nd):
    dims, block, Nv = (32, 16, 16, 16), (4, 4, 4, 4), 24
    print("case c2 shape Galerkin", flush=True)
    lat, op, ctx, P, agg, Vc = _setup(nd, dims, block, Nv, seed=12)
    vc = synth.gaussian_vectors((Vc, 2, 2 * Nv), 5)
    # restrict(prolong(x)) = x since P^+ P = I
    back = host(ctx.ndtm_mg_restrict(ctx.ndtm_mg_prolong(dev(vc))))
    assert rel_err(back, vc) < 1e-12
    m = np.sqrt(8.111e-5)
    got = host(ctx.ndtm_mg_coarse_apply(dev(vc), m))
    f = omg.prolong(P, vc, agg).reshape(dims + (2, 4, 3))
    want = omg.restrict(P, op.D_full(f, odd_shift=m).reshape(lat.V, 2, 4, 3), agg, Vc)
    assert rel_err(got, want) < 1e-12
    ctx.close()


def _hybrid(nd, cfg, n_mms, mgp, guess=1, tol=1e-10, amp=None, predict=0):
    c = synth.CONFIGS[cfg]
    dims = c["dims"]
    U = synth.gauge_field(dims, c["gauge_seed"], amp if amp else c["amp"])
    b = synth.gaussian_spinor(dims, c["rhs_seed"])
    ctx = nd.Context(dims)
    ctx.ndtm_set_gauge(dev(U))
    ctx.ndtm_set_params(K, MB, EB)
    ctx.ndtm_set_shifts(list(c["shifts"]))
    ctx.ndtm_mg_setup(ctx.mg_params(**mgp))
    xs, rep = ctx.ndtm_solve(dev(b), ctx.solve_params(tol=tol, n_mmscg=n_mms, guess=guess, mms_predict=predict))
    op = NDOperator(Lattice(dims, U), K, MB, EB)
    return ctx, op, b, c["shifts"], xs, rep


def test_hybrid_config1(nd):
    print("case c1 hybrid", flush=True)
    ctx, op, b, sig, xs, rep = _hybrid(nd, "c1", 7, dict(block=(2, 2, 2, 2), n_vec=8))
    print("report", rep, flush=True)
    for i, s in enumerate(sig):
        r = rel_residual(op, host(xs[i]), b, s)
        assert r <= 1e-10, (i, s, r)
    assert rep["method"] == [0] * 7 + [1] * 3
    ctx.close()


def test_hybrid_config2(nd):
    print("case c2 hybrid", flush=True)
    ctx, op, b, sig, xs, rep = _hybrid(nd, "c2", 9, dict())
    print("report", {k: rep[k] for k in ("iterations", "rounds", "true_res", "guess_res", "t_mms_ms", "t_mg_ms")},
          flush=True)
    for i in range(12):
        r = rel_residual(op, host(xs[i]), b, sig[i])
        assert r <= 1e-10, (i, r)
        # the three smallest shifts are the multigrid's (case C), none fell back to CG
        assert rep["method"][i] == (1 if i >= 9 else 0), rep["method"]
    ctx.close()


def test_paired_signs_config2(nd):
    """Case C with the two signs in lock-step, each paired cycle solving its two coarse
    systems by the batched matrix-core coarse solve: every shift meets 1e-10 by the
    oracle's residual, the multigrid shifts by multigrid (no CG fallback)."""
    print("case c2 hybrid, paired signs", flush=True)
    _, _, _, _, _, rep1 = _hybrid(nd, "c2", 9, dict(pair_signs=0))
    ctx, op, b, sig, xs, rep = _hybrid(nd, "c2", 9, dict(pair_signs=1))
    print("unpaired", rep1["iterations"][9:], rep1["t_mg_ms"], "paired", rep["iterations"][9:], rep["t_mg_ms"],
          flush=True)
    for i in range(12):
        assert rel_residual(op, host(xs[i]), b, sig[i]) <= 1e-10, i
        assert rep["method"][i] == (1 if i >= 9 else 0), rep["method"]
    ctx.close()


def test_graph_replay_matches_eager(nd):
    """The multigrid cycle replayed from captured HIP graphs (many replays, with
    eager FGMRES work between them) gives bitwise the same solutions as eager launches."""
    print("case c2 graphs vs eager", flush=True)
    c = synth.CONFIGS["c2"]
    dims = c["dims"]
    U = synth.gauge_field(dims, c["gauge_seed"], c["amp"])
    b = dev(synth.gaussian_spinor(dims, c["rhs_seed"]))
    ctx = nd.Context(dims)
    ctx.ndtm_set_gauge(dev(U))
    ctx.ndtm_set_params(K, MB, EB)
    ctx.ndtm_set_shifts(list(c["shifts"]))
    ctx.ndtm_mg_setup(ctx.mg_params())
    out = []
    for g in (0, 1, 1):
        xs, rep = ctx.ndtm_solve(b, ctx.solve_params(n_mmscg=9, guess=0, use_graphs=g, mms_predict=0))
        out.append(([host(x) for x in xs[9:]], rep["iterations"][9:]))
    for k in (1, 2):
        assert out[k][1] == out[0][1]
        for a, e in zip(out[k][0], out[0][0]):
            assert np.array_equal(a, e)
    ctx.close()


def test_projection_guess_config1(nd):
    """Minimal-residual guess over the converged solutions: every shift converges
    (oracle residual), the guess is no worse than Lagrange, and its residual
    matches the oracle's own optimum over the span of the oracle's solutions
    where that optimum lies well above the node residuals."""
    print("case c1 hybrid, projection guess", flush=True)
    ctx, op, b, sig, xs, rep = _hybrid(nd, "c1", 7, dict(block=(2, 2, 2, 2), n_vec=8), guess=3)
    print("report", {k: rep[k] for k in ("iterations", "guess_res", "lagrange_res", "guess_kind")}, flush=True)
    for i, s in enumerate(sig):
        assert rel_residual(op, host(xs[i]), b, s) <= 1e-10, (i, s)
    xo = [solvers.cg(lambda v, s=s: op.Q_hat2(v, s), b, tol=1e-13)[0] for s in sig]
    bn = np.sqrt(norm2(b))
    for t in range(7, 10):
        assert rep["guess_kind"][t] == 3
        assert rep["guess_res"][t] <= rep["lagrange_res"][t] * (1 + 1e-9)
        x, _ = solvers.projection_guess(lambda v: op.Q_hat2(v, sig[t]), xo[:t], b)
        ro = np.sqrt(norm2(b - op.Q_hat2(x, sig[t]))) / bn
        print("t", t, "gpu", rep["guess_res"][t], "oracle optimum", ro, flush=True)
        if ro > 1e-8:
            # well above the node residuals: both reach the same optimum
            assert abs(rep["guess_res"][t] - ro) <= 0.05 * ro
        else:
            # near the floor set by the node residuals (<= 1e-10 each, amplified by
            # the coefficients of the nearly collinear solutions) only the scale agrees
            assert rep["guess_res"][t] <= 1e-8
    ctx.close()


def test_multigrid_failure_falls_back_to_cg(nd):
    """A multigrid shift that cannot reach the tolerance (FGMRES capped at 2
    iterations, one round) is finished by FP64 CG: every shift still converges
    (oracle residual) and the report says method 2."""
    print("case c1 hybrid, multigrid capped", flush=True)
    c = synth.CONFIGS["c1"]
    dims = c["dims"]
    U = synth.gauge_field(dims, c["gauge_seed"], c["amp"])
    b = synth.gaussian_spinor(dims, c["rhs_seed"])
    ctx = nd.Context(dims)
    ctx.ndtm_set_gauge(dev(U))
    ctx.ndtm_set_params(K, MB, EB)
    ctx.ndtm_set_shifts(list(c["shifts"]))
    ctx.ndtm_mg_setup(ctx.mg_params(block=(2, 2, 2, 2), n_vec=8))
    xs, rep = ctx.ndtm_solve(dev(b), ctx.solve_params(n_mmscg=7, guess=1, fgmres_maxiter=2, max_rounds=1,
                                                      mms_predict=0))
    print("report", {k: rep[k] for k in ("method", "iterations", "true_res")}, flush=True)
    op = NDOperator(Lattice(dims, U), K, MB, EB)
    assert rep["method"][7:] == [2, 2, 2]
    for i, s in enumerate(c["shifts"]):
        assert rel_residual(op, host(xs[i]), b, s) <= 1e-10, (i, s)
    ctx.close()


def test_predicted_guesses_config1(nd):
    """Shifts n+1, n+2 ride along in the multi-shift CG (section 4.2, guesses via
    MMS-CG): the multi-shift iteration count is that of the n shifts alone (the
    passengers are not waited for), every shift converges (oracle residual), and a
    passenger whose iterate already met the tolerance is returned as it is: within
    the appendix A distance of the oracle's multi-shift solution."""
    print("case c1 hybrid, predicted guesses", flush=True)
    ctx, op, b, sig, xs0, rep0 = _hybrid(nd, "c1", 7, dict(block=(2, 2, 2, 2), n_vec=8), guess=1, predict=0)
    xs, rep = ctx.ndtm_solve(dev(b), ctx.solve_params(n_mmscg=7, guess=1, mms_predict=2))
    print("report", {k: rep[k] for k in ("mms_iterations", "iterations", "guess_kind", "guess_res", "true_res")},
          flush=True)
    assert abs(rep["mms_iterations"] - rep0["mms_iterations"]) <= 2
    for i, s in enumerate(sig):
        assert rel_residual(op, host(xs[i]), b, s) <= 1e-10, (i, s)
    assert rep["guess_kind"][9] != nd.NDTM_GUESS_MMS  # only shifts 7 and 8 are carried
    xo, _, _ = solvers.mms_cg(lambda v: op.Q_hat2(v, sig[-1]), b, sig - sig[-1], tol=1e-10)
    bn = np.sqrt(norm2(b))
    for t in (7, 8):
        if rep["guess_kind"][t] == nd.NDTM_GUESS_MMS and rep["iterations"][t] == 0:
            assert np.linalg.norm(host(xs[t]) - xo[t]) <= 2e-10 * bn / sig[t]
        elif rep["guess_kind"][t] == nd.NDTM_GUESS_MMS:
            # the multigrid started from the iterate, which beat this run's Lagrange guess
            assert rep["guess_res"][t] <= rep["lagrange_res"][t] * (1 + 1e-9)
    ctx.close()


def test_coarse_solve_to_tolerance(nd):
    """With coarse_tol > 0 the coarse GMRES(2) restarts on the true coarse residual
    until it is below the tolerance: the oracle's dense coarse operator (built from
    the same P) confirms ||b_c - D'_c x_c|| <= coarse_tol ||b_c|| for both signs of
    m, where a single two-iteration cycle stays well above it."""
    dims, block, Nv = (8, 8, 8, 8), (4, 4, 4, 4), 8
    print("case 8^4 coarse solve to tolerance", flush=True)
    U = synth.gauge_field(dims, 31, 0.3)
    lat = Lattice(dims, U)
    op = NDOperator(lat, K, MB, EB)
    tv = synth.gaussian_vectors((Nv, lat.V, 4, 3), 32)
    P = omg.build_prolongator(tv, dims, block)
    agg = omg.aggregate_of_site(dims, block)
    Vc = int(np.prod(omg.coarse_dims(dims, block)))
    Dc = omg.coarse_wilson_dense(lat, op.a, P, agg, Vc)
    Bo = omg.odd_projector_coarse(lat, P, agg, Vc)
    bc = synth.gaussian_vectors((Vc, 2, 2 * Nv), 6)
    res = {}
    # both coarse solvers: GMRES on the full coarse system and on its odd Schur complement
    # (even-odd reduction on the coarsest level)
    for eo in (0, 1):
        for tol in (0.0, 1e-9):
            ctx = nd.Context(dims)
            ctx.ndtm_set_gauge(dev(U))
            ctx.ndtm_set_params(K, MB, EB)
            ctx.ndtm_mg_setup(ctx.mg_params(block=block, n_vec=Nv, precision=0, coarse_iters=2, coarse_tol=tol,
                                            coarse_cycles=400, coarse_eo=eo), test_vectors=dev(tv))
            for m in (0.01, -0.01):
                xc = host(ctx.ndtm_mg_coarse_solve(dev(bc), m))
                r = bc - omg.coarse_nd_apply(Dc, Bo, xc, Nv, MB, EB, m=m)
                res[(eo, tol, m)] = np.linalg.norm(r) / np.linalg.norm(bc)
            ctx.close()
    print("relative coarse residuals", res, flush=True)
    for eo in (0, 1):
        for m in (0.01, -0.01):
            assert res[(eo, 1e-9, m)] <= 1e-9
            assert res[(eo, 0.0, m)] > 1e-6
        # one GMRES(2) cycle on the Schur complement leaves a smaller residual than on the
        # full system (the reduced system is better conditioned)
    assert all(res[(1, 0.0, m)] < res[(0, 0.0, m)] for m in (0.01, -0.01))


def test_near_critical_coarse_tolerance_config(nd):
    """kappa = 0.133 (near the critical value of these links) on 8^4: the
    multigrid shifts converge (oracle residual) with the coarse system solved
    to a tolerance, in no more outer iterations than with the fixed coarse solve."""
    dims = (8, 8, 8, 8)
    kap = 0.133
    print("case 8^4 kappa 0.133 hybrid, coarse fixed vs to tolerance", flush=True)
    U = synth.gauge_field(dims, 41, 0.3)
    b = synth.gaussian_spinor(dims, 42)
    shifts = synth.geometric_shifts(10, 1e-4)
    op = NDOperator(Lattice(dims, U), kap, MB, EB)
    its, meth = {}, {}
    for tol in (0.0, 1e-2):
        ctx = nd.Context(dims)
        ctx.ndtm_set_gauge(dev(U))
        ctx.ndtm_set_params(kap, MB, EB)
        ctx.ndtm_set_shifts(list(shifts))
        ctx.ndtm_mg_setup(ctx.mg_params(block=(4, 4, 4, 4), coarse_tol=tol, coarse_cycles=50))
        xs, rep = ctx.ndtm_solve(dev(b), ctx.solve_params(n_mmscg=7, guess=1, mms_predict=0))
        its[tol], meth[tol] = rep["iterations"][7:], rep["method"][7:]
        print("coarse_tol", tol, "method", meth[tol], "iterations", its[tol], "t_mg_ms", rep["t_mg_ms"], flush=True)
        for i, s in enumerate(shifts):
            assert rel_residual(op, host(xs[i]), b, s) <= 1e-10, (tol, i)
        ctx.close()
    # solved to a tolerance, the multigrid finishes every shift itself
    assert meth[1e-2] == [1, 1, 1]
    if meth[0.0] == [1, 1, 1]:
        assert sum(its[1e-2]) <= sum(its[0.0])


@pytest.mark.parametrize("dims,block,Nv,k", [((4, 2, 2, 4), (2, 2, 2, 2), 4, 3), ((8, 8, 8, 8), (4, 4, 4, 4), 8, 8),
                                             ((8, 8, 8, 8), (4, 4, 4, 4), 6, 5)])
def test_coarse_apply_multi_parity(nd, dims, block, Nv, k):
    """The batched coarse stencil on the matrix cores (k systems, each with its own m)
    against the oracle's dense coarse operator built from the same P, and against k
    calls of the one-system kernel; 2 N_v of 8 and 12 exercise the masked rows of a
    16-row tile, k < 8 the masked columns."""
    print(f"case dims={dims} Nv={Nv} k={k} batched coarse stencil", flush=True)
    lat, op, ctx, P, agg, Vc = _setup(nd, dims, block, Nv)
    Dc = omg.coarse_wilson_dense(lat, op.a, P, agg, Vc)
    Bo = omg.odd_projector_coarse(lat, P, agg, Vc)
    ms = [0.0, 0.0316, -0.05, 0.01, -0.0316, 0.2, 1e-3, -1e-3][:k]
    xc = synth.gaussian_vectors((k, Vc, 2, 2 * Nv), 8)
    got = host(ctx.ndtm_mg_coarse_apply_multi(dev(xc), ms))
    for r in range(k):
        want = omg.coarse_nd_apply(Dc, Bo, xc[r], Nv, MB, EB, m=ms[r])
        assert rel_err(got[r], want) < 1e-12, r
        single = host(ctx.ndtm_mg_coarse_apply(dev(xc[r].copy()), ms[r]))
        assert rel_err(got[r], single) < 1e-13, r
    ctx.close()


def test_coarse_apply_multi_config2_shape(nd):
    """At the 16^3x32 shape (2 N_v = 48, three row tiles, 512 coarse sites) the
    batched stencil matches the one-system kernel for 8 systems; bad k is refused."""
    dims, block, Nv = (32, 16, 16, 16), (4, 4, 4, 4), 24
    print("case c2 shape batched coarse stencil", flush=True)
    lat, op, ctx, P, agg, Vc = _setup(nd, dims, block, Nv, seed=12)
    ms = [np.sqrt(s) * sg for s in (8.111e-5, 2.848e-5, 1e-5, 2.31e-4) for sg in (1, -1)]
    xc = synth.gaussian_vectors((8, Vc, 2, 2 * Nv), 9)
    got = host(ctx.ndtm_mg_coarse_apply_multi(dev(xc), ms))
    for r in range(8):
        single = host(ctx.ndtm_mg_coarse_apply(dev(xc[r].copy()), ms[r]))
        assert rel_err(got[r], single) < 1e-13, r
    import ctypes
    x9 = dev(synth.gaussian_vectors((9, Vc, 2, 2 * Nv), 1))
    y9 = x9.clone()
    m9 = (ctypes.c_double * 9)()
    for kbad in (0, 9):
        rc = ctx.lib.ndtm_mg_coarse_apply_multi(ctx.h, y9.data_ptr(), x9.data_ptr(), kbad, m9, None)
        assert rc == -1, kbad
    ctx.close()


def test_coarse_solve_multi(nd):
    """k coarse systems solved together (one matrix-core stencil launch per Arnoldi
    step) against k one-system coarse solves with an FP64 cycle: one GMRES cycle from
    zero agrees to rounding, with the same residual under the oracle's dense coarse
    operator; restarted to coarse_tol every system reaches it; bad k and aliased
    pointers are refused."""
    dims, block, Nv, k = (8, 8, 8, 8), (4, 4, 4, 4), 8, 5
    print(f"case dims={dims} Nv={Nv} k={k} batched coarse solve", flush=True)
    lat, op, ctx, P, agg, Vc = _setup(nd, dims, block, Nv)
    Dc = omg.coarse_wilson_dense(lat, op.a, P, agg, Vc)
    Bo = omg.odd_projector_coarse(lat, P, agg, Vc)
    ms = [0.0, 0.0316, -0.0316, 0.01, 0.2][:k]
    bc = synth.gaussian_vectors((k, Vc, 2, 2 * Nv), 10)

    def res(x, r):
        return rel_err(omg.coarse_nd_apply(Dc, Bo, x, Nv, MB, EB, m=ms[r]), bc[r])

    got = host(ctx.ndtm_mg_coarse_solve_multi(dev(bc), ms))
    for r in range(k):
        single = host(ctx.ndtm_mg_coarse_solve(dev(bc[r].copy()), ms[r]))
        rg, rs = res(got[r], r), res(single, r)
        print("system", r, "m", ms[r], "residual batched", rg, "single", rs, flush=True)
        assert rel_err(got[r], single) < 1e-9, r
        assert abs(rg - rs) <= 1e-8 * rs + 1e-14, r
        assert rg < 1.0, r
    # restarted on the true coarse residual down to coarse_tol
    tv = synth.gaussian_vectors((Nv, lat.V, 4, 3), 32)
    ctx.ndtm_mg_setup(ctx.mg_params(block=block, n_vec=Nv, precision=0, coarse_tol=1e-8, coarse_cycles=60),
                      test_vectors=dev(tv))
    P2 = omg.build_prolongator(tv, dims, block)
    Dc = omg.coarse_wilson_dense(lat, op.a, P2, agg, Vc)
    Bo = omg.odd_projector_coarse(lat, P2, agg, Vc)
    got = host(ctx.ndtm_mg_coarse_solve_multi(dev(bc), ms))
    for r in range(k):
        single = host(ctx.ndtm_mg_coarse_solve(dev(bc[r].copy()), ms[r]))
        rg, rs = res(got[r], r), res(single, r)
        print("restarted system", r, "residual batched", rg, "single", rs, flush=True)
        assert rg <= 2e-8 and rs <= 2e-8, r
    import ctypes
    x = dev(bc)
    y = x.clone()
    m9 = (ctypes.c_double * 9)()
    for kbad in (0, 9):
        assert ctx.lib.ndtm_mg_coarse_solve_multi(ctx.h, y.data_ptr(), x.data_ptr(), kbad, m9, None) == -1, kbad
    assert ctx.lib.ndtm_mg_coarse_solve_multi(ctx.h, x.data_ptr(), x.data_ptr(), k, m9, None) == -1
    ctx.close()


def test_coarse_solve_multi_config2_shape(nd):
    """At the 16^3x32 shape (512 coarse sites, 2 N_v = 48) the batched coarse solve of
    8 systems matches 8 one-system solves with an FP64 cycle."""
    dims, block, Nv = (32, 16, 16, 16), (4, 4, 4, 4), 24
    print("case c2 shape batched coarse solve", flush=True)
    lat, op, ctx, P, agg, Vc = _setup(nd, dims, block, Nv, seed=12)
    ms = [np.sqrt(s) * sg for s in (8.111e-5, 2.848e-5, 1e-5, 2.31e-4) for sg in (1, -1)]
    bc = synth.gaussian_vectors((8, Vc, 2, 2 * Nv), 11)
    got = host(ctx.ndtm_mg_coarse_solve_multi(dev(bc), ms))
    for r in range(8):
        single = host(ctx.ndtm_mg_coarse_solve(dev(bc[r].copy()), ms[r]))
        err = rel_err(got[r], single)
        print("system", r, "rel diff", err, flush=True)
        assert err < 1e-9, r
    ctx.close()


def test_coarse_solve_multi_fp32_cycle_and_one_system(nd):
    """With the default FP32 cycle the batched solve still runs in FP64 on the FP64
    coarse operator: one system (k = 1) agrees with the one-system FP32 solve to FP32
    accuracy and with the oracle's residual of it."""
    dims, block, Nv = (8, 8, 8, 8), (4, 4, 4, 4), 8
    print("case batched coarse solve, k = 1, FP32 cycle setup", flush=True)
    U = synth.gauge_field(dims, 31, 0.3)
    lat = Lattice(dims, U)
    op = NDOperator(lat, K, MB, EB)
    tv = synth.gaussian_vectors((Nv, lat.V, 4, 3), 32)
    ctx = nd.Context(dims)
    ctx.ndtm_set_gauge(dev(U))
    ctx.ndtm_set_params(K, MB, EB)
    ctx.ndtm_mg_setup(ctx.mg_params(block=block, n_vec=Nv, precision=1), test_vectors=dev(tv))
    P = omg.build_prolongator(tv, dims, block)
    agg = omg.aggregate_of_site(dims, block)
    Vc = int(np.prod(omg.coarse_dims(dims, block)))
    Dc = omg.coarse_wilson_dense(lat, op.a, P, agg, Vc)
    Bo = omg.odd_projector_coarse(lat, P, agg, Vc)
    m = 0.0316
    bc = synth.gaussian_vectors((1, Vc, 2, 2 * Nv), 12)
    got = host(ctx.ndtm_mg_coarse_solve_multi(dev(bc), [m]))[0]
    single = host(ctx.ndtm_mg_coarse_solve(dev(bc[0].copy()), m))
    rg = rel_err(omg.coarse_nd_apply(Dc, Bo, got, Nv, MB, EB, m=m), bc[0])
    rs = rel_err(omg.coarse_nd_apply(Dc, Bo, single, Nv, MB, EB, m=m), bc[0])
    print("k=1 rel diff", rel_err(got, single), "residual FP64 batched", rg, "FP32 single", rs, flush=True)
    assert rel_err(got, single) < 1e-4
    assert abs(rg - rs) <= 1e-3 * rs + 1e-6
    ctx.close()


def test_automatic_hybrid_split(nd):
    """n_mmscg = NDTM_NMMS_AUTO: without a multigrid setup every shift goes to the
    multi-shift CG; with one, the first solve sends one shift to the multigrid (its
    cost is measured), later ones take the cost model's n (section 4.4), and every
    shift still meets 1e-10 by the oracle's residual."""
    print("case automatic hybrid split c1", flush=True)
    c = synth.CONFIGS["c1"]
    dims = c["dims"]
    U = synth.gauge_field(dims, c["gauge_seed"], c["amp"])
    b = synth.gaussian_spinor(dims, c["rhs_seed"])
    op = NDOperator(Lattice(dims, U), K, MB, EB)
    sig = c["shifts"]
    ctx = nd.Context(dims)
    ctx.ndtm_set_gauge(dev(U))
    ctx.ndtm_set_params(K, MB, EB)
    ctx.ndtm_set_shifts(list(sig))
    sp = ctx.solve_params(n_mmscg=nd.NDTM_NMMS_AUTO, use_graphs=0)
    _, rep = ctx.ndtm_solve(dev(b), sp)
    assert rep["n_mmscg"] == len(sig)
    ctx.ndtm_mg_setup(ctx.mg_params(block=(2, 2, 2, 2), n_vec=8))
    xs, rep = ctx.ndtm_solve(dev(b), sp)
    assert rep["n_mmscg"] == len(sig) - 1
    chosen = []
    for _ in range(2):
        xs, rep = ctx.ndtm_solve(dev(b), sp)
        chosen.append(rep["n_mmscg"])
        for i, s in enumerate(sig):
            assert rel_residual(op, host(xs[i]), b, s) <= 1e-10
    assert all(1 <= n <= len(sig) for n in chosen)
    print("auto n", chosen, flush=True)
    ctx.close()
