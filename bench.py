"""Benchmark: all-shift solve of the non-degenerate twisted-mass multi-shift systems.

One step = one solve of all shifted systems (Q^2 + sigma_i) x_i = b for one
synthetic right-hand side, to a true relative residual of 1e-10 per shift, on
the 16^3x32 lattice with 12 shifts geometric in [1e-5, 1] (kappa = 0.1275,
mubar = 0.1408, epsbar = 0.1521, links exp(0.3 i H)), by the hybrid solver:
multi-shift CG for the 9 largest shifts, the two-level aggregation multigrid
(case C, FGMRES, FP64 defect correction) for the 3 smallest, started from the
Lagrange guesses refined by a minimal-residual projection over the converged
solutions.  The multigrid setup (test vectors, prolongator, coarse operator) is
done once before the timed region and reported separately, as it is reused
across right-hand sides.  Inputs are resident in HBM before the timed region.

Beside the headline (hybrid) the same K steps are timed for plain multi-shift
CG over all 12 shifts (the speed-up reference), the hybrid with plain Lagrange
guesses, the mixed-precision form and, when trained weights are present, the
learned-guess form.  A separate block
times the even-odd stencil on a 32^3x64 lattice (the 16^3x32 field tiled 2x in
every direction), where the working set is far above the 256 MB last-level
cache.  Prints one JSON line.

Roofline: the headline form's K steps are run once more with every kernel
class timed by HIP events on the launch stream; the dominant class (largest
summed time) gives achieved GB/s = its algorithmic bytes / its summed kernel
time.
cpu_baseline: the FP64 NumPy oracle timed on a bounded sample (a few
multi-shift CG iterations on the same lattice) and scaled to one solve.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "All-shift rational solve time at 1e-10 vs plain MMS-CG; Dslash HBM GB/s"
HBM_PEAK_GBS = 8000.0
N_MMS = 9


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="c2")
    ap.add_argument("--forms", default="hybrid,plain,hybrid_direct,plain_direct,hybrid_projection,lagrange,mixed,learned",
                    help="comma list; the first is the headline value")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-dslash", action="store_true")
    ap.add_argument("--no-copy", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=2)
    ap.add_argument("--dslash-reps", type=int, default=50)
    return ap.parse_args()


def cpu_baseline(cfg, U, b, gpu_iters, n_iter):
    """Times n_iter iterations of the oracle's multi-shift CG on one host thread."""
    from threadpoolctl import threadpool_limits

    import synth
    from oracle import solvers
    from oracle.lattice import Lattice, NDOperator

    op = NDOperator(Lattice(cfg["dims"], U), synth.KAPPA, synth.MUBAR, synth.EPSBAR)
    sig = np.asarray(cfg["shifts"])
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        solvers.mms_cg(lambda v: op.Q_hat2(v, sig[-1]), b, sig - sig[-1], tol=1e-10, maxiter=n_iter)
        dt = time.perf_counter() - t0
    per_iter = dt / n_iter
    est = per_iter * gpu_iters
    return {"value": 1.0 / est, "unit": "solves/s", "cores": 1, "kind": "oracle",
            "sample": f"{n_iter} oracle multi-shift CG iterations on the same lattice and shifts "
                      f"({per_iter:.2f} s each), scaled to the {gpu_iters} iterations the plain "
                      f"multi-shift CG takes for the whole solve ({est:.0f} s per solve)"}


def form_params(ctx, nd, form):
    # the multigrid cycle runs eagerly (use_graphs=0): a captured cycle replays
    # bit-identically but was not faster, and eager launches stay visible to the
    # per-class event timers
    hyb = dict(tol=1e-10, n_mmscg=N_MMS, use_graphs=0)
    if form == "plain":
        return ctx.solve_params(tol=1e-10)
    if form == "plain_direct":
        # shifted solutions and directions updated every iteration instead of once per block
        return ctx.solve_params(tol=1e-10, mms_defer=0)
    if form == "hybrid":
        # the paper's recipe (section 4.2): shifts n+1, n+2 start from their multi-shift
        # iterates, the rest from Lagrange interpolation over the converged solutions
        return ctx.solve_params(guess=nd.NDTM_GUESS_LAGRANGE, mms_predict=2, **hyb)
    if form == "hybrid_direct":
        return ctx.solve_params(guess=nd.NDTM_GUESS_LAGRANGE, mms_predict=2, mms_defer=0, **hyb)
    if form == "hybrid_projection":
        # Lagrange guesses refined by the minimal-residual projection over the converged solutions
        return ctx.solve_params(guess=nd.NDTM_GUESS_PROJECTION, mms_predict=2, **hyb)
    if form == "lagrange":
        # no predicted guesses: every multigrid shift starts from Lagrange interpolation
        return ctx.solve_params(guess=nd.NDTM_GUESS_LAGRANGE, mms_predict=0, **hyb)
    if form == "mixed":
        return ctx.solve_params(guess=nd.NDTM_GUESS_LAGRANGE, precision=nd.NDTM_PREC_F16, **hyb)
    if form == "learned":
        return ctx.solve_params(guess=nd.NDTM_GUESS_MLP, mms_predict=0, **hyb)
    raise ValueError(form)


def run_form(ctx, nd, bd, xs, form, steps, warmup, profile):
    import torch

    params = form_params(ctx, nd, form)
    for _ in range(warmup):
        ctx.ndtm_solve(bd, params, xs=xs)
    torch.cuda.synchronize()
    if profile:
        ctx.ndtm_profile_enable((1 << len(nd.PROF_CLASSES)) - 1)
        for k in range(len(nd.PROF_CLASSES)):
            ctx.ndtm_profile_read(k, reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = []
    for _ in range(steps):
        _, rep = ctx.ndtm_solve(bd, params, xs=xs)
        reps.append(rep)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = None
    if profile:
        ctx.ndtm_profile_enable(0)
        prof = {nd.PROF_CLASSES[k]: ctx.ndtm_profile_read(k) for k in range(len(nd.PROF_CLASSES))}
    last = reps[-1]
    return {
        "ms_per_solve": 1000.0 * dt / steps,
        "solves_per_s": steps / dt,
        "worst_true_res": max(max(r["true_res"]) for r in reps),
        "mms_iterations": last["mms_iterations"],
        "mg_iterations": [it for it, m in zip(last["iterations"], last["method"]) if m != 0],
        "iterations_per_shift": list(last["iterations"]),
        "guess_res": [g for g, m in zip(last["guess_res"], last["method"]) if m != 0],
        "guess_kind": [g for g, m in zip(last["guess_kind"], last["method"]) if m != 0],
        "t_mms_ms": last["t_mms_ms"], "t_mg_ms": last["t_mg_ms"], "t_guess_ms": last["t_guess_ms"],
    }, prof


def dslash_block(nd, U_small, d0, reps):
    """Q-hat applications on the lattice of twice the extent (the field tiled 2x per direction)."""
    import torch

    import synth

    U = np.tile(U_small.reshape(tuple(d0) + U_small.shape[1:]), (2, 2, 2, 2, 1, 1, 1))
    dims = U.shape[:4]
    U = U.reshape((-1,) + U_small.shape[1:])
    ctx = nd.Context(dims)
    ctx.ndtm_set_gauge(torch.from_numpy(U).to("cuda:0"))
    del U
    ctx.ndtm_set_params(synth.KAPPA, synth.MUBAR, synth.EPSBAR)
    x = torch.from_numpy(synth.gaussian_spinor(dims, 99)).to("cuda:0")
    y = torch.empty_like(x)
    out = {"lattice": list(dims)}
    for prec, name in ((nd.NDTM_PREC_F64, "f64"), (nd.NDTM_PREC_F32, "f32"), (nd.NDTM_PREC_F16, "f16")):
        for _ in range(3):
            ctx.ndtm_apply(nd.NDTM_OP_QHAT, x, prec=prec, out=y)
        torch.cuda.synchronize()
        ctx.ndtm_profile_enable(1 << prec)
        ctx.ndtm_profile_read(prec, reset=True)
        for _ in range(reps):
            ctx.ndtm_apply(nd.NDTM_OP_QHAT, x, prec=prec, out=y)
        torch.cuda.synchronize()
        ctx.ndtm_profile_enable(0)
        ms, n, by = ctx.ndtm_profile_read(prec, reset=True)
        gbs = by / (ms * 1e-3) / 1e9
        out[name] = {"gbs": gbs, "frac": gbs / HBM_PEAK_GBS, "avg_launch_us": 1000.0 * ms / n,
                     "alg_bytes_per_launch": by / n, "launches": n}
    ctx.close()
    return out


def coarse_batched_block(ctx, nd, reps=50):
    """The coarse stencil of the 16^3x32 hierarchy for 8 systems (the 3 multigrid shifts'
    signs and more): one batched launch on the matrix cores against 8 one-system launches."""
    import torch

    import synth

    k, Vc, Nv = 8, ctx.Vc, ctx.n_vec
    xc = torch.from_numpy(synth.gaussian_vectors((k, Vc, 2, 2 * Nv), 9)).to("cuda:0")
    yc = torch.empty_like(xc)
    ms = [0.009 * (1 if r % 2 == 0 else -1) * (r // 2 + 1) for r in range(k)]
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(fn, n=reps):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        e0.record()
        for _ in range(n):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) * 1000.0 / n

    def singles():
        for r in range(k):
            ctx.ndtm_mg_coarse_apply(xc[r], ms[r])

    t_multi = timed(lambda: ctx.ndtm_mg_coarse_apply_multi(xc, ms, out=yc))
    t_single = timed(singles)

    # the coarse solve (one GMRES(coarse_iters) cycle from zero per system): the 8 systems
    # together in FP64, the batched stencil in every Arnoldi step, against 8 one-system
    # solves in the cycle precision
    def solve_singles():
        for r in range(k):
            ctx.ndtm_mg_coarse_solve(xc[r], ms[r])

    t_solve_multi = timed(lambda: ctx.ndtm_mg_coarse_solve_multi(xc, ms, out=yc), 10)
    t_solve_single = timed(solve_singles, 10)
    n2 = 2 * Nv
    block_bytes = Vc * (9 * n2 * n2 + 2 * Nv * Nv) * 16.0
    vec_bytes = 2 * k * Vc * 2 * n2 * 16.0
    flops = k * Vc * 9 * n2 * n2 * 2 * 8.0
    return {"systems": k, "coarse_sites": Vc, "dof_per_site": 2 * n2, "precision": "f64",
            "us_batched": t_multi, "us_one_system_each": t_single,
            "speedup": t_single / t_multi,
            "batched_gbs": (block_bytes + vec_bytes) / (t_multi * 1e-6) / 1e9,
            "batched_tflops": flops / (t_multi * 1e-6) / 1e12,
            "solve": {"us_batched_f64": t_solve_multi, "us_one_system_each_cycle_precision": t_solve_single,
                      "note": "one GMRES cycle from zero per system; the one-system solves run in the "
                              "cycle precision (FP32 by default), the batched one in FP64"}}


def copy_ceiling():
    """Measured streaming ceiling: a device-to-device copy of 2 GiB (read + write)."""
    import torch

    a = torch.empty(1 << 29, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    return 10 * 2 * a.numel() * 4 / (e0.elapsed_time(e1) * 1e-3) / 1e9


def recorded_traffic(kernel_class, dims):
    """HBM bytes per launch of the dominant kernel class from the committed counter
    summary, if it was taken on this lattice (the 32x16x16x16 hybrid solve) and the
    stencil source is unchanged since."""
    import hashlib
    import re

    if tuple(dims) != (32, 16, 16, 16):
        return None
    path = os.path.join(ROOT, "profiles", f"{kernel_class}_16x16x16x32_hybrid_counters.md")
    src = os.path.join(ROOT, "paper_1805_09584_amd", "csrc", "kern_dslash.hip")
    if not os.path.exists(path):
        return None
    m = re.search(r"traffic_json: (\{.*\})", open(path).read())
    if not m:
        return None
    rec = json.loads(m.group(1))
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    return rec["bytes_per_launch"] if rec.get("source_sha256") == sha else None


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1 "
                                   "(multi-GPU sharding is described in the design notes, not built)"}))
        sys.exit(2)
    import torch

    import paper_1805_09584_amd as nd
    import synth

    cfg = synth.CONFIGS[args.config]
    dims = cfg["dims"]
    U = synth.gauge_field(dims, cfg["gauge_seed"], cfg["amp"])
    b = synth.gaussian_spinor(dims, cfg["rhs_seed"])
    dev = torch.device("cuda:0")
    ctx = nd.Context(dims)
    Ud = torch.from_numpy(U).to(dev)
    ctx.ndtm_set_gauge(Ud)
    # field import (links already in device memory): SU(3) check and repacking into the
    # even/odd FP64, FP32 and FP16 link arrays, averaged over three calls
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(3):
        ctx.ndtm_set_gauge(Ud)
    torch.cuda.synchronize()
    set_gauge_ms = 1000.0 * (time.perf_counter() - t0) / 3
    del Ud
    ctx.ndtm_set_params(synth.KAPPA, synth.MUBAR, synth.EPSBAR)
    ctx.ndtm_set_shifts(list(cfg["shifts"]))
    bd = torch.from_numpy(b).to(dev)
    xs = [torch.empty_like(bd) for _ in cfg["shifts"]]

    forms = [f for f in args.forms.split(",") if f]
    setup_ms = None
    if any(f != "plain" for f in forms):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.ndtm_mg_setup(ctx.mg_params())
        torch.cuda.synchronize()
        setup_ms = 1000.0 * (time.perf_counter() - t0)
    weights = nd.trained_weights_path()
    if "learned" in forms:
        if weights and os.path.exists(weights):
            ctx.ndtm_mlp_set_weights(np.load(weights)["w"])
        else:
            forms.remove("learned")

    coarse_batched = coarse_batched_block(ctx, nd) if setup_ms is not None else None
    results = {}
    spectrum = None
    for f in forms:
        results[f], _ = run_form(ctx, nd, bd, xs, f, args.steps, args.warmup, profile=False)
        if f == "plain":
            # extreme eigenvalues of Q^2 for this field from the Lanczos matrix of the plain
            # solve's recorded CG coefficients (available when the solve fits one block of
            # deferred updates)
            try:
                lo, hi = ctx.ndtm_spectrum_estimate()
                spectrum = {"lambda_min": lo, "lambda_max": hi, "source": "Lanczos matrix of the plain "
                            "multi-shift CG coefficients (base shift removed)"}
            except nd.NdtmError:
                spectrum = None
    # roofline: the same K steps of the headline form again, with every kernel
    # class timed by HIP events on the launch stream (the event pairs add a few
    # percent, so the headline value comes from the unprofiled pass above)
    prof_run, prof = run_form(ctx, nd, bd, xs, forms[0], args.steps, 0, profile=True)
    head = results[forms[0]]
    # the multigrid kernels do no work in the headline form here (its guesses already meet
    # the tolerance): time their classes in one solve of the form without predicted guesses
    mg_classes = None
    if "lagrange" in forms:
        _, mprof = run_form(ctx, nd, bd, xs, "lagrange", 1, 0, profile=True)
        mg_classes = {k: {"ms": v[0], "launches": v[1], "gbs": (v[2] / (v[0] * 1e-3) / 1e9) if v[0] > 0 else 0.0,
                          "avg_launch_us": 1000.0 * v[0] / v[1]}
                      for k, v in mprof.items() if v[1] > 0 and k in ("restrict", "prolong", "coarse", "hop_f32")}
    dom = max(prof, key=lambda k: prof[k][0])
    ms, nl, by = prof[dom]
    achieved = by / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
    classes = {k: {"ms": v[0], "launches": v[1], "gbs": (v[2] / (v[0] * 1e-3) / 1e9) if v[0] > 0 else 0.0}
               for k, v in prof.items() if v[1] > 0}
    speedup = {f: results["plain"]["ms_per_solve"] / results[f]["ms_per_solve"]
               for f in results if "plain" in results and f != "plain"}
    out = {
        "metric": METRIC,
        "value": head["solves_per_s"],
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_solve"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"ND twisted-mass multi-shift solve, {'x'.join(map(str, dims))} (T,Lz,Ly,Lx), "
                               f"{len(cfg['shifts'])} shifts geometric in [{cfg['shifts'][-1]:g},1], tol 1e-10, "
                               f"{forms[0]} ({N_MMS} multi-shift CG + {len(cfg['shifts']) - N_MMS} multigrid case C"
                               + (", the first two multigrid shifts carried in the multi-shift CG for predicted "
                                  "initial guesses, Lagrange-interpolated guesses for the rest; shifted vectors "
                                  "formed once per block of up to 256 iterations)"
                                  if forms[0] == "hybrid" else ")")
                               if forms[0] != "plain" else "plain multi-shift CG",
                   "lattice": list(dims), "n_shifts": len(cfg["shifts"]), "form": forms[0],
                   "kappa": synth.KAPPA, "mubar": synth.MUBAR, "epsbar": synth.EPSBAR, "link_amp": cfg["amp"]},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": recorded_traffic(dom, dims),
                     "launches": nl, "avg_launch_us": 1000.0 * ms / max(nl, 1),
                     "alg_bytes_per_launch": by / max(nl, 1)},
        "kernel_classes": classes,
        "mg_kernel_classes": mg_classes,
        "spectrum_q2": spectrum,
        "coarse_batched": coarse_batched,
        "ms_per_step_profiled": prof_run["ms_per_solve"],
        "forms": results,
        "speedup_vs_plain": speedup,
        "mg_setup_ms": setup_ms,
        "set_gauge_ms": set_gauge_ms,
    }
    if not args.no_dslash:
        out["dslash_large"] = dslash_block(nd, U, dims, args.dslash_reps)
    if not args.no_copy:
        out["copy_ceiling_gbs"] = copy_ceiling()
        cp, rd, wr = ctx.ndtm_stream_bandwidth(1 << 30, 10)
        out["stream_ceiling_gbs"] = {"copy": cp, "read": rd, "write": wr,
                                     "note": "library's 16-byte non-temporal streaming kernels, 1 GiB"}
    if not args.no_cpu_baseline:
        it = results["plain"]["mms_iterations"] if "plain" in results else head["mms_iterations"]
        out["cpu_baseline"] = cpu_baseline(cfg, U, b, it, args.cpu_iters)
    ctx.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
