"""Benchmark: all-shift solves of the non-degenerate twisted-mass multi-shift systems.

Workload (default, the largest lattice that fits one GPU): 96x48^3 (T, Lz, Ly, Lx),
links exp(0.3 i H) (gauge seed 15), kappa = 0.1275, mubar = 0.1408, epsbar = 0.1521,
12 shifts geometric in [1e-5, 1], tolerance 1e-10 per shift (true relative residual,
FP64), 8 Gaussian right-hand sides (seeds 25..32) solved back to back with one
multigrid setup reused across them.  One step = one all-shift solve of one right-hand
side; the K timed steps cycle through the 8 right-hand sides, all resident in HBM
before the timed region.  The multigrid setup (test vectors, prolongator, coarse
operator) is timed separately, as it is shared by the right-hand sides.

Forms (the first is the headline `value`):
  full    the workload's full pipeline: multi-shift CG for the 9 largest shifts, the
          two-level aggregation multigrid (case C, FGMRES, FP64 defect correction) for
          the 3 smallest, started from their multi-shift iterates (shifts 10, 11) and
          from the learned guess with Lagrange as fallback (shift 12), in the
          mixed-precision form (FP64 vectors and recurrences; the multi-shift stencil
          moves to FP32, then FP16 storage as the residual falls)
  full_f64  the same in FP64 (the multigrid cycle inside FP64 FGMRES and defect correction)
  plain   multi-shift CG for all 12 shifts in FP64 (the speed-up reference)
  plain_mixed  plain in the mixed-precision form
  hybrid  full_f64 with Lagrange guesses only
  mixed   hybrid in the mixed-precision form
  lagrange  hybrid without the multi-shift iterates as guesses: the three smallest shifts
          go through the multigrid from Lagrange guesses
The multigrid setup (shared by all forms) builds the cycle in FP16 storage (P and the
smoothers' links in FP16; fields, coarse operator and arithmetic in FP32) with SAP
post-smoothing: 2 sweeps over the 4^4 aggregates as blocks, 4 minimal-residual steps per
block solve (--mg-smoother 0 for minimal-residual steps on the whole lattice); the setup's
inverse iteration runs its CG in FP32 (--mg-setup-prec 0 for FP64).
All forms run the same kernels on the same GPU; every shift's FP64 true residual is
reported.  Roofline: the dominant kernel class of the headline form (largest summed
time), timed by HIP events on its launch stream during the timed region; achieved
= algorithmic bytes per launch (per output site 1920 B FP64, 960 B FP32, 488 B FP16)
/ average launch time.  cpu_baseline: the FP64 NumPy oracle on the host, timed on a
bounded sample of this workload and scaled to one all-shift solve (see its "sample").
Prints one JSON line.
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
N_RHS = {"c5": 8}  # right-hand sides of a configuration (seeds rhs_seed, rhs_seed + 1, ...)
ALG_SITE_BYTES = {"hop_f64": 1920.0, "hop_f32": 960.0, "hop_f16": 488.0}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--config", default="c5")
    ap.add_argument("--steps", type=int, default=None, help="timed solves (default: one per right-hand side)")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--forms", default="full,plain,full_f64,plain_mixed,hybrid",
                    help="comma list; the first is the headline value")
    ap.add_argument("--fgmres-restart", type=int, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-dslash", action="store_true")
    ap.add_argument("--no-copy", action="store_true")
    ap.add_argument("--dslash-reps", type=int, default=20)
    ap.add_argument("--cpu-iters", type=int, default=2)
    ap.add_argument("--mg-pair", type=int, default=1, help="case C's two signs in lock-step (needs FP64 coarse blocks)")
    ap.add_argument("--mg-prec", type=int, default=2, help="multigrid cycle precision (2: FP16 storage)")
    ap.add_argument("--mg-eo", type=int, default=1, help="even-odd coarsest level in the single-sign cycles")
    ap.add_argument("--mg-smoother", type=int, default=1, help="0: minimal-residual steps; 1: SAP sweeps")
    ap.add_argument("--mg-smooth-iters", type=int, default=None,
                    help="post-smoothing sweeps (SAP, default 2) or steps (MR, default: the library's 8)")
    ap.add_argument("--sap-mr-iters", type=int, default=4, help="minimal-residual steps per SAP block solve")
    ap.add_argument("--mg-setup-prec", type=int, default=1,
                    help="precision of the setup's inverse iteration (0: FP64, 1: FP32)")
    ap.add_argument("--mlp-weights", default=None,
                    help="weights of the learned guess proposer (.npz, key 'w'; default: the shipped ones)")
    return ap.parse_args()


def cpu_baseline(cfg, U, b, gpu_iters, n_iter):
    """The FP64 oracle on one host thread, on a bounded sample of the workload: n_iter
    multi-shift CG iterations on a two-timeslice slab of the same field (same spatial
    volume, so the same per-site work), scaled by the volume ratio to one iteration on
    the whole lattice and by the iterations the GPU's plain multi-shift CG takes."""
    from threadpoolctl import threadpool_limits

    import synth
    from oracle import solvers
    from oracle.lattice import Lattice, NDOperator

    dims = tuple(cfg["dims"])
    T, Lz, Ly, Lx = dims
    slab_t = 2 if T > 4 else T
    sdims = (slab_t, Lz, Ly, Lx)
    V, Vs = int(np.prod(dims)), int(np.prod(sdims))
    Us = U.reshape(dims + (4, 3, 3))[:slab_t].reshape(Vs, 4, 3, 3)
    bs = b[: Vs // 2]
    op = NDOperator(Lattice(sdims, Us), synth.KAPPA, synth.MUBAR, synth.EPSBAR)
    sig = np.asarray(cfg["shifts"])
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        solvers.mms_cg(lambda v: op.Q_hat2(v, sig[-1]), bs, sig - sig[-1], tol=1e-10, maxiter=n_iter)
        dt = time.perf_counter() - t0
    per_iter = dt / n_iter * (V / Vs)
    est = per_iter * gpu_iters
    out = {"value": 1.0 / est, "unit": "solves/s", "cores": 1, "kind": "oracle",
           "sample": f"{n_iter} oracle multi-shift CG iterations ({len(sig)} shifts) on a "
                     f"{'x'.join(map(str, sdims))} slab of the same field, {dt:.1f} s on one core; scaled "
                     f"by the volume ratio {V // Vs} to {per_iter:.0f} s per iteration on the whole lattice "
                     f"and by the {gpu_iters} iterations of the GPU's plain multi-shift CG: {est:.0f} s "
                     f"per all-shift solve (extrapolated)"}
    # a full oracle solve of the 4^4 configuration (10 shifts), not extrapolated
    c1 = synth.CONFIGS["c1"]
    U1 = synth.gauge_field(c1["dims"], c1["gauge_seed"], c1["amp"])
    b1 = synth.gaussian_spinor(c1["dims"], c1["rhs_seed"])
    op1 = NDOperator(Lattice(c1["dims"], U1), synth.KAPPA, synth.MUBAR, synth.EPSBAR)
    s1 = np.asarray(c1["shifts"])
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        _, it1, _ = solvers.mms_cg(lambda v: op1.Q_hat2(v, s1[-1]), b1, s1 - s1[-1], tol=1e-10)
        dt1 = time.perf_counter() - t0
    out["full_solve_4x4x4x4"] = {"seconds": dt1, "iterations": int(it1), "shifts": len(s1), "cores": 1}
    return out


MIXED_FORMS = ("full", "plain_mixed", "mixed")


def form_params(ctx, nd, form, restart):
    # the multigrid cycle runs eagerly (use_graphs=0): a captured cycle replays bit-identically
    # but was not faster, and eager launches stay visible to the per-class event timers
    hyb = dict(tol=1e-10, n_mmscg=N_MMS, use_graphs=0)
    if restart:
        hyb["fgmres_restart"] = restart
    if form == "plain":
        return ctx.solve_params(tol=1e-10)
    if form == "full":
        return ctx.solve_params(guess=nd.NDTM_GUESS_MLP, mms_predict=2, precision=nd.NDTM_PREC_F16, **hyb)
    if form == "full_f64":
        return ctx.solve_params(guess=nd.NDTM_GUESS_MLP, mms_predict=2, **hyb)
    if form == "hybrid":
        return ctx.solve_params(guess=nd.NDTM_GUESS_LAGRANGE, mms_predict=2, **hyb)
    if form == "lagrange":
        return ctx.solve_params(guess=nd.NDTM_GUESS_LAGRANGE, mms_predict=0, **hyb)
    if form == "plain_mixed":
        return ctx.solve_params(tol=1e-10, precision=nd.NDTM_PREC_F16)
    if form == "mixed":
        return ctx.solve_params(guess=nd.NDTM_GUESS_LAGRANGE, mms_predict=2, precision=nd.NDTM_PREC_F16, **hyb)
    raise ValueError(form)


def run_form(ctx, nd, bds, xs, form, steps, warmup, profile, restart):
    import torch

    params = form_params(ctx, nd, form, restart)
    for w in range(warmup):
        ctx.ndtm_solve(bds[w % len(bds)], params, xs=xs)
    torch.cuda.synchronize()
    if profile:
        for k in range(len(nd.PROF_CLASSES)):
            ctx.ndtm_profile_read(k, reset=True)
        ctx.ndtm_profile_enable((1 << len(nd.PROF_CLASSES)) - 1)
    reps = []
    allocs0 = ctx.ndtm_workspace_stats()["device_allocs"]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        _, rep = ctx.ndtm_solve(bds[k % len(bds)], params, xs=xs)
        reps.append(rep)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    allocs = ctx.ndtm_workspace_stats()["device_allocs"] - allocs0
    prof = None
    if profile:
        ctx.ndtm_profile_enable(0)
        prof = {}
        for k, name in enumerate(nd.PROF_CLASSES):
            ms, n, by = ctx.ndtm_profile_read(k)
            prof[name] = (ms, n, by, ctx.ndtm_profile_moved(k))
    last = reps[-1]
    return {
        "ms_per_solve": 1000.0 * dt / steps,
        "ms_per_solve_each": [r["t_total_ms"] for r in reps],
        "device_allocs_timed": allocs,
        "solves_per_s": steps / dt,
        "worst_true_res": max(max(r["true_res"]) for r in reps),
        "true_res_per_rhs": [max(r["true_res"]) for r in reps],
        "mms_iterations_per_rhs": [r["mms_iterations"] for r in reps],
        "mms_first_f32_f16": [last["mms_it32"], last["mms_it16"]],
        "mg_iterations": [it for it, m in zip(last["iterations"], last["method"]) if m != 0],
        "methods": list(last["method"]),
        "iterations_per_shift": list(last["iterations"]),
        "guess_res": [g for g, m in zip(last["guess_res"], last["method"]) if m != 0],
        "guess_kind": [g for g, m in zip(last["guess_kind"], last["method"]) if m != 0],
        "mlp_res": [g for g, m in zip(last["mlp_res"], last["method"]) if m != 0],
        "lagrange_res": [g for g, m in zip(last["lagrange_res"], last["method"]) if m != 0],
        "t_mms_ms": last["t_mms_ms"], "t_mg_ms": last["t_mg_ms"], "t_guess_ms": last["t_guess_ms"],
    }, prof


def dslash_block(ctx, nd, dims, reps):
    """Q-hat applications (two stencil passes each) on the workload's lattice in each precision."""
    import torch

    import synth

    x = torch.from_numpy(synth.gaussian_spinor(dims, 99)).to("cuda:0")
    y = torch.empty_like(x)
    out = {"lattice": list(dims), "note": "ndtm_apply(QHAT) in a loop; per stencil pass, HIP events on the "
                                          "launch stream; algorithmic bytes 1920/960/488 B per output site"}
    for prec, name in ((nd.NDTM_PREC_F64, "f64"), (nd.NDTM_PREC_F32, "f32"), (nd.NDTM_PREC_F16, "f16")):
        for _ in range(3):
            ctx.ndtm_apply(nd.NDTM_OP_QHAT, x, prec=prec, out=y)
        torch.cuda.synchronize()
        ctx.ndtm_profile_read(prec, reset=True)
        ctx.ndtm_profile_enable(1 << prec)
        for _ in range(reps):
            ctx.ndtm_apply(nd.NDTM_OP_QHAT, x, prec=prec, out=y)
        torch.cuda.synchronize()
        ctx.ndtm_profile_enable(0)
        ms, n, by = ctx.ndtm_profile_read(prec)
        mv = ctx.ndtm_profile_moved(prec)
        ctx.ndtm_profile_read(prec, reset=True)
        gbs = by / (ms * 1e-3) / 1e9
        out[name] = {"gbs": gbs, "frac": gbs / HBM_PEAK_GBS, "avg_launch_us": 1000.0 * ms / n,
                     "alg_bytes_per_launch": by / n, "moved_gbs": mv / (ms * 1e-3) / 1e9, "launches": n}
    del x, y
    return out


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
    gbs = 10 * 2 * a.numel() * 4 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, b
    return gbs


def recorded_traffic(kernel_class, dims):
    """HBM bytes per launch of a kernel class from the committed counter summary of this
    lattice, if the stencil source is unchanged since the counters were taken."""
    import hashlib
    import re

    tag = "x".join(map(str, tuple(dims)[::-1][:3])) + "x" + str(dims[0])
    path = os.path.join(ROOT, "profiles", f"{kernel_class}_{tag}_counters.md")
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
    import synth

    cfg = synth.CONFIGS[args.config]
    dims = cfg["dims"]
    n_rhs = N_RHS.get(args.config, 1)
    steps = args.steps if args.steps is not None else max(n_rhs, 1)
    # inputs on the host before anything touches the GPU (the link exponentials of large
    # lattices are taken by forked worker processes)
    t0 = time.perf_counter()
    U = synth.gauge_field(dims, cfg["gauge_seed"], cfg["amp"], workers=16)
    bs = [synth.gaussian_spinor(dims, cfg["rhs_seed"] + k) for k in range(n_rhs)]
    log(f"inputs {dims} x {n_rhs} rhs generated in {time.perf_counter() - t0:.1f} s")

    import torch

    import paper_1805_09584_amd as nd

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
    bds = [torch.from_numpy(b).to(dev) for b in bs]
    b0 = bs[0]
    del bs
    xs = [torch.empty_like(bds[0]) for _ in cfg["shifts"]]
    big = int(np.prod(dims)) > 4_000_000
    restart = args.fgmres_restart if args.fgmres_restart else (8 if big else None)

    forms = [f for f in args.forms.split(",") if f]
    setup_ms = None
    smooth_iters = None
    mgp = None
    if any(f not in ("plain", "plain_mixed") for f in forms):
        # cycle in FP16 storage (FP16 P and links, FP32 fields and arithmetic); on the large
        # lattice the FP64 copies of P and the coarse blocks are freed after the setup (the
        # cycle reads only its own copies)
        mgp = ctx.mg_params(keep_f64=0 if big else 1, precision=args.mg_prec, pair_signs=args.mg_pair,
                            coarse_eo=args.mg_eo, smoother=args.mg_smoother, sap_mr_iters=args.sap_mr_iters,
                            setup_prec=args.mg_setup_prec)
        if args.mg_smooth_iters is not None:
            mgp.smooth_iters = args.mg_smooth_iters
        elif args.mg_smoother == 1:
            mgp.smooth_iters = 2
        smooth_iters = mgp.smooth_iters
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.ndtm_mg_setup(mgp)
        torch.cuda.synchronize()
        setup_ms = 1000.0 * (time.perf_counter() - t0)
        log(f"multigrid setup {setup_ms / 1000:.1f} s")
    weights = args.mlp_weights or nd.trained_weights_path()
    if any(f in ("full", "full_f64") for f in forms):
        if weights and os.path.exists(weights):
            ctx.ndtm_mlp_set_weights(np.load(weights)["w"])
        else:
            forms = [f for f in forms if f not in ("full", "full_f64")]

    results = {}
    prof = None
    for f in forms:
        head = f == forms[0]
        results[f], p = run_form(ctx, nd, bds, xs, f, steps, args.warmup, profile=head, restart=restart)
        if head:
            prof = p
        log(f"form {f}: {results[f]['ms_per_solve']:.1f} ms per solve, worst residual "
            f"{results[f]['worst_true_res']:.2e}")
    head = results[forms[0]]
    dom = max(prof, key=lambda k: prof[k][0])
    ms, nl, by, mv = prof[dom]
    achieved = by / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
    classes = {k: {"ms": v[0], "launches": v[1], "avg_launch_us": 1000.0 * v[0] / v[1],
                   "gbs": (v[2] / (v[0] * 1e-3) / 1e9) if v[0] > 0 else 0.0,
                   "moved_gbs": (v[3] / (v[0] * 1e-3) / 1e9) if v[0] > 0 else 0.0}
               for k, v in prof.items() if v[1] > 0}
    speedup = {f: results["plain"]["ms_per_solve"] / results[f]["ms_per_solve"]
               for f in results if "plain" in results and f != "plain"}
    mem = ctx.ndtm_workspace_stats()
    out = {
        "metric": METRIC,
        "value": head["solves_per_s"],
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_solve"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64/f32/f16" if forms[0] in MIXED_FORMS else "f64",
        "data": "synthetic",
        "config": {"workload": f"ND twisted-mass multi-shift solves, {'x'.join(map(str, dims))} (T,Lz,Ly,Lx), "
                               f"{len(cfg['shifts'])} shifts geometric in [{cfg['shifts'][-1]:g},1], tol 1e-10, "
                               f"{n_rhs} right-hand side(s) back to back with one multigrid setup, form "
                               f"'{forms[0]}'",
                   "lattice": list(dims), "n_shifts": len(cfg["shifts"]), "n_rhs": n_rhs, "form": forms[0],
                   "n_mmscg": N_MMS if forms[0] != "plain" else len(cfg["shifts"]),
                   "kappa": synth.KAPPA, "mubar": synth.MUBAR, "epsbar": synth.EPSBAR, "link_amp": cfg["amp"]},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": recorded_traffic(dom, dims),
                     "launches": nl, "avg_launch_us": 1000.0 * ms / max(nl, 1),
                     "alg_bytes_per_launch": by / max(nl, 1),
                     "alg_bytes_per_site": ALG_SITE_BYTES.get(dom),
                     "moved_gbs": mv / (ms * 1e-3) / 1e9 if ms > 0 else 0.0},
        "kernel_classes": classes,
        "forms": results,
        "speedup_vs_plain": speedup,
        "mg_setup_ms": setup_ms,
        "mg_cycle": {"precision": args.mg_prec, "pair_signs": args.mg_pair, "coarse_eo": args.mg_eo,
                     "smoother": "sap" if args.mg_smoother == 1 else "mr", "smooth_iters": smooth_iters,
                     "sap_mr_iters": args.sap_mr_iters if args.mg_smoother == 1 else None,
                     "setup_precision": "f32" if args.mg_setup_prec == 1 else "f64"},
        "fgmres_restart": restart or 16,
        "mlp_weights": os.path.basename(weights) if any(f in ("full", "full_f64") for f in forms) else None,
        "set_gauge_ms": set_gauge_ms,
        "device_storage_gb": {"live": mem["live"] / 1e9, "peak": mem["peak"] / 1e9},
    }
    # the solve's fields go back before the stencil block takes its own
    ctx.ndtm_trim()
    if not args.no_dslash:
        out["dslash"] = dslash_block(ctx, nd, dims, args.dslash_reps)
    if not args.no_copy:
        out["copy_ceiling_gbs"] = copy_ceiling()
        cp, rd, wr = ctx.ndtm_stream_bandwidth(1 << 30, 10)
        out["stream_ceiling_gbs"] = {"copy": cp, "read": rd, "write": wr,
                                     "note": "library's 16-byte non-temporal streaming kernels, 1 GiB"}
    ctx.close()
    if not args.no_cpu_baseline:
        it = (results["plain"]["mms_iterations_per_rhs"][0] if "plain" in results
              else head["mms_iterations_per_rhs"][0])
        log("cpu baseline")
        out["cpu_baseline"] = cpu_baseline(cfg, U, b0, it, args.cpu_iters)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
