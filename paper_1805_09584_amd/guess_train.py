"""Training of the learned initial-guess proposer on solves the method makes itself.

Data: for each seeded gauge field (link amplitude drawn from U[0.2, 0.4]) and
right-hand side, the plain multi-shift CG solves all shifts to a relative
residual of 1e-10.  Every multigrid target t (a shift after the first n_mms)
then gives one sample, built by ndtm_mlp_sample from the converged solutions
of the shifts above it: the features, the mask of filled slots and the exact
quadratic form (G, h) of the guess residual.  Training is full-batch Adam
through ndtm_mlp_train (FP32 forward/backward kernels); inference at solve
time uses the BF16 kernel.  The learned proposal is kept only where its
predicted residual beats the Lagrange guess, so the evaluation reports the
residual of the chosen guess relative to Lagrange, next to the least-squares
optimum over the same span (the best any mixing of these solutions can do).

Usage (on a GPU):  python -m paper_1805_09584_amd.guess_train --out W.npz
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from multiprocessing import Pool

import numpy as np

_ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if _ROOT not in sys.path:
    sys.path.insert(0, _ROOT)

N_MMS = 9


def init_weights(seed, n_in=59, width=64, n_out=11, out_scale=1e-2):
    """Flat FP32 initial weights (W1, b1, W2, b2, W3, b3, row-major): Gaussian with
    variance 1/fan_in for the tanh layers and a small output layer, so the first
    proposals stay close to the Lagrange guess."""
    rng = np.random.default_rng(seed)
    parts = [rng.standard_normal((width, n_in)) / np.sqrt(n_in), np.zeros(width),
             rng.standard_normal((width, width)) / np.sqrt(width), np.zeros(width),
             rng.standard_normal((n_out, width)) * out_scale, np.zeros(n_out)]
    return np.concatenate([p.ravel() for p in parts]).astype(np.float32)


def _field(args):
    import synth

    dims, seed, amp = args
    return synth.gauge_field(dims, seed, amp)


def field_plan(n, seed0, amp_seed, lo=0.2, hi=0.4):
    amps = np.random.default_rng(amp_seed).uniform(lo, hi, n)
    return [(seed0 + i, float(amps[i])) for i in range(n)]


def collect(dims, plan, shifts, rhs_seed0, pool, log=print):
    """Samples (features, mask, G, h, tau) of the multigrid targets of every field in plan.

    pool: a multiprocessing pool that generates the gauge fields on the host; it
    must have been started before this process touched the GPU."""
    import torch

    import paper_1805_09584_amd as nd
    import synth

    shifts = np.asarray(shifts, dtype=np.float64)
    out = {k: [] for k in ("F", "mask", "G", "h", "tau", "field", "target", "amp")}
    ctx = nd.Context(dims)
    ctx.ndtm_set_params(synth.KAPPA, synth.MUBAR, synth.EPSBAR)
    ctx.ndtm_set_shifts(list(shifts))
    prm = ctx.solve_params(tol=1e-10)
    t0 = time.time()
    for i, U in enumerate(pool.imap(_field, [(dims, s, a) for s, a in plan])):
        seed, amp = plan[i]
        ctx.ndtm_set_gauge(torch.from_numpy(U).to("cuda:0"))
        b = torch.from_numpy(synth.gaussian_spinor(dims, rhs_seed0 + seed)).to("cuda:0")
        xs, rep = ctx.ndtm_solve(b, prm)
        for t in range(N_MMS, len(shifts)):
            f, m, G, h, info = ctx.ndtm_mlp_sample(xs[:t], shifts[:t], shifts[t], b)
            out["F"].append(f)
            out["mask"].append(m)
            out["G"].append(G)
            out["h"].append(h)
            out["tau"].append(info[0])
            out["field"].append(seed)
            out["target"].append(t)
            out["amp"].append(amp)
        if (i + 1) % 25 == 0:
            log(f"fields {i + 1}/{len(plan)}  {time.time() - t0:.0f} s  mms its {rep['mms_iterations']}")
    ctx.close()
    return {k: np.asarray(v) for k, v in out.items()}


def predicted_loss(y, mask, G, h):
    ym = (mask * y).astype(np.float64)
    return 1.0 + np.einsum("bi,bi->b", 2.0 * h + np.einsum("bij,bj->bi", G, ym), ym)


def ls_loss(mask, G, h):
    L = np.zeros(len(mask))
    for s in range(len(mask)):
        idx = np.nonzero(mask[s])[0]
        Gs = G[s][np.ix_(idx, idx)].astype(np.float64)
        hs = h[s][idx].astype(np.float64)
        y, *_ = np.linalg.lstsq(Gs, -hs, rcond=1e-7)
        L[s] = 1.0 + 2.0 * hs @ y + y @ Gs @ y
    return L


def evaluate(ctx, data):
    """Residual ratios (chosen guess / Lagrange) per sample, BF16 inference."""
    y, _ = ctx.ndtm_mlp_forward(data["F"], bf16=True)
    L = predicted_loss(y, data["mask"], data["G"], data["h"])
    chosen = np.minimum(np.maximum(L, 0.0), 1.0)
    Ls = np.clip(ls_loss(data["mask"], data["G"], data["h"]), 0.0, 1.0)
    ratio = np.sqrt(chosen)
    res = {"n": int(len(L)), "kept_fraction": float(np.mean(L < 1.0)),
           "geomean_ratio": float(np.exp(np.mean(np.log(np.maximum(ratio, 1e-300))))),
           "median_ratio": float(np.median(ratio)),
           "ls_geomean_ratio": float(np.exp(np.mean(np.log(np.maximum(np.sqrt(Ls), 1e-300)))))}
    for t in sorted(set(data["target"].tolist())):
        sel = data["target"] == t
        res[f"target{t}"] = {"geomean_ratio": float(np.exp(np.mean(np.log(np.maximum(ratio[sel], 1e-300))))),
                             "ls_geomean_ratio": float(np.exp(np.mean(np.log(np.maximum(np.sqrt(Ls[sel]),
                                                                                         1e-300))))),
                             "lagrange_median_res": float(np.median(data["tau"][sel]))}
    return res


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--dims", default="32,16,16,16")
    ap.add_argument("--train-fields", type=int, default=200)
    ap.add_argument("--test-fields", type=int, default=50)
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--seed", type=int, default=4000)
    ap.add_argument("--workers", type=int, default=12)
    ap.add_argument("--out", required=True)
    ap.add_argument("--report", default=None)
    a = ap.parse_args(argv)
    import paper_1805_09584_amd as nd
    import synth

    def log(msg):
        print(msg, flush=True)

    dims = tuple(int(x) for x in a.dims.split(","))
    shifts = synth.geometric_shifts(12, 1e-5)
    # the host workers are forked before anything here initialises the GPU
    with Pool(a.workers) as pool:
        train = collect(dims, field_plan(a.train_fields, 1000, 5000), shifts, 3000, pool, log)
        log(f"train samples {len(train['F'])}")
        test = collect(dims, field_plan(a.test_fields, 2000, 5001), shifts, 3000, pool, log)
        log(f"held-out samples {len(test['F'])}")
    ctx = nd.Context(dims)
    ctx.ndtm_mlp_set_weights(init_weights(a.seed))
    before = evaluate(ctx, test)
    t0 = time.time()
    hist = ctx.ndtm_mlp_train(train["F"], train["mask"], train["G"], train["h"], a.steps, a.lr)
    t_train = time.time() - t0
    w = ctx.ndtm_mlp_get_weights()
    rep = {"dims": list(dims), "train_samples": int(len(train["F"])), "test_samples": int(len(test["F"])),
           "steps": a.steps, "lr": a.lr, "train_seconds": t_train,
           "loss_first": float(hist[0]), "loss_last": float(hist[-1]),
           "train_eval": evaluate(ctx, train), "test_eval": evaluate(ctx, test), "test_eval_init": before}
    log(json.dumps(rep))
    np.savez(a.out, w=w, hist=hist)
    if a.report:
        with open(a.report, "w") as f:
            json.dump(rep, f, indent=1)
    ctx.close()


if __name__ == "__main__":
    main()
