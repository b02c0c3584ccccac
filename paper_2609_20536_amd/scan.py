"""Full-size phase-diagram scan and surrogate refinement (host orchestration).

The 16 x 16 (beta, Delta) grid (beta in [0.5, 1.5], Delta in [0, 1], Dcut
per point from {24, 32, 48, 64}, |n| <= 10, 40 steps) is scanned by the
zero-field route: three HOTRG runs per point (beta -+ 1e-3 for C_v, and the
central run with the second-moment chains for chi and chi_n at h = 0), all in
U(1) charge blocks. The surrogate (2-128-128-4 MLP) is trained on the grid
(90/10 split), proposes two refinement points per Delta of a 256 x 256
lattice (the predicted C_v and chi maxima: 512 points), and each proposal is
verified by a Dcut = 64 FP64 HOTRG run at zero field (accepted when the
predicted f is within 1e-3 relative of HOTRG's).

Every computation runs in the library (gxy_run_batch, gxy_observables,
gxy_mlp_*); this module assembles run lists and arrays and times them.

    python -m paper_2609_20536_amd.scan [--out results.json] [--workers 16]
"""

from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import surrogate as S
from . import workloads as W
from .hotrg import Context, Surrogate


def scan_grid(ctx: Context, prec: int = W.PREC_FP64, fp64_steps: int = 0,
              workers: int = 16, grid=None):
    grid = W.grid_points() if grid is None else grid
    t0 = time.perf_counter()
    obs, res = S.grid_observables_zero_field(ctx, grid, workers=workers, prec=prec,
                                             fp64_steps=fp64_steps)
    el = time.perf_counter() - t0
    return grid, obs, el


def refine(ctx: Context, grid, obs: np.ndarray, workers: int = 16, epochs: int = 5000,
           tol: float = 1e-3):
    X = np.array([[g.beta, g.delta] for g in grid])
    tr, va = W.mlp_split(len(grid))
    tr, va = np.array(tr), np.array(va)
    t0 = time.perf_counter()
    net = Surrogate(ctx, seed=W.MLP_SEED)
    hist = net.train(X[tr], obs[tr], epochs=epochs, lr=1e-3, log_targets=S.LOG_TARGETS)
    t_train = time.perf_counter() - t0
    pred = net.predict(X[va], bf16=False)
    val_rel = np.abs(pred - obs[va]) / np.maximum(np.abs(obs[va]), 1e-300)
    t0 = time.perf_counter()
    props = net.propose(nbeta=256, ndelta=256, beta_lo=0.5, beta_hi=1.5, delta_lo=0.0,
                        delta_hi=1.0, seed=W.MLP_SEED, jitter=0.5)
    t_prop = time.perf_counter() - t0
    t0 = time.perf_counter()
    ver = S.verify(ctx, net, props, dcut=64, nmax=10, nsteps=40, tol=tol, workers=workers)
    t_ver = time.perf_counter() - t0
    net.close()
    return {
        "train_points": int(len(tr)), "validation_points": int(len(va)), "epochs": epochs,
        "final_loss": float(hist[-1]), "train_seconds": t_train,
        "validation_median_rel_err": [float(x) for x in np.median(val_rel, axis=0)],
        "proposals": int(len(props)), "propose_seconds": t_prop,
        "verification_runs": int(len(props)), "verify_seconds": t_ver,
        "verify_runs_per_s": len(props) / t_ver,
        "acceptance": ver["acceptance"],
        "median_rel_err_f": float(np.median(ver["rel_err"])),
        "max_rel_err_f": float(np.max(ver["rel_err"])),
    }


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=None)
    ap.add_argument("--workers", type=int, default=16)
    ap.add_argument("--no-refine", action="store_true")
    ap.add_argument("--no-reduced", action="store_true")
    args = ap.parse_args(argv)
    ctx = Context(0)
    out = {"grid": "16 x 16 (beta, Delta), Dcut per point from {24,32,48,64}, |n| <= 10, "
                   "40 steps, zero-field route (3 runs per point)"}
    grid, obs, el = scan_grid(ctx, workers=1)
    out["plain_fp64"] = {"seconds": el, "points_per_s": len(grid) / el, "workers": 1}
    print(f"scan: plain FP64 grid {el:.1f}s", file=sys.stderr, flush=True)
    _, obs_b, el = scan_grid(ctx, workers=args.workers)
    out["batched_fp64"] = {"seconds": el, "points_per_s": len(grid) / el,
                           "workers": args.workers,
                           "same_bits_as_plain": bool(np.array_equal(obs, obs_b))}
    print(f"scan: batched FP64 grid {el:.1f}s", file=sys.stderr, flush=True)
    if not args.no_reduced:
        for name, prec, k in (("batched_fp32", W.PREC_FP32, 12),
                              ("batched_bf16x3", W.PREC_BF16X3, 16)):
            _, o2, el = scan_grid(ctx, prec=prec, fp64_steps=k, workers=args.workers)
            beta = np.array([g.beta for g in grid])
            df = np.abs(o2[:, 0] - obs[:, 0])
            out[name] = {"seconds": el, "points_per_s": len(grid) / el, "fp64_steps": k,
                         "max_abs_df": float(df.max()),
                         "max_rel_dchi": float(np.max(np.abs(o2[:, 2] - obs[:, 2]) / obs[:, 2])),
                         "max_abs_dcv": float(np.max(np.abs(o2[:, 1] - obs[:, 1])))}
            print(f"scan: {name} grid {el:.1f}s", file=sys.stderr, flush=True)
    out["observables"] = {"beta": [g.beta for g in grid], "delta": [g.delta for g in grid],
                          "dcut": [g.dcut for g in grid], "f": obs[:, 0].tolist(),
                          "cv": obs[:, 1].tolist(), "chi": obs[:, 2].tolist(),
                          "chi_n": obs[:, 3].tolist()}
    if not args.no_refine:
        out["refine"] = refine(ctx, grid, obs, workers=args.workers)
        print("scan: surrogate refinement done", file=sys.stderr, flush=True)
    ctx.close()
    line = json.dumps(out)
    if args.out:
        with open(args.out, "w") as f:
            f.write(line + "\n")
    summary = {k: v for k, v in out.items() if k != "observables"}
    print(json.dumps(summary), flush=True)


if __name__ == "__main__":
    main()
