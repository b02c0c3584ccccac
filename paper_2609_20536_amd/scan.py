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

    python -m paper_2609_20536_amd.scan [--passes plain,fp64,fp32,bf16x3]
        [--refine] [--reference earlier.json] [--out results.json]
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
              workers: int = 16, grid=None, chunk: int = 64, label: str = ""):
    """Observables of the grid in chunks of `chunk` points (one batch each,
    a progress line after each); returns the grid, the (n, 4) array and the
    summed batch time."""
    grid = W.grid_points() if grid is None else grid
    parts, el = [], 0.0
    for c0 in range(0, len(grid), chunk):
        t0 = time.perf_counter()
        obs, _ = S.grid_observables_zero_field(ctx, grid[c0:c0 + chunk], workers=workers,
                                               prec=prec, fp64_steps=fp64_steps)
        el += time.perf_counter() - t0
        parts.append(obs)
        print(f"scan: {label} points {c0 + len(obs)}/{len(grid)} ({el:.1f}s)",
              file=sys.stderr, flush=True)
    return grid, np.concatenate(parts), el


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
    t_ver, rel = 0.0, []
    for c0 in range(0, len(props), 128):
        t0 = time.perf_counter()
        ver = S.verify(ctx, net, props[c0:c0 + 128], dcut=64, nmax=10, nsteps=40, tol=tol,
                       workers=workers)
        t_ver += time.perf_counter() - t0
        rel.append(ver["rel_err"])
        print(f"scan: verified {c0 + len(ver['rel_err'])}/{len(props)} ({t_ver:.1f}s)",
              file=sys.stderr, flush=True)
    rel = np.concatenate(rel)
    net.close()
    return {
        "train_points": int(len(tr)), "validation_points": int(len(va)), "epochs": epochs,
        "final_loss": float(hist[-1]), "train_seconds": t_train,
        "validation_median_rel_err": [float(x) for x in np.median(val_rel, axis=0)],
        "proposals": int(len(props)), "propose_seconds": t_prop,
        "verification_runs": int(len(props)), "verify_seconds": t_ver,
        "verify_runs_per_s": len(props) / t_ver,
        "acceptance": float(np.mean(rel <= tol)),
        "median_rel_err_f": float(np.median(rel)),
        "max_rel_err_f": float(np.max(rel)),
    }


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=None)
    ap.add_argument("--workers", type=int, default=16)
    ap.add_argument("--passes", default="plain,fp64,fp32,bf16x3",
                    help="comma list of plain (FP64, one run after another), fp64, fp32, "
                         "bf16x3 (batched)")
    ap.add_argument("--refine", action="store_true", help="train, propose and verify")
    ap.add_argument("--reference", default=None,
                    help="JSON of an earlier FP64 scan: its observables are the reference")
    args = ap.parse_args(argv)
    passes = [x for x in args.passes.split(",") if x]
    ctx = Context(0)
    out = {"grid": "16 x 16 (beta, Delta), Dcut per point from {24,32,48,64}, |n| <= 10, "
                   "40 steps, zero-field route (3 runs per point)"}
    ref = None
    if args.reference:
        with open(args.reference) as f:
            o = json.load(f)["observables"]
        ref = np.stack([o["f"], o["cv"], o["chi"], o["chi_n"]], axis=1)
    grid = W.grid_points()
    forms = {"plain": (W.PREC_FP64, 0, 1), "fp64": (W.PREC_FP64, 0, args.workers),
             "fp32": (W.PREC_FP32, 12, args.workers), "bf16x3": (W.PREC_BF16X3, 16, args.workers)}
    for name in passes:
        prec, k, workers = forms[name]
        _, obs, el = scan_grid(ctx, prec=prec, fp64_steps=k, workers=workers, label=name)
        row = {"seconds": el, "points_per_s": len(grid) / el, "workers": workers,
               "fp64_steps": k}
        if ref is None and prec == W.PREC_FP64:
            ref = obs
        elif ref is not None:
            row["max_abs_df_vs_fp64"] = float(np.max(np.abs(obs[:, 0] - ref[:, 0])))
            row["max_abs_dcv_vs_fp64"] = float(np.max(np.abs(obs[:, 1] - ref[:, 1])))
            row["max_rel_dchi_vs_fp64"] = float(np.max(np.abs(obs[:, 2] - ref[:, 2]) / ref[:, 2]))
            row["max_rel_dchin_vs_fp64"] = float(np.max(np.abs(obs[:, 3] - ref[:, 3]) / ref[:, 3]))
        out[name] = row
    if ref is not None:
        out["observables"] = {"beta": [g.beta for g in grid], "delta": [g.delta for g in grid],
                              "dcut": [g.dcut for g in grid], "f": ref[:, 0].tolist(),
                              "cv": ref[:, 1].tolist(), "chi": ref[:, 2].tolist(),
                              "chi_n": ref[:, 3].tolist()}
    if args.refine and ref is not None:
        out["refine"] = refine(ctx, grid, ref, workers=args.workers)
        print("scan: surrogate refinement done", file=sys.stderr, flush=True)
    ctx.close()
    if args.out:
        with open(args.out, "w") as f:
            f.write(json.dumps(out) + "\n")
    print(json.dumps({k: v for k, v in out.items() if k != "observables"}), flush=True)


if __name__ == "__main__":
    main()
