"""Surrogate-guided scans of the gXY phase diagram (host orchestration).

Every computation runs in the library: HOTRG runs (gxy_run_batch), the
finite-difference observables (gxy_observables), and the MLP's training,
inference and proposals (gxy_mlp_*). This module only assembles the run
lists and the arrays passed between them.

Pipeline:
1. observables (f, C_v, chi, chi_n) on a (beta, Delta) grid from seven HOTRG
   runs per point (Ch. 3, eqs. spech, susc; central differences);
2. train the surrogate on them (chi and chi_n through their logarithms);
3. propose, per Delta of a fine lattice, the beta of the predicted C_v and
   chi maxima;
4. verify proposals by HOTRG (free energy at zero field): a proposal is
   accepted when the predicted f is within 1e-3 (relative) of HOTRG's,
   otherwise HOTRG's value stands.

gain_experiment measures what the surrogate buys: the error of the C_v peak
location along beta at fixed Delta, from the same number of HOTRG points
spent uniformly over the beta range or inside a window around the
surrogate's proposal.
"""

from __future__ import annotations

from typing import Dict, List, Sequence, Tuple

import numpy as np

from . import workloads as W
from .hotrg import Context, Surrogate

LOG_TARGETS = 0b1100   # chi, chi_n enter the network as logarithms


def grid_observables(ctx: Context, points: Sequence[Tuple[float, float]], dcut: int,
                     nmax: int = 10, nsteps: int = 40, workers: int = 8,
                     prec: int = W.PREC_FP64, fp64_steps: int = 0,
                     db: float = W.BETA_FD_STEP) -> np.ndarray:
    """(f, C_v, chi, chi_n) for each (beta, Delta); seven runs per point."""
    runs = []
    for b, d in points:
        runs += W.observable_runs(b, d, dcut, nmax, nsteps, prec, fp64_steps, db)
    res = ctx.run_batch(runs, workers=workers)
    bad = [i for i, r in enumerate(res) if r.status != 0]
    if bad:
        raise RuntimeError(f"{len(bad)} HOTRG runs failed (first: {runs[bad[0]]})")
    n = len(points)
    lnz = np.array([[res[7 * k + j].lnz_per_site for j in range(3)] for k in range(n)])
    mh = np.array([[res[7 * k + 3 + j].m_cos1 for j in range(2)] for k in range(n)])
    mh1 = np.array([[res[7 * k + 5 + j].m_cos2 for j in range(2)] for k in range(n)])
    beta = np.array([p[0] for p in points], dtype=np.float64)
    return ctx.observables(beta, lnz, mh, mh1, db, W.FIELD_FD_STEP, W.FIELD_FD_STEP)


def grid_observables_zero_field(ctx: Context, grid: Sequence, workers: int = 16,
                                prec: int = W.PREC_FP64, fp64_steps: int = 0,
                                nmax: int = 10, nsteps: int = 40,
                                db: float = W.BETA_FD_STEP) -> Tuple[np.ndarray, list]:
    """(f, C_v, chi, chi_n) for grid points with their own Dcut (objects with
    beta, delta, dcut), three runs per point (W.zero_field_runs): C_v by the
    library's central difference, chi and chi_n at zero field from the
    second-moment chains. Returns the (n, 4) array and the run results."""
    runs = []
    for g in grid:
        runs += W.zero_field_runs(g.beta, g.delta, g.dcut, nmax, nsteps, prec, fp64_steps, db)
    res = ctx.run_batch(runs, workers=workers)
    bad = [i for i, r in enumerate(res) if r.status != 0]
    if bad:
        raise RuntimeError(f"{len(bad)} HOTRG runs failed (first: {runs[bad[0]]})")
    n = len(grid)
    lnz = np.array([[res[3 * k + j].lnz_per_site for j in range(3)] for k in range(n)])
    zero = np.zeros((n, 2))
    beta = np.array([g.beta for g in grid], dtype=np.float64)
    obs = ctx.observables(beta, lnz, zero, zero, db, 1.0, 1.0)
    obs[:, 2] = [res[3 * k + 1].chi0 for k in range(n)]
    obs[:, 3] = [res[3 * k + 1].chi0_n for k in range(n)]
    return obs, res


def cv_along_beta(ctx: Context, delta: float, betas: Sequence[float], dcut: int,
                  nmax: int, nsteps: int, workers: int = 8,
                  db: float = W.BETA_FD_STEP) -> np.ndarray:
    """C_v(beta) at zero field from three runs per beta (beta, beta +- db)."""
    runs = [W.Point(beta=b + s, delta=delta, nmax=nmax, dcut=dcut, nsteps=nsteps, impurities=0)
            for b in betas for s in (-db, 0.0, db)]
    res = ctx.run_batch(runs, workers=workers)
    if any(r.status != 0 for r in res):
        raise RuntimeError("HOTRG run failed")
    lnz = np.array([[res[3 * k + j].lnz_per_site for j in range(3)] for k in range(len(betas))])
    zero = np.zeros((len(betas), 2))
    return ctx.observables(np.asarray(betas, dtype=np.float64), lnz, zero, zero, db, 1.0,
                           1.0)[:, 1]


def peak_location(x: np.ndarray, y: np.ndarray) -> float:
    """Vertex of the parabola through the largest sample and its neighbours
    (the sample itself at the ends)."""
    i = int(np.argmax(y))
    if i == 0 or i == len(y) - 1:
        return float(x[i])
    x0, x1, x2 = x[i - 1], x[i], x[i + 1]
    y0, y1, y2 = y[i - 1], y[i], y[i + 1]
    den = (x0 - x1) * (x0 - x2) * (x1 - x2)
    a = (x2 * (y1 - y0) + x1 * (y0 - y2) + x0 * (y2 - y1)) / den
    b = (x2 * x2 * (y0 - y1) + x1 * x1 * (y2 - y0) + x0 * x0 * (y1 - y2)) / den
    if a >= 0.0:
        return float(x1)
    return float(-b / (2.0 * a))


def train(ctx: Context, X: np.ndarray, Y: np.ndarray, epochs: int = 5000,
          seed: int = W.MLP_SEED) -> Tuple[Surrogate, np.ndarray]:
    net = Surrogate(ctx, seed=seed)
    hist = net.train(X, Y, epochs=epochs, lr=1e-3, log_targets=LOG_TARGETS)
    return net, hist


def verify(ctx: Context, net: Surrogate, proposals: np.ndarray, dcut: int = 64,
           nmax: int = 10, nsteps: int = 40, tol: float = 1e-3,
           workers: int = 8) -> Dict[str, object]:
    """HOTRG free energy at each proposal (zero field, FP64) against the
    surrogate's prediction; accepted where the relative error is <= tol."""
    runs = [W.Point(beta=float(b), delta=float(d), nmax=nmax, dcut=dcut, nsteps=nsteps,
                    impurities=0) for b, d in proposals]
    res = ctx.run_batch(runs, workers=workers)
    f_hotrg = np.array([-r.lnz_per_site / p.beta for r, p in zip(res, runs)])
    f_pred = net.predict(proposals, bf16=True)[:, 0]
    rel = np.abs(f_pred - f_hotrg) / np.abs(f_hotrg)
    accepted = rel <= tol
    return {"f_hotrg": f_hotrg, "f_pred": f_pred, "rel_err": rel, "accepted": accepted,
            "acceptance": float(np.mean(accepted)),
            "f_final": np.where(accepted, f_pred, f_hotrg)}


def gain_experiment(ctx: Context, deltas: Sequence[float] = (0.3, 0.6, 0.9),
                    dcut: int = 16, nmax: int = 5, nsteps: int = 24,
                    train_grid: Tuple[int, int] = (21, 6), budget: int = 6,
                    reference_points: int = 41, beta_range: Tuple[float, float] = (0.5, 1.5),
                    epochs: int = 5000, workers: int = 8,
                    window: float = 2.0, db: float = 0.02) -> Dict[str, object]:
    """C_v peak location along beta at fixed Delta, uniform vs surrogate-guided.

    Reference: the peak from a dense scan (reference_points betas). Uniform:
    `budget` betas spread over the whole range. Guided: the surrogate is
    trained on a coarse (beta, Delta) grid of observables, proposes the C_v
    maximum at each Delta, and the same `budget` betas are spread over
    `window` coarse-grid spacings on either side of it. Both estimates use the
    parabola vertex through the largest sample and its neighbours.

    C_v here is the central second difference with step db = 0.02 (the
    scans' 1e-3 turns each change of the kept states between beta - db and
    beta + db into a spike of order (jump in ln Z/V) / db^2; a wider step
    damps those spikes by (0.02 / 0.001)^2 = 400 on the same smooth curve).
    """
    lo, hi = beta_range
    nb, nd = train_grid
    grid = [(lo + (hi - lo) * i / (nb - 1), j / (nd - 1)) for i in range(nb) for j in range(nd)]
    Y = grid_observables(ctx, grid, dcut, nmax, nsteps, workers, db=db)
    X = np.array(grid)
    net, hist = train(ctx, X, Y, epochs=epochs)
    out = {"deltas": list(deltas), "budget": budget, "train_points": len(grid),
           "final_loss": float(hist[-1]), "rows": []}
    spacing = (hi - lo) / (nb - 1)
    for d in deltas:
        ref_b = np.linspace(lo, hi, reference_points)
        ref = peak_location(ref_b, cv_along_beta(ctx, d, ref_b, dcut, nmax, nsteps, workers, db))
        uni_b = np.linspace(lo, hi, budget)
        uni = peak_location(uni_b, cv_along_beta(ctx, d, uni_b, dcut, nmax, nsteps, workers, db))
        lat = np.stack([np.linspace(lo, hi, 256), np.full(256, d)], axis=1)
        pred = net.predict(lat, bf16=True)
        bp = peak_location(lat[:, 0], pred[:, 1])
        g_lo, g_hi = max(lo, bp - window * spacing), min(hi, bp + window * spacing)
        gui_b = np.linspace(g_lo, g_hi, budget)
        gui = peak_location(gui_b, cv_along_beta(ctx, d, gui_b, dcut, nmax, nsteps, workers, db))
        out["rows"].append({"delta": d, "reference": ref, "uniform": uni, "proposed": bp,
                            "guided": gui, "err_uniform": abs(uni - ref),
                            "err_guided": abs(gui - ref)})
    eu = np.mean([r["err_uniform"] for r in out["rows"]])
    eg = np.mean([r["err_guided"] for r in out["rows"]])
    out["mean_err_uniform"] = float(eu)
    out["mean_err_guided"] = float(eg)
    out["gain"] = float(eu / max(eg, 1e-15))
    net.close()
    return out
