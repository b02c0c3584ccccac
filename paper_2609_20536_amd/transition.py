"""Transition temperatures of the gXY model from HOTRG runs (host orchestration).

The thesis (Ch. 3, Sec. "Numerical Results") locates the BKT and half-BKT
transitions from susceptibility peaks in a small symmetry-breaking field and
extrapolates them to zero field, and the Ising-like transition from the peak
of the specific heat:

* the dominant order parameter picks the field: h (coupling to cos theta,
  magnetisation M) for Delta > 0.36, h1 (coupling to cos q theta, M_1) for
  Delta <= 0.36;
* chi = dM/dh by the central difference at a central field hbar (eq. susc);
  along a temperature scan at fixed hbar its maximum gives T_peak(hbar);
* T_peak(hbar) for several hbar is fitted by T = a + b hbar^c, and a is the
  zero-field critical temperature (the fit form of the thesis's reference
  for the XY model; Fig. Tc0p32 quotes a, b, c for Delta = 0.32);
* the Ising-like line: the temperature of the C_v maximum at zero field
  (C_v = beta^2 d^2(ln Z/V)/d beta^2, eq. spech).

Every HOTRG run and every finite difference runs in the library
(gxy_run_batch, gxy_observables); this module builds the run lists, finds
the peaks and does the three-parameter fit on the host.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Dict, List, Sequence, Tuple

import numpy as np

from . import workloads as W
from .hotrg import Context

FIELD_SWITCH_DELTA = 0.36   # h for Delta above it, h1 at or below it
CHI_FIELD_STEP = 1e-4       # central-difference step of the susceptibility


def field_for(delta: float) -> str:
    """'h' (M = <cos theta>) for Delta > 0.36, 'h1' (M_1 = <cos q theta>) else."""
    return "h" if delta > FIELD_SWITCH_DELTA else "h1"


def susceptibility_along_t(ctx: Context, delta: float, temps: Sequence[float], hbar: float,
                           fieldname: str, dcut: int, nmax: int, nsteps: int, q: int = 2,
                           dh: float = CHI_FIELD_STEP, workers: int = 8) -> np.ndarray:
    """chi(T) at central field hbar: two runs per temperature (hbar -+ dh),
    with the impurity chain of the chosen order parameter."""
    imp = W.IMP_COS1 if fieldname == "h" else W.IMP_COS2
    runs = []
    for t in temps:
        for s in (-dh, dh):
            kw = {fieldname: hbar + s}
            runs.append(W.Point(beta=1.0 / t, delta=delta, nmax=nmax, dcut=dcut, nsteps=nsteps,
                                impurities=imp, q=q, **kw))
    res = ctx.run_batch(runs, workers=workers)
    if any(r.status != 0 for r in res):
        raise RuntimeError("HOTRG run failed")
    n = len(temps)
    m = np.array([[getattr(res[2 * k + j], "m_cos1" if imp == W.IMP_COS1 else "m_cos2")
                   for j in range(2)] for k in range(n)])
    beta = 1.0 / np.asarray(temps, dtype=np.float64)
    zero3, zero2 = np.zeros((n, 3)), np.zeros((n, 2))
    if imp == W.IMP_COS1:
        out = ctx.observables(beta, zero3, m, zero2, 1.0, dh, 1.0)
        return out[:, 2]
    out = ctx.observables(beta, zero3, zero2, m, 1.0, 1.0, dh)
    return out[:, 3]


def cv_along_t(ctx: Context, delta: float, temps: Sequence[float], dcut: int, nmax: int,
               nsteps: int, q: int = 2, db: float = W.BETA_FD_STEP,
               workers: int = 8) -> np.ndarray:
    """C_v(T) at zero field from three runs per temperature (beta, beta -+ db)."""
    betas = 1.0 / np.asarray(temps, dtype=np.float64)
    runs = [W.Point(beta=b + s, delta=delta, nmax=nmax, dcut=dcut, nsteps=nsteps, impurities=0,
                    q=q) for b in betas for s in (-db, 0.0, db)]
    res = ctx.run_batch(runs, workers=workers)
    if any(r.status != 0 for r in res):
        raise RuntimeError("HOTRG run failed")
    n = len(betas)
    lnz = np.array([[res[3 * k + j].lnz_per_site for j in range(3)] for k in range(n)])
    zero = np.zeros((n, 2))
    return ctx.observables(betas, lnz, zero, zero, db, 1.0, 1.0)[:, 1]


def vertex(x: Sequence[float], y: Sequence[float]) -> float:
    """Abscissa of the maximum: the vertex of the parabola through the
    largest sample and its two neighbours (the sample itself at the ends or
    where the three points are not concave)."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    i = int(np.argmax(y))
    if i == 0 or i == len(y) - 1:
        return float(x[i])
    # divided differences of the three points
    d1 = (y[i] - y[i - 1]) / (x[i] - x[i - 1])
    d2 = (y[i + 1] - y[i]) / (x[i + 1] - x[i])
    curv = (d2 - d1) / (x[i + 1] - x[i - 1])
    if not curv < 0.0:
        return float(x[i])
    # p(x) = y_{i-1} + d1 (x - x_{i-1}) + curv (x - x_{i-1})(x - x_i)
    return float(0.5 * (x[i - 1] + x[i]) - 0.5 * d1 / curv)


def fit_power_law(hbars: Sequence[float], tpeaks: Sequence[float],
                  c_range: Tuple[float, float] = (0.02, 3.0)) -> Tuple[float, float, float, float]:
    """Least-squares fit T = a + b hbar^c. For fixed c the fit is linear in
    (a, b); c minimises the residual on c_range (golden-section search on a
    bracket found by a coarse scan). Returns (a, b, c, rms residual)."""
    h = np.asarray(hbars, dtype=np.float64)
    t = np.asarray(tpeaks, dtype=np.float64)
    if len(h) < 3:
        raise ValueError("need at least three central fields")

    def lin(c):
        A = np.stack([np.ones_like(h), h ** c], axis=1)
        coef, *_ = np.linalg.lstsq(A, t, rcond=None)
        r = A @ coef - t
        return float(r @ r), coef

    grid = np.linspace(c_range[0], c_range[1], 300)
    vals = [lin(c)[0] for c in grid]
    k = int(np.argmin(vals))
    lo, hi = grid[max(k - 1, 0)], grid[min(k + 1, len(grid) - 1)]
    g = (math.sqrt(5.0) - 1.0) / 2.0
    x1, x2 = hi - g * (hi - lo), lo + g * (hi - lo)
    f1, f2 = lin(x1)[0], lin(x2)[0]
    for _ in range(100):
        if f1 <= f2:
            hi, x2, f2 = x2, x1, f1
            x1 = hi - g * (hi - lo)
            f1 = lin(x1)[0]
        else:
            lo, x1, f1 = x1, x2, f2
            x2 = lo + g * (hi - lo)
            f2 = lin(x2)[0]
    c = 0.5 * (lo + hi)
    ss, (a, b) = lin(c)
    return float(a), float(b), float(c), math.sqrt(ss / len(h))


@dataclass
class Transition:
    delta: float
    field: str
    hbars: List[float]
    tpeaks: List[float]
    a: float                 # zero-field critical temperature
    b: float
    c: float
    rms: float
    t_cv: float              # temperature of the zero-field C_v maximum
    chi: Dict[float, List[float]] = field(default_factory=dict)
    cv: List[float] = field(default_factory=list)


def transition_temperature(ctx: Context, delta: float, temps: Sequence[float],
                           hbars: Sequence[float], dcut: int, nmax: int, nsteps: int,
                           q: int = 2, workers: int = 8) -> Transition:
    """T_c(Delta) by the thesis's procedure: chi peaks at each central field,
    the fit T_peak = a + b hbar^c (T_c = a), and the zero-field C_v peak."""
    fld = field_for(delta)
    chis, tp = {}, []
    for hb in hbars:
        chi = susceptibility_along_t(ctx, delta, temps, hb, fld, dcut, nmax, nsteps, q=q,
                                     workers=workers)
        chis[float(hb)] = [float(v) for v in chi]
        tp.append(vertex(temps, chi))
    a, b, c, rms = fit_power_law(hbars, tp)
    cv = cv_along_t(ctx, delta, temps, dcut, nmax, nsteps, q=q, workers=workers)
    return Transition(delta, fld, [float(x) for x in hbars], tp, a, b, c, rms,
                      vertex(temps, cv), chis, [float(v) for v in cv])
