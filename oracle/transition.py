"""FP64 CPU oracle of the transition-temperature procedure (plain numpy/scipy).

TEST INFRASTRUCTURE ONLY: the reference the GPU pipeline is checked against.
It shares no code with the library or its Python package; only the test
suite may import it.

The procedure (Ch. 3, Sec. "Numerical Results"): the field that couples to
the dominant order parameter is h (cos theta) for Delta > 0.36 and h1
(cos q theta) otherwise; the susceptibility chi = dM/dh is the central
difference of the impurity expectation value at hbar -+ dh (eq. susc); its
maximum along a temperature scan gives T_peak(hbar); T_peak(hbar) over
several central fields is fitted by a + b hbar^c, a being the zero-field
critical temperature; the Ising-like transition is the temperature of the
zero-field C_v maximum (eq. spech). Each step follows the definition with a
library routine where one applies: the parabola through the three samples
around the maximum by numpy.polyfit, the three-parameter fit by
scipy.optimize.curve_fit.

Pinned by: exact parabolas and exact power laws (tests/test_oracle_transition.py);
the runs themselves are the pinned HOTRG oracle.
"""

from __future__ import annotations

import math
from typing import Dict, List, Sequence

import numpy as np
from scipy.optimize import curve_fit

from . import hotrg as o


def chi_scan(delta: float, temps: Sequence[float], hbar: float, use_h: bool, dcut: int,
             nmax: int, nsteps: int, q: int = 2, dh: float = 1e-4) -> np.ndarray:
    """chi(T) = [M(hbar + dh) - M(hbar - dh)] / (2 dh) at beta = 1/T."""
    out = []
    for t in temps:
        ms = []
        for s in (-dh, dh):
            if use_h:
                r = o.run_point(1.0 / t, delta, h=hbar + s, nmax=nmax, dcut=dcut, nsteps=nsteps,
                                impurities=o.IMP_COS1, q=q)
                ms.append(r.m_cos1)
            else:
                r = o.run_point(1.0 / t, delta, h1=hbar + s, nmax=nmax, dcut=dcut,
                                nsteps=nsteps, impurities=o.IMP_COS2, q=q)
                ms.append(r.m_cos2)
        out.append((ms[1] - ms[0]) / (2.0 * dh))
    return np.array(out)


def cv_scan(delta: float, temps: Sequence[float], dcut: int, nmax: int, nsteps: int,
            q: int = 2, db: float = 1e-3) -> np.ndarray:
    """C_v(T) = beta^2 [l(beta - db) - 2 l(beta) + l(beta + db)] / db^2, l = ln Z/V."""
    out = []
    for t in temps:
        b = 1.0 / t
        l = [o.run_point(b + s, delta, nmax=nmax, dcut=dcut, nsteps=nsteps, impurities=0,
                         q=q).lnz_per_site for s in (-db, 0.0, db)]
        out.append(b * b * (l[0] - 2.0 * l[1] + l[2]) / (db * db))
    return np.array(out)


def peak(temps: Sequence[float], y: Sequence[float]) -> float:
    """Maximum of the parabola through the largest sample and its neighbours;
    the sample itself at the ends of the scan or without concavity."""
    t = np.asarray(temps, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    i = int(np.argmax(y))
    if i == 0 or i == len(y) - 1:
        return float(t[i])
    c2, c1, _ = np.polyfit(t[i - 1:i + 2], y[i - 1:i + 2], 2)
    if not c2 < 0.0:
        return float(t[i])
    return float(-c1 / (2.0 * c2))


def fit_tc(hbars: Sequence[float], tpeaks: Sequence[float]) -> Dict[str, float]:
    """Least-squares a + b hbar^c through (hbar, T_peak); T_c = a."""
    h = np.asarray(hbars, dtype=np.float64)
    t = np.asarray(tpeaks, dtype=np.float64)

    def model(x, a, b, c):
        return a + b * np.power(x, c)

    p0 = (float(t.min()), float((t.max() - t.min()) / max(h.max() ** 0.5, 1e-300)), 0.5)
    (a, b, c), _ = curve_fit(model, h, t, p0=p0, maxfev=20000, xtol=1e-14, ftol=1e-14)
    res = model(h, a, b, c) - t
    return {"a": float(a), "b": float(b), "c": float(c),
            "rms": float(math.sqrt(float(res @ res) / len(h)))}


def transition(delta: float, temps: Sequence[float], hbars: Sequence[float], dcut: int,
               nmax: int, nsteps: int, q: int = 2) -> Dict[str, object]:
    use_h = delta > 0.36
    tp: List[float] = []
    chis = {}
    for hb in hbars:
        chi = chi_scan(delta, temps, hb, use_h, dcut, nmax, nsteps, q)
        chis[float(hb)] = chi
        tp.append(peak(temps, chi))
    fit = fit_tc(hbars, tp)
    cv = cv_scan(delta, temps, dcut, nmax, nsteps, q)
    return {"field": "h" if use_h else "h1", "tpeaks": tp, "chi": chis, "cv": cv,
            "t_cv": peak(temps, cv), **fit}
