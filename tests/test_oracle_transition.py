"""Pins of the transition-temperature oracle (oracle/transition.py) and of
the package's host-side peak and fit (paper_2609_20536_amd/transition.py),
each against exact synthetic data: parabolas with a known vertex and power
laws T = a + b hbar^c with known parameters (the values the thesis quotes
for Delta = 0.32 among them); and the package's run lists and finite
differences against a stand-in context with known M(h) and ln Z(beta).
No GPU."""

import numpy as np
import pytest

from oracle import transition as ot
from paper_2609_20536_amd import transition as pt

TEMPS = np.round(np.arange(0.55, 1.31, 0.05), 4)


@pytest.mark.parametrize("top", [0.6123, 0.83, 1.0071, 1.2])
def test_peak_of_exact_parabola(top):
    y = 3.0 - 7.5 * (TEMPS - top) ** 2
    assert ot.peak(TEMPS, y) == pytest.approx(top, abs=1e-12)
    assert pt.vertex(TEMPS, y) == pytest.approx(top, abs=1e-12)


def test_peak_at_the_end_of_the_scan_is_the_end_sample():
    y = TEMPS.copy()                        # increasing: maximum at the last sample
    assert ot.peak(TEMPS, y) == TEMPS[-1] and pt.vertex(TEMPS, y) == TEMPS[-1]
    assert ot.peak(TEMPS, -y) == TEMPS[0] and pt.vertex(TEMPS, -y) == TEMPS[0]


@pytest.mark.parametrize("a,b,c", [(0.685, 0.48, 0.29), (0.893, 1.7, 0.6), (0.72, 0.2, 1.1)])
def test_power_law_fit_recovers_exact_parameters(a, b, c):
    h = np.array([1e-3, 2e-3, 4e-3, 8e-3, 1.6e-2, 3.2e-2])
    t = a + b * h ** c
    fo = ot.fit_tc(h, t)
    assert fo["a"] == pytest.approx(a, abs=1e-7)
    assert fo["b"] == pytest.approx(b, rel=1e-6)
    assert fo["c"] == pytest.approx(c, abs=1e-6)
    fa, fb, fc, rms = pt.fit_power_law(h, t)
    assert fa == pytest.approx(a, abs=1e-7) and fb == pytest.approx(b, rel=1e-6)
    assert fc == pytest.approx(c, abs=1e-6) and rms < 1e-9


def test_power_law_fits_agree_on_noisy_data():
    """Both fits minimise the same sum of squares: on data off the model they
    reach the same (a, b, c) (a well-posed case: c away from 0)."""
    rng = np.random.default_rng(3)
    h = np.array([1e-3, 2e-3, 4e-3, 8e-3, 1.6e-2, 3.2e-2])
    t = 0.7 + 0.5 * h ** 0.35 + 1e-4 * rng.standard_normal(len(h))
    fo = ot.fit_tc(h, t)
    fa, fb, fc, _ = pt.fit_power_law(h, t)
    assert fa == pytest.approx(fo["a"], abs=1e-6) and fc == pytest.approx(fo["c"], abs=1e-5)


def test_field_choice_follows_the_dominant_order_parameter():
    assert pt.field_for(0.6) == "h" and pt.field_for(0.36) == "h1" and pt.field_for(0.1) == "h1"


class _FakeCtx:
    """Stands in for the library context: records the run list and answers
    with m = 2 h (or 3 h1) and ln Z/V = beta^3, and does the central
    differences of gxy_observables in numpy."""

    def __init__(self):
        self.points = []

    def run_batch(self, pts, workers=1):
        from types import SimpleNamespace
        self.points = list(pts)
        return [SimpleNamespace(status=0, m_cos1=2.0 * p.h, m_cos2=3.0 * p.h1,
                                lnz_per_site=p.beta ** 3) for p in pts]

    def observables(self, beta, lnz, m_h, m_h1, dbeta, dh, dh1):
        out = np.empty((len(beta), 4))
        out[:, 0] = -lnz[:, 1] / beta
        out[:, 1] = beta ** 2 * (lnz[:, 2] - 2 * lnz[:, 1] + lnz[:, 0]) / dbeta ** 2
        out[:, 2] = (m_h[:, 1] - m_h[:, 0]) / (2 * dh)
        out[:, 3] = (m_h1[:, 1] - m_h1[:, 0]) / (2 * dh1)
        return out


def test_susceptibility_run_list_and_differences():
    """Two runs per temperature at hbar -+ dh of the chosen field, with the
    matching impurity chain; chi = dM/dh of the fake M."""
    from paper_2609_20536_amd import workloads as W
    temps = [0.7, 0.9]
    for fld, imp, slope in (("h", W.IMP_COS1, 2.0), ("h1", W.IMP_COS2, 3.0)):
        c = _FakeCtx()
        chi = pt.susceptibility_along_t(c, 0.5, temps, 0.004, fld, dcut=8, nmax=3, nsteps=6, q=3)
        assert np.allclose(chi, slope, rtol=1e-9)
        assert len(c.points) == 4
        for k, p in enumerate(c.points):
            assert p.beta == pytest.approx(1.0 / temps[k // 2]) and p.impurities == imp and p.q == 3
            f = getattr(p, fld)
            assert f == pytest.approx(0.004 + (-1e-4 if k % 2 == 0 else 1e-4))
            assert getattr(p, "h1" if fld == "h" else "h") == 0.0


def test_cv_run_list_and_differences():
    """Three zero-field runs per temperature at beta -+ db; C_v of
    ln Z/V = beta^3 is beta^2 * 6 beta."""
    c = _FakeCtx()
    temps = [0.8, 1.25]
    cv = pt.cv_along_t(c, 0.4, temps, dcut=8, nmax=3, nsteps=6)
    b = 1.0 / np.array(temps)
    assert np.allclose(cv, b ** 2 * 6.0 * b, rtol=1e-6)
    assert len(c.points) == 6 and all(p.impurities == 0 and p.h == 0 and p.h1 == 0 for p in c.points)
