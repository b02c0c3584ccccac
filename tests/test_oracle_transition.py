"""Pins of the transition-temperature oracle (oracle/transition.py) and of
the package's host-side peak and fit (paper_2609_20536_amd/transition.py),
each against exact synthetic data: parabolas with a known vertex and power
laws T = a + b hbar^c with known parameters (the values the thesis quotes
for Delta = 0.32 among them). No GPU."""

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
