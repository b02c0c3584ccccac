"""Pins of the oracle's finite-difference observables against exact derivatives.

The specific heat C_v = beta^2 d^2(ln Z/V)/d beta^2 (Ch. 3, eq. spech) and the
susceptibilities chi = d<cos theta>/dh, chi_n = d<cos 2 theta>/dh1 (eqs. susc,
mag) are formed by the oracle from central differences of runs. Here they are
checked against the exact derivatives of the same lattice integral on the
2 x 2 periodic torus, where untruncated HOTRG is exact:

* C_v from the product rule on Z(beta) = sum over a K^4 angle grid of the
  bond weights, with d t_n / d beta and d^2 t_n / d beta^2 taken from the
  Bessel-product series (scipy's I_k and I_k' = (I_{k-1} + I_{k+1}) / 2);
* chi from the fluctuation formula d<cos theta_A>/dh =
  beta (<cos theta_A S> - <cos theta_A><S>), S = sum_i cos theta_i, by the
  same grid (likewise chi_n with cos 2 theta and h1).

The bond weights are trigonometric polynomials of degree 2 nmax, so the
trapezoid rule on K = 32 points is exact for the zero-field integrands.
A dropped beta^2, a step of dh in place of 2 dh or a wrong sign fails here;
the mutation tests at the end plant those mistakes in the oracle.
"""

import math

import numpy as np
import pytest
from scipy.special import iv

import oracle.hotrg as o
import oracle.transition as ot

NMAX = 3
K = 32
M_SUM = 40   # terms of the Bessel-product series


# --------------------------------------------------------------------------
# independent helpers (scipy Bessel functions and an angle grid; no oracle code)
# --------------------------------------------------------------------------

def _coeff_derivs(beta, delta, nmax=NMAX):
    """t_n, dt_n/dbeta, d^2t_n/dbeta^2 for n = -nmax..nmax from
    t_n = sum_m I_{n-2m}(beta Delta) I_m(beta (1 - Delta))."""
    a, b = beta * delta, beta * (1.0 - delta)

    def I(k, x, der):
        if der == 0:
            return iv(k, x)
        if der == 1:
            return 0.5 * (iv(k - 1, x) + iv(k + 1, x))
        return 0.25 * (iv(k - 2, x) + 2.0 * iv(k, x) + iv(k + 2, x))

    out = np.zeros((3, 2 * nmax + 1))
    for i, n in enumerate(range(-nmax, nmax + 1)):
        for m in range(-M_SUM, M_SUM + 1):
            k = n - 2 * m
            f0, f1, f2 = I(k, a, 0), I(k, a, 1), I(k, a, 2)
            g0, g1, g2 = I(m, b, 0), I(m, b, 1), I(m, b, 2)
            out[0, i] += f0 * g0
            out[1, i] += delta * f1 * g0 + (1 - delta) * f0 * g1
            out[2, i] += (delta ** 2 * f2 * g0 + 2 * delta * (1 - delta) * f1 * g1
                          + (1 - delta) ** 2 * f0 * g2)
    return out


def _grid():
    th = 2 * np.pi * np.arange(K) / K
    return np.meshgrid(th, th, th, th, indexing="ij")   # angles of sites A, B, C, D


def _bond(coef, phi):
    n = np.arange(-NMAX, NMAX + 1)
    return np.tensordot(np.cos(np.multiply.outer(phi, n)), coef, axes=([-1], [0]))


def exact_cv_per_site(beta, delta):
    """beta^2 d^2(ln Z / 4)/d beta^2 on the 2x2 torus, character-truncated at
    |n| <= NMAX. Each of the four neighbour pairs (A,B), (C,D), (A,C), (B,D)
    is joined by two bonds, so its factor is u = w^2."""
    c = _coeff_derivs(beta, delta)
    A, B, C, D = _grid()
    u, du, d2u = [], [], []
    for phi in (A - B, C - D, A - C, B - D):
        w, w1, w2 = (_bond(c[j], phi) for j in range(3))
        u.append(w * w)
        du.append(2 * w * w1)
        d2u.append(2 * (w1 * w1 + w * w2))
    Z = np.sum(u[0] * u[1] * u[2] * u[3])
    Z1 = Z2 = 0.0
    for j in range(4):
        rest = np.prod([u[i] for i in range(4) if i != j], axis=0)
        Z1 += np.sum(du[j] * rest)
        Z2 += np.sum(d2u[j] * rest)
        for k in range(j + 1, 4):
            rest2 = np.prod([u[i] for i in range(4) if i not in (j, k)], axis=0)
            Z2 += 2.0 * np.sum(du[j] * du[k] * rest2)
    d2lnz = Z2 / Z - (Z1 / Z) ** 2
    return beta * beta * d2lnz / 4.0


def exact_chi(beta, delta, h, h1, harmonic):
    """d<cos(harmonic theta)>/dh (harmonic 1) or /dh1 (harmonic 2) on the 2x2
    torus by the fluctuation formula, with site weight
    exp(beta h cos theta + beta h1 cos 2 theta)."""
    c = _coeff_derivs(beta, delta)
    A, B, C, D = _grid()
    wt = np.ones_like(A)
    for phi in (A - B, C - D, A - C, B - D):
        wt = wt * _bond(c[0], phi) ** 2
    for x in (A, B, C, D):
        wt = wt * np.exp(beta * h * np.cos(x) + beta * h1 * np.cos(2 * x))
    obs = np.cos(harmonic * A)
    S = sum(np.cos(harmonic * x) for x in (A, B, C, D))
    Z = wt.sum()
    mean_o = (wt * obs).sum() / Z
    mean_s = (wt * S).sum() / Z
    return beta * ((wt * obs * S).sum() / Z - mean_o * mean_s)


def _exact_torus(beta, delta, h=0.0, h1=0.0, imps=0):
    return o.run_point(beta, delta, h=h, h1=h1, nmax=NMAX, dcut=10 ** 9, nsteps=2,
                       impurities=imps)


# --------------------------------------------------------------------------
# the helpers themselves
# --------------------------------------------------------------------------

def test_helper_coefficients_match_quadrature_and_its_derivative():
    """The series t_n and its beta-derivative agree with the 4096-point
    quadrature of w and of d w / d beta = [Delta cos + (1-Delta) cos 2] w."""
    beta, delta = 0.7, 0.6
    c = _coeff_derivs(beta, delta)
    phi = 2 * np.pi * np.arange(4096) / 4096
    hh = delta * np.cos(phi) + (1 - delta) * np.cos(2 * phi)
    n = np.arange(-NMAX, NMAX + 1)
    cosn = np.cos(np.multiply.outer(n, phi))
    assert np.allclose(c[0], cosn @ np.exp(beta * hh) / 4096, rtol=0, atol=1e-15)
    assert np.allclose(c[1], cosn @ (hh * np.exp(beta * hh)) / 4096, rtol=0, atol=1e-15)
    assert np.allclose(c[2], cosn @ (hh * hh * np.exp(beta * hh)) / 4096, rtol=0, atol=1e-15)


def test_helper_cv_matches_high_precision_difference():
    """The product-rule C_v equals a fourth-order central difference of the
    grid's own ln Z (a check of the helper's algebra, no oracle involved)."""
    beta, delta, e = 0.7, 0.6, 1e-2
    A, B, C, D = _grid()

    def lnz(b):
        c = _coeff_derivs(b, delta)[0]
        wt = np.ones_like(A)
        for phi in (A - B, C - D, A - C, B - D):
            wt = wt * _bond(c, phi) ** 2
        return math.log(wt.sum() / K ** 4) / 4.0
    l = [lnz(beta + k * e) for k in (-2, -1, 0, 1, 2)]
    d2 = (-l[0] + 16 * l[1] - 30 * l[2] + 16 * l[3] - l[4]) / (12 * e * e)
    assert beta * beta * d2 == pytest.approx(exact_cv_per_site(beta, delta), rel=1e-6)


# --------------------------------------------------------------------------
# observables_from_runs (the oracle's f, C_v, chi, chi_n)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("beta,delta", [(0.7, 0.6), (1.3, 0.35)])
def test_observables_cv_and_f_match_exact_derivative(beta, delta):
    db = 1e-3
    lnz = [_exact_torus(beta + s, delta).lnz_per_site for s in (-db, 0.0, db)]
    obs = o.observables_from_runs(beta, lnz, [0.0, 0.0], [0.0, 0.0], db, 1e-4, 1e-4)
    exact = exact_cv_per_site(beta, delta)
    assert exact > 0.01
    assert obs["cv"] == pytest.approx(exact, rel=2e-6)
    # f = -(1/beta) ln Z/V, with ln Z/V of the grid integral
    A, B, C, D = _grid()
    c = _coeff_derivs(beta, delta)[0]
    wt = np.ones_like(A)
    for phi in (A - B, C - D, A - C, B - D):
        wt = wt * _bond(c, phi) ** 2
    assert obs["f"] == pytest.approx(-math.log(wt.sum() / K ** 4) / 4.0 / beta, rel=1e-13)


@pytest.mark.parametrize("beta,delta,hc", [(0.8, 0.6, 0.2), (1.2, 0.3, 1e-3)])
def test_observables_chi_matches_fluctuation_formula(beta, delta, hc):
    dh = 1e-4
    m_h = [_exact_torus(beta, delta, h=hc + s, imps=o.IMP_COS1).m_cos1 for s in (-dh, dh)]
    m_h1 = [_exact_torus(beta, delta, h1=hc + s, imps=o.IMP_COS2).m_cos2 for s in (-dh, dh)]
    obs = o.observables_from_runs(beta, [0.0, 1.0, 0.0], m_h, m_h1, 1e-3, dh, dh)
    chi = exact_chi(beta, delta, hc, 0.0, 1)
    chin = exact_chi(beta, delta, 0.0, hc, 2)
    assert chi > 0.05 and chin > 0.05
    assert obs["chi"] == pytest.approx(chi, rel=1e-6)
    assert obs["chi_n"] == pytest.approx(chin, rel=1e-6)


# --------------------------------------------------------------------------
# the transition oracle's scans (their own finite differences)
# --------------------------------------------------------------------------

def test_transition_cv_scan_matches_exact_derivative():
    temps = [1 / 0.7, 1 / 1.3]
    cv = ot.cv_scan(0.6, temps, dcut=10 ** 9, nmax=NMAX, nsteps=2)
    for t, c in zip(temps, cv):
        assert c == pytest.approx(exact_cv_per_site(1 / t, 0.6), rel=2e-6)


@pytest.mark.parametrize("use_h", [True, False])
def test_transition_chi_scan_matches_fluctuation_formula(use_h):
    temps = [1 / 0.8, 1 / 1.2]
    hbar = 0.05
    chi = ot.chi_scan(0.45, temps, hbar, use_h, dcut=10 ** 9, nmax=NMAX, nsteps=2)
    for t, c in zip(temps, chi):
        h, h1 = (hbar, 0.0) if use_h else (0.0, hbar)
        exact = exact_chi(1 / t, 0.45, h, h1, 1 if use_h else 2)
        assert c == pytest.approx(exact, rel=1e-6)


# --------------------------------------------------------------------------
# planted mistakes in the oracle's formulas must fail the pins above
# --------------------------------------------------------------------------

_orig_obs = o.observables_from_runs


def _obs_no_beta2(beta, lnz, m_h, m_h1, dbeta, dh, dh1):
    r = _orig_obs(beta, lnz, m_h, m_h1, dbeta, dh, dh1)
    r["cv"] /= beta * beta                   # mistake: dropped beta^2
    return r


def _obs_chi_half_step(beta, lnz, m_h, m_h1, dbeta, dh, dh1):
    r = _orig_obs(beta, lnz, m_h, m_h1, dbeta, dh, dh1)
    r["chi"] = (m_h[1] - m_h[0]) / dh        # mistake: dh for 2 dh
    return r


def _obs_chin_half_step(beta, lnz, m_h, m_h1, dbeta, dh, dh1):
    r = _orig_obs(beta, lnz, m_h, m_h1, dbeta, dh, dh1)
    r["chi_n"] = (m_h1[1] - m_h1[0]) / dh1   # mistake: dh1 for 2 dh1
    return r


def _obs_cv_wrong_sign(beta, lnz, m_h, m_h1, dbeta, dh, dh1):
    r = _orig_obs(beta, lnz, m_h, m_h1, dbeta, dh, dh1)
    r["cv"] = beta * beta * (lnz[2] + 2 * lnz[1] - lnz[0]) / dbeta ** 2   # mistake: signs
    return r


def _obs_chi_reversed(beta, lnz, m_h, m_h1, dbeta, dh, dh1):
    r = _orig_obs(beta, lnz, m_h, m_h1, dbeta, dh, dh1)
    r["chi"] = (m_h[0] - m_h[1]) / (2 * dh)  # mistake: reversed difference
    return r


def _obs_f_sign(beta, lnz, m_h, m_h1, dbeta, dh, dh1):
    r = _orig_obs(beta, lnz, m_h, m_h1, dbeta, dh, dh1)
    r["f"] = lnz[1] / beta                   # mistake: f = +T ln Z
    return r


OBS_MUTATIONS = {
    "cv_dropped_beta2": _obs_no_beta2,
    "chi_dh_for_2dh": _obs_chi_half_step,
    "chin_dh1_for_2dh1": _obs_chin_half_step,
    "cv_wrong_signs": _obs_cv_wrong_sign,
    "chi_reversed": _obs_chi_reversed,
    "f_sign": _obs_f_sign,
}


def _fails(check):
    try:
        check()
    except AssertionError:
        return True
    return False


@pytest.mark.parametrize("name", sorted(OBS_MUTATIONS))
def test_observable_mutation_is_caught(name, monkeypatch):
    monkeypatch.setattr(o, "observables_from_runs", OBS_MUTATIONS[name])
    checks = [lambda: test_observables_cv_and_f_match_exact_derivative(1.3, 0.35),
              lambda: test_observables_chi_matches_fluctuation_formula(0.8, 0.6, 0.2)]
    assert any(_fails(c) for c in checks), "mutation survived every pin"


def _cv_scan_no_beta2(delta, temps, dcut, nmax, nsteps, q=2, db=1e-3):
    out = []
    for t in temps:
        b = 1.0 / t
        l = [o.run_point(b + s, delta, nmax=nmax, dcut=dcut, nsteps=nsteps, impurities=0,
                         q=q).lnz_per_site for s in (-db, 0.0, db)]
        out.append((l[0] - 2.0 * l[1] + l[2]) / (db * db))   # mistake: no beta^2
    return np.array(out)


def _chi_scan_half_step(delta, temps, hbar, use_h, dcut, nmax, nsteps, q=2, dh=1e-4):
    return 2.0 * _orig_chi_scan(delta, temps, hbar, use_h, dcut, nmax, nsteps, q, dh)


_orig_chi_scan = ot.chi_scan


def test_transition_scan_mutations_are_caught(monkeypatch):
    with monkeypatch.context() as m:
        m.setattr(ot, "cv_scan", _cv_scan_no_beta2)
        assert _fails(test_transition_cv_scan_matches_exact_derivative)
    with monkeypatch.context() as m:
        m.setattr(ot, "chi_scan", _chi_scan_half_step)   # (= a step of dh for 2 dh)
        assert _fails(lambda: test_transition_chi_scan_matches_fluctuation_formula(True))
        assert _fails(lambda: test_transition_chi_scan_matches_fluctuation_formula(False))
