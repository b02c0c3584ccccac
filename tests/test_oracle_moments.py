"""Pins of the oracle's zero-field susceptibility from summed insertions.

The oracle carries, besides the pure block tensor, the block tensor with one
cos(k theta) insertion averaged over the block's sites and the one with two
insertions averaged over ordered pairs of sites; at the end
<m^2> = Tr T2 / Tr T with m the site average, and the susceptibility of
Ch. 3 (eq. susc) is chi = beta V (<m^2> - <m>^2) by the fluctuation
relation. These tests fix that against:

* beta = 0, where the sites decouple and V <m^2> = <cos^2> = 1/2 exactly at
  any size and truncation;
* the 2x2 torus, against d<cos theta>/dh at h = 0 by the fluctuation
  formula on an angle grid (independent helper of test_oracle_observables);
* the 4x2 torus, against brute-force traces of the network with the
  insertions placed at every pair of sites (site tensors built here from the
  angle integral of the insertion, not from the oracle);
* truncated runs, against the finite difference of the impurity expectation
  value in h (truncation-level agreement that improves with Dcut).
Planted mistakes in the second-moment update must fail.
"""

import numpy as np
import pytest

import oracle.hotrg as o
import tests.test_oracle_pins as pins
from tests.test_oracle_observables import exact_chi


def _moment_run(beta, delta, nmax, dcut, nsteps, q=2, which=o.IMP_COS1_SQ | o.IMP_COS2_SQ):
    return o.run_point(beta, delta, nmax=nmax, dcut=dcut, nsteps=nsteps, impurities=which, q=q)


@pytest.mark.parametrize("nsteps,dcut", [(2, 10 ** 9), (6, 8), (11, 5)])
def test_beta_zero_gives_half_per_site(nsteps, dcut):
    r = _moment_run(0.0, 0.4, 3, dcut, nsteps)
    V = 2.0 ** nsteps
    assert r.msq_cos1 * V == pytest.approx(0.5, rel=1e-14)
    assert r.msq_cos2 * V == pytest.approx(0.5, rel=1e-14)
    assert r.m_cos1 == 0.0 and r.chi0 == 0.0 and r.chi0_n == 0.0


@pytest.mark.parametrize("beta,delta", [(0.8, 0.6), (1.2, 0.3), (0.5, 0.9)])
def test_two_by_two_matches_fluctuation_formula(beta, delta):
    r = _moment_run(beta, delta, 3, 10 ** 9, 2)
    assert r.m_cos1 == 0.0 and r.m_cos2 == 0.0
    assert r.chi0 == pytest.approx(exact_chi(beta, delta, 0.0, 0.0, 1), rel=1e-12)
    assert r.chi0_n == pytest.approx(exact_chi(beta, delta, 0.0, 0.0, 2), rel=1e-12)


def _site_tensor(f, t, nmax, K=64):
    """sqrt(t_l t_r t_u t_d) times the Fourier coefficient of f(theta) at
    Q = n_u + n_r - n_d - n_l, by a K-point angle sum (exact for the
    trigonometric polynomials used here)."""
    n = np.arange(-nmax, nmax + 1)
    l, r, u, d = np.meshgrid(n, n, n, n, indexing="ij")
    Q = u + r - d - l
    th = 2 * np.pi * np.arange(K) / K
    coef = {int(x): float(np.mean(f(th) * np.cos(x * th))) for x in np.unique(Q)}
    amp = np.sqrt(t[l + nmax] * t[r + nmax] * t[u + nmax] * t[d + nmax])
    return amp * np.vectorize(coef.get)(Q)


@pytest.mark.parametrize("k", [1, 2])
def test_four_by_two_brute_force_pairs(k):
    beta, delta, nmax = 0.9, 0.4, 1
    r = _moment_run(beta, delta, nmax, 10 ** 9, 3)
    t = o.char_coeffs(beta, delta, nmax)
    T = _site_tensor(lambda a: np.ones_like(a), t, nmax)
    T1 = _site_tensor(lambda a: np.cos(k * a), t, nmax)
    T2 = _site_tensor(lambda a: np.cos(k * a) ** 2, t, nmax)
    Lx, Ly = 2, 4                      # first step contracts the vertical bond
    pos = [(x, y) for x in range(Lx) for y in range(Ly)]
    Z = pins.torus_trace({p: T for p in pos}, Lx, Ly)
    s2 = 0.0
    for i in pos:
        for j in pos:
            sites = {p: T for p in pos}
            if i == j:
                sites[i] = T2
            else:
                sites[i] = T1
                sites[j] = T1
            s2 += pins.torus_trace(sites, Lx, Ly)
    msq = s2 / Z / 64.0
    got = r.msq_cos1 if k == 1 else r.msq_cos2
    assert got == pytest.approx(msq, rel=1e-12)


def test_truncated_runs_approach_the_field_derivative():
    """chi from the insertions against [m(dh) - m(-dh)] / (2 dh) of the
    impurity chain in a field (a different truncation: no symmetry sectors)
    on 16 sites, closer as Dcut grows (measured: 11 %, 5 %, 1 %, 0.6 % at
    Dcut = 6, 14, 24, 40; on 1024 sites the charge-conserving truncation of
    the zero-field route converges more slowly)."""
    beta, delta, dh, nsteps = 0.6, 0.7, 1e-5, 4
    gaps = []
    for dcut in (6, 24):
        r = _moment_run(beta, delta, 3, dcut, nsteps, which=o.IMP_COS1_SQ)
        m = [o.run_point(beta, delta, h=s, nmax=3, dcut=dcut, nsteps=nsteps,
                         impurities=o.IMP_COS1).m_cos1 for s in (-dh, dh)]
        fd = (m[1] - m[0]) / (2 * dh)
        gaps.append(abs(r.chi0 - fd) / fd)
        assert r.chi0 > 0.5
    assert gaps[1] < 0.02 and gaps[1] < gaps[0] / 5


def test_harmonic_q_two_by_two():
    """q = 3: the second coupling and the second insertion on cos 3 theta."""
    beta, delta, q = 1.0, 0.4, 3
    r = _moment_run(beta, delta, 3, 10 ** 9, 2, q=q)
    # the fluctuation formula on the grid with cos 3 theta
    K = 48
    th = 2 * np.pi * np.arange(K) / K
    A, B, C, D = np.meshgrid(th, th, th, th, indexing="ij")
    t = o.char_coeffs_bessel(beta, delta, 3, q=q)
    n = np.arange(-3, 4)

    def w(phi):
        return np.tensordot(np.cos(np.multiply.outer(phi, n)), t, axes=([-1], [0]))
    wt = w(A - B) ** 2 * w(C - D) ** 2 * w(A - C) ** 2 * w(B - D) ** 2
    S = sum(np.cos(q * x) for x in (A, B, C, D))
    chi = beta * (wt * S * S).sum() / wt.sum() / 4.0
    assert r.chi0_n == pytest.approx(chi, rel=1e-12)


# --------------------------------------------------------------------------
# planted mistakes in the second-moment update
# --------------------------------------------------------------------------

_orig_project = o.project
_orig_square = o.square_factors


def _checks():
    return [lambda: test_beta_zero_gives_half_per_site(6, 8),
            lambda: test_two_by_two_matches_fluctuation_formula(0.8, 0.6),
            lambda: test_four_by_two_brute_force_pairs(1)]


def _fails(c):
    try:
        c()
    except AssertionError:
        return True
    return False


def _square_without_constant(qmax, q=2):
    a, b = _orig_square(qmax, q)
    mid = qmax
    a[mid] = 0.0                  # mistake: cos^2 = cos(2 theta)/2 only
    b[mid] = 0.0
    return a, b


def test_square_factor_mistake_is_caught(monkeypatch):
    monkeypatch.setattr(o, "square_factors", _square_without_constant)
    assert any(_fails(c) for c in _checks())


def _cross_once(P, x2, T, x1):
    return 0.25 * (o.project(P, x2, T) + o.project(P, T, x2) + o.project(P, x1, x1))


def _half_average(P, x2, T, x1):
    return 0.5 * (o.project(P, x2, T) + o.project(P, T, x2) + 2.0 * o.project(P, x1, x1))


@pytest.mark.parametrize("bad", [_cross_once, _half_average])
def test_second_moment_update_mistake_is_caught(bad, monkeypatch):
    monkeypatch.setattr(o, "second_moment_update", bad)
    assert any(_fails(c) for c in _checks())
