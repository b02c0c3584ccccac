"""Pins of the configurational-temperature oracle (oracle/lgt.py) against
what the definitions and exact identities fix, independently of the oracle's
own formulas (Ch. 4, eq. another-form; Ch. 5, eqs. grad_hess, beta_lat,
plaq_2d and the Wilson action).

* Plaquette: gauge invariance under random gauge transformations, a single
  excited link, and a uniform magnetic flux.
* Gradient, Hessian (diagonal and full), g^T h g: finite differences of the
  Wilson action alone.
* Estimator: the divergence of g / |g|^2 by finite differences of g.
* The exact identity <h_l> = beta <g_l^2> under the conditional law of one
  link (integration by parts on the circle), by quadrature of exp(-S).
* Equilibrium configurations (heat bath) of the two-dimensional theory:
  <cos theta_P> = I_1(beta) / I_0(beta) and <Tr h> / <|g|^2> = beta, and the
  plaquettes the thesis tabulates on a 32 x 32 lattice
  (tests/golden/lgt_u1_2d_table.json).
"""

import json
import os

import numpy as np
import pytest
from scipy.special import iv

import oracle.lgt as L

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _random(d, dims, seed):
    rng = np.random.default_rng(seed)
    return rng.uniform(-np.pi, np.pi, size=(d,) + tuple(reversed(dims)))


def _gauge(theta, alpha):
    d = theta.shape[0]
    return np.stack([theta[mu] + alpha - L.shift(alpha, d, mu) for mu in range(d)])


CASES = [(2, (3, 4)), (3, (2, 3, 4)), (4, (2, 3, 2, 3)), (2, (2, 3))]


@pytest.mark.parametrize("d,dims", CASES)
def test_plaquettes_are_gauge_invariant(d, dims):
    th = _random(d, dims, 1)
    alpha = np.random.default_rng(2).uniform(-np.pi, np.pi, size=th.shape[1:])
    for (m1, n1, a), (m2, n2, b) in zip(L.plaquettes(th), L.plaquettes(_gauge(th, alpha))):
        assert (m1, n1) == (m2, n2)
        assert np.max(np.abs(np.exp(1j * a) - np.exp(1j * b))) < 1e-13
    e0, e1 = L.estimator(th), L.estimator(_gauge(th, alpha))
    for k in ("sum_g2", "sum_h", "g_h_g", "plaquette"):
        assert e0[k] == pytest.approx(e1[k], rel=1e-12, abs=1e-12)


def test_mutated_plaquette_is_not_gauge_invariant(monkeypatch):
    """theta_nu taken at n + nu instead of n + mu: the check above fails."""
    def bad(theta):
        d = theta.shape[0]
        return [(mu, nu, theta[mu] + L.shift(theta[nu], d, nu) - L.shift(theta[mu], d, nu)
                 - theta[nu]) for mu in range(d) for nu in range(mu + 1, d)]
    th = _random(3, (3, 3, 4), 5)
    alpha = np.random.default_rng(6).uniform(-np.pi, np.pi, size=th.shape[1:])
    monkeypatch.setattr(L, "plaquettes", bad)
    a = L.plaquettes(th)[0][2]
    b = L.plaquettes(_gauge(th, alpha))[0][2]
    assert np.max(np.abs(np.exp(1j * a) - np.exp(1j * b))) > 1e-3


@pytest.mark.parametrize("d", [2, 3, 4])
def test_single_excited_link(d):
    """One link at angle t, the rest zero: exactly 2(d - 1) plaquettes take
    +-t, g = 2 (d - 1) sin t and h = 2 (d - 1) cos t on that link, and each
    neighbour in a shared plaquette has |g| = sin t."""
    dims = (4,) * d
    th = np.zeros((d,) + dims)
    t = 0.7
    idx = (1,) + (2,) * d
    th[idx] = t
    nz = sum(int(np.count_nonzero(np.abs(p) > 1e-15)) for _, _, p in L.plaquettes(th))
    assert nz == 2 * (d - 1)
    for _, _, p in L.plaquettes(th):
        assert set(np.round(p[np.abs(p) > 0], 15)) <= {t, -t}
    g, hd = L.gradient_hdiag(th)
    assert g[idx] == pytest.approx(2 * (d - 1) * np.sin(t), rel=1e-14)
    assert hd[idx] == pytest.approx(2 * (d - 1) * np.cos(t) + 0.0, rel=1e-14)
    mag = np.sort(np.abs(g[np.abs(g) > 1e-15]))
    assert len(mag) == 1 + 3 * 2 * (d - 1)
    assert np.allclose(mag, [np.sin(t)] * 6 * (d - 1) + [2 * (d - 1) * np.sin(t)], rtol=1e-14)


@pytest.mark.parametrize("d", [2, 4])
def test_uniform_flux(d):
    """theta_1(x) = B x_0 with the twist theta_0(L0 - 1, x_1) = -B L0 x_1
    carries flux B = 2 pi k / (L0 L1) through every 01 plaquette and none
    elsewhere: g vanishes on every link and h is 2 cos B + 2 (d - 2) on the
    0- and 1-links."""
    dims = (4, 6) + (3,) * (d - 2)
    L0, L1 = dims[0], dims[1]
    B = 2 * np.pi * 5 / (L0 * L1)
    th = np.zeros((d,) + tuple(reversed(dims)))
    x0 = np.arange(L0)
    x1 = np.arange(L1)
    th1 = th[1].reshape(-1, L1, L0)
    th1[:] = B * x0[None, None, :]
    th0 = th[0].reshape(-1, L1, L0)
    th0[:, :, L0 - 1] = -B * L0 * x1[None, :]
    for mu, nu, p in L.plaquettes(th):
        want = B if (mu, nu) == (0, 1) else 0.0
        assert np.max(np.abs(np.exp(1j * p) - np.exp(1j * want))) < 1e-12
    g, hd = L.gradient_hdiag(th)
    assert np.max(np.abs(g)) < 1e-12
    for mu in (0, 1):
        assert np.allclose(hd[mu], 2 * np.cos(B) + 2 * (d - 2), atol=1e-12)


def _fd1(f, x, i, eps):
    xp, xm = x.copy(), x.copy()
    xp.flat[i] += eps
    xm.flat[i] -= eps
    return (f(xp) - f(xm)) / (2 * eps)


@pytest.mark.parametrize("d,dims", CASES[:3])
def test_gradient_and_hessian_diagonal_are_derivatives_of_the_action(d, dims):
    beta = 1.3
    th = _random(d, dims, 11)
    g, hd = L.gradient_hdiag(th)
    S = lambda x: L.action(x, beta)  # noqa: E731
    eps = 1e-3
    for i in range(th.size):
        # fourth-order stencils (truncation ~ eps^4)
        def at(k):
            x = th.copy()
            x.flat[i] += k * eps
            return S(x)
        d1 = (-at(2) + 8 * at(1) - 8 * at(-1) + at(-2)) / (12 * eps) / beta
        d2 = (-at(2) + 16 * at(1) - 30 * at(0) + 16 * at(-1) - at(-2)) / (12 * eps ** 2) / beta
        assert d1 == pytest.approx(g.flat[i], abs=1e-9)
        assert d2 == pytest.approx(hd.flat[i], abs=2e-7)


def test_full_hessian_is_the_second_derivative_of_the_action():
    beta = 0.9
    th = _random(3, (2, 3, 2), 13)
    H = L.hessian(th).toarray()
    n = th.size
    eps = 1e-4
    S = lambda x: L.action(x, beta) / beta  # noqa: E731
    for i in range(n):
        for j in range(n):
            def at(a, b):
                x = th.copy()
                x.flat[i] += a * eps
                x.flat[j] += b * eps
                return S(x)
            fd = (at(1, 1) - at(1, -1) - at(-1, 1) + at(-1, -1)) / (4 * eps ** 2)
            assert fd == pytest.approx(H[i, j], abs=2e-6), (i, j)


@pytest.mark.parametrize("d,dims", [(2, (4, 4)), (3, (2, 3, 4)), (4, (2, 2, 3, 2))])
def test_g_h_g_is_the_curvature_along_g(d, dims):
    """g^T h g = (1/beta) d^2/dt^2 S(theta + t g) at t = 0."""
    beta = 1.1
    th = _random(d, dims, 17)
    e = L.estimator(th)
    g, _ = L.gradient_hdiag(th)
    u = g / np.linalg.norm(g)
    eps = 1e-3
    f = lambda t: L.action(th + t * u, beta) / beta  # noqa: E731
    d2 = (-f(2 * eps) + 16 * f(eps) - 30 * f(0) + 16 * f(-eps) - f(-2 * eps)) / (12 * eps ** 2)
    assert d2 * e["sum_g2"] == pytest.approx(e["g_h_g"], rel=1e-6, abs=1e-8)


@pytest.mark.parametrize("d,dims", [(2, (3, 3)), (3, (2, 2, 3)), (2, (2, 5))])
def test_estimator_is_the_divergence_of_g_over_g_squared(d, dims):
    """beta_full = sum_l d/dtheta_l (g_l / |g|^2) (Ch. 4, eq. temp_eq
    integrand), by central differences of the oracle's gradient only."""
    th = _random(d, dims, 19)
    F = lambda x: (lambda g: g / np.sum(g * g))(L.gradient_hdiag(x)[0])  # noqa: E731
    eps = 1e-5
    div = 0.0
    for i in range(th.size):
        xp, xm = th.copy(), th.copy()
        xp.flat[i] += eps
        xm.flat[i] -= eps
        div += (F(xp).flat[i] - F(xm).flat[i]) / (2 * eps)
    e = L.estimator(th)
    assert e["beta_full"] == pytest.approx(div, rel=1e-6)
    assert e["trace_h"] == pytest.approx(e["sum_h"], rel=1e-14)


def test_mutated_estimator_fails_the_divergence(monkeypatch):
    monkeypatch.setattr(L, "estimator_value", lambda tr, g2, ghg: tr / g2 + 2.0 * ghg / g2 ** 2)
    with pytest.raises(AssertionError):
        test_estimator_is_the_divergence_of_g_over_g_squared(2, (3, 3))


def test_mutated_link_sign_fails_the_derivatives(monkeypatch):
    monkeypatch.setattr(L, "_plaquette_links", lambda mu, nu: [
        (mu, {}, +1), (nu, {mu: 1}, +1), (mu, {nu: 1}, +1), (nu, {}, -1)])
    with pytest.raises(AssertionError):
        test_gradient_and_hessian_diagonal_are_derivatives_of_the_action(2, (3, 4))


@pytest.mark.parametrize("d,dims,beta", [(2, (4, 4), 1.7), (3, (2, 2, 4), 0.6),
                                         (4, (2, 2, 2, 2), 2.5)])
def test_conditional_identity_h_equals_beta_g_squared(d, dims, beta):
    """For one link with the others fixed, integration by parts over the
    circle gives int (h_l - beta g_l^2) exp(-S) d theta_l = 0: the
    conditional mean of h_l equals beta times that of g_l^2. Evaluated by
    the periodic trapezoid rule (exponentially accurate), with S from the
    action alone."""
    th = _random(d, dims, 23)
    for link in (0, th.size // 2, th.size - 1):
        K = 512
        ts = -np.pi + 2 * np.pi * np.arange(K) / K
        Ss, hs, g2s = [], [], []
        for t in ts:
            x = th.copy()
            x.flat[link] = t
            Ss.append(L.action(x, beta))
            g, hd = L.gradient_hdiag(x)
            hs.append(hd.flat[link])
            g2s.append(g.flat[link] ** 2)
        w = np.exp(-(np.array(Ss) - min(Ss)))
        eh = np.sum(w * np.array(hs)) / np.sum(w)
        eg2 = np.sum(w * np.array(g2s)) / np.sum(w)
        assert eh == pytest.approx(beta * eg2, rel=1e-10, abs=1e-12)


def _heatbath(beta, dims, ntherm, nmeas, seed):
    rng = np.random.default_rng(seed)
    th = rng.uniform(-np.pi, np.pi, size=(2,) + tuple(reversed(dims)))
    for _ in range(ntherm):
        L.heatbath_sweep(th, beta, rng)
    P, H, G = [], [], []
    for _ in range(nmeas):
        L.heatbath_sweep(th, beta, rng)
        e = L.estimator(th, full=False)
        P.append(e["plaquette"])
        H.append(e["sum_h"])
        G.append(e["sum_g2"])
    return np.array(P), np.array(H), np.array(G)


def _err(x, nb=20):
    b = np.array_split(x, nb)
    m = np.array([np.mean(y) for y in b])
    return np.std(m, ddof=1) / np.sqrt(nb)


@pytest.mark.parametrize("beta", [0.5, 1.0, 2.0])
def test_equilibrium_two_dimensional_theory(beta):
    """Heat-bath configurations of the 2D theory on 8 x 8: the plaquette
    average approaches I_1/I_0 (Ch. 5, eq. plaq_2d; the torus correction is
    of order (I_1/I_0)^64) and the ratio of means <Tr h> / <|g|^2> is beta
    (exact for any volume), within five standard errors."""
    P, H, G = _heatbath(beta, (8, 8), 100, 1500, seed=int(beta * 10))
    assert abs(np.mean(P) - iv(1, beta) / iv(0, beta)) < 5 * _err(P) + 1e-4
    r = np.mean(H) / np.mean(G)
    # error of the ratio from batch means of H - beta G
    assert abs(r - beta) * np.mean(G) < 5 * _err(H - beta * G) + 1e-9


def test_thesis_table_two_dimensional_plaquette():
    """The thesis's 32 x 32 plaquettes (Ch. 5, table tab:2d_u1_l32_l32)
    against the closed form I_1/I_0 and against heat-bath configurations of
    the oracle at the same couplings. The table's rows at beta = 9 and 10
    lie 10 and 58 of their errors below I_1/I_0 (the chapter notes that its
    sampling deviates at large beta), so the closed form is compared for
    beta <= 8. (Its beta_M, the mean of per-configuration ratios, carries a
    finite-volume bias that the ratio of means above does not, so it is not
    compared.)"""
    rows = json.load(open(os.path.join(GOLDEN, "lgt_u1_2d_table.json")))["rows"]
    for r in rows:
        if r["beta"] > 8.0:
            continue
        exact = iv(1, r["beta"]) / iv(0, r["beta"])
        assert abs(r["P"] - exact) < 5 * r["P_err"] + 2e-5
    for r in rows:
        if r["beta"] in (0.5, 1.0):
            P, _, _ = _heatbath(r["beta"], (8, 8), 100, 800, seed=7)
            assert abs(np.mean(P) - r["P"]) < 5 * (_err(P) + r["P_err"])


def test_extents_below_two_are_refused():
    with pytest.raises(ValueError):
        L.plaquettes(np.zeros((2, 3, 1)))
