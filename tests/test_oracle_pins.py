"""Pins of the CPU oracle against mathematics that does not come from it.

Each test fixes part of the oracle with an independent route: a library
special function, a closed form, a brute-force tensor trace written here,
a direct theta-quadrature of the lattice integral, or an exact symmetry of
the model. The oracle itself is test infrastructure (see oracle/__init__).
"""

import math

import numpy as np
import pytest
from scipy.special import iv

import oracle.hotrg as o


# --------------------------------------------------------------------------
# independent helpers (no oracle arithmetic)
# --------------------------------------------------------------------------

def torus_trace(site_tensors, Lx, Ly):
    """Brute-force contraction of an Lx x Ly periodic network.

    site_tensors[(x, y)] is T[l, r, u, d]; the right leg of (x, y) joins the
    left leg of (x+1, y) and the down leg of (x, y) joins the up leg of
    (x, y+1), both periodically.
    """
    ops = []
    for y in range(Ly):
        for x in range(Lx):
            h_left = y * Lx + (x - 1) % Lx
            h_right = y * Lx + x
            v_up = Lx * Ly + ((y - 1) % Ly) * Lx + x
            v_down = Lx * Ly + y * Lx + x
            ops += [site_tensors[(x, y)], [h_left, h_right, v_up, v_down]]
    return float(np.einsum(*ops, [], optimize="greedy"))


def theta_integral_2x2(t, beta, h=0.0, h1=0.0, K=40, observable=None, q=2):
    """Z (or <obs(theta_A)> Z) on the 2x2 periodic torus by trapezoid rule.

    Bond weight w(phi) = sum_{|n|<=nmax} t_n e^{i n phi} (character-truncated),
    site weight exp(beta h cos theta + beta h1 cos q theta). Every pair of
    neighbouring sites on the 2x2 torus is joined by two bonds:
    Z = (1/K^4) sum_{A,B,C,D} s_A s_B s_C s_D w(A-B)^2 w(C-D)^2 w(A-C)^2 w(B-D)^2.
    For fixed (A, D) the sums over B and over C are the same,
    M(A, D) = sum_X s_X w(A-X)^2 w(X-D)^2, so Z = (1/K^4) sum s_A s_D M(A, D)^2.
    """
    nmax = (len(t) - 1) // 2
    th = 2 * np.pi * np.arange(K) / K
    ns = np.arange(-nmax, nmax + 1)

    def w(phi):
        return np.tensordot(np.cos(np.multiply.outer(phi, ns)), t, axes=([-1], [0]))

    s = np.exp(beta * h * np.cos(th) + beta * h1 * np.cos(q * th))
    W2 = w(np.subtract.outer(th, th)) ** 2
    M = W2 @ (s[:, None] * W2)
    sa = s if observable is None else s * observable(th)
    return float(sa @ (M * M) @ s) / K ** 4


def untruncated(beta, delta, nmax, nsteps, h=0.0, h1=0.0, imps=0, first="y"):
    return o.run_point(beta, delta, h=h, h1=h1, nmax=nmax, dcut=10 ** 9,
                       nsteps=nsteps, impurities=imps, first=first)


# --------------------------------------------------------------------------
# special functions and character coefficients
# --------------------------------------------------------------------------

@pytest.mark.parametrize("k", [0, 1, 2, 5, 11, -3])
@pytest.mark.parametrize("x", [1e-4, 0.05, 0.7, 1.5, 6.0])
def test_bessel_matches_scipy(k, x):
    assert o.bessel_i(k, x) == pytest.approx(iv(k, x), rel=1e-14, abs=1e-300)


@pytest.mark.parametrize("beta", [0.3, 1.0, 1.5])
@pytest.mark.parametrize("delta", [0.0, 0.3, 0.7, 1.0])
def test_quadrature_equals_bessel_series(beta, delta):
    tq = o.char_coeffs(beta, delta, 10)
    tb = o.char_coeffs_bessel(beta, delta, 10)
    assert np.max(np.abs(tq - tb)) <= 1e-14 * math.exp(beta)


@pytest.mark.parametrize("beta", [0.5, 1.0, 1.5])
@pytest.mark.parametrize("delta", [0.0, 0.25, 0.5, 1.0])
def test_character_closed_sums(beta, delta):
    t = o.char_coeffs(beta, delta, 40)
    n = np.arange(-40, 41)
    tol = 1e-14 * math.exp(beta) * 10
    assert abs(t.sum() - math.exp(beta)) <= tol                       # w(0)
    assert abs(((-1.0) ** n * t).sum() - math.exp(beta * (1 - 2 * delta))) <= tol  # w(pi)
    t2 = o.char_coeffs(2 * beta, delta, 0)[0]                         # Parseval
    assert abs((t * t).sum() - t2) <= tol


@pytest.mark.parametrize("beta", [0.4, 1.0, 1.5])
def test_delta_limits_reduce_to_bessel(beta):
    t1 = o.char_coeffs(beta, 1.0, 8)
    tol = 1e-15 * math.exp(beta)   # trapezoid error is absolute, ~eps * w_max
    assert np.allclose(t1, iv(np.arange(-8, 9), beta), rtol=1e-13, atol=tol)
    t0 = o.char_coeffs(beta, 0.0, 8)
    n = np.arange(-8, 9)
    even = n % 2 == 0
    assert np.allclose(t0[even], iv(n[even] // 2, beta), rtol=1e-13, atol=tol)
    assert np.max(np.abs(t0[~even])) <= 1e-15 * math.exp(beta)


def test_beta_zero_coefficients():
    t = o.char_coeffs(0.0, 0.37, 5)
    assert t[5] == 1.0 and np.count_nonzero(t) == 1


def test_field_factors_zero_field_exact():
    F, FM, FM1 = o.field_factors(1.3, 0.0, 0.0, 8)
    q = np.arange(-8, 9)
    assert np.array_equal(F, (q == 0).astype(float))
    assert np.array_equal(FM, 0.5 * (np.abs(q) == 1))
    assert np.array_equal(FM1, 0.5 * (np.abs(q) == 2))


def test_field_factors_are_fourier_coefficients():
    """F(Q) is the Q-th Fourier coefficient of exp(bh cos th + bh1 cos 2th)."""
    beta, h, h1 = 1.1, 0.3, 0.2
    F, FM, FM1 = o.field_factors(beta, h, h1, 6)
    K = 256
    th = 2 * np.pi * np.arange(K) / K
    s = np.exp(beta * h * np.cos(th) + beta * h1 * np.cos(2 * th))
    for a, Q in enumerate(range(-6, 7)):
        assert F[a] == pytest.approx(np.mean(s * np.cos(Q * th)), abs=1e-15)
        assert FM[a] == pytest.approx(np.mean(np.cos(th) * s * np.cos(Q * th)), abs=1e-15)
        assert FM1[a] == pytest.approx(np.mean(np.cos(2 * th) * s * np.cos(Q * th)), abs=1e-15)


# --------------------------------------------------------------------------
# tensors, conventions, contraction
# --------------------------------------------------------------------------

@pytest.mark.parametrize("beta,delta,nmax", [(1.0, 0.5, 3), (0.7, 0.2, 10), (1.4, 0.9, 6)])
def test_one_by_one_torus(beta, delta, nmax):
    r = o.run_point(beta, delta, nmax=nmax, dcut=12, nsteps=0, impurities=0)
    t = o.char_coeffs(beta, delta, nmax)
    assert math.exp(r.lnz_per_site) == pytest.approx(t.sum() ** 2, rel=1e-14)


def test_charge_law_elementwise():
    nmax = 4
    T, imps = o.initial_tensors(1.0, 0.4, 0.0, 0.0, nmax, impurities=3)
    n = np.arange(-nmax, nmax + 1)
    l, r, u, d = np.meshgrid(n, n, n, n, indexing="ij")
    viol = (l + d) != (r + u)
    assert np.all(T[viol] == 0.0) and np.all(T[~viol] > 0.0)
    assert np.all(imps[1][np.abs(u + r - d - l) != 1] == 0.0)
    assert np.all(imps[2][np.abs(u + r - d - l) != 2] == 0.0)


@pytest.mark.parametrize("beta,delta,h,h1", [(0.8, 0.5, 0.0, 0.0), (1.1, 0.3, 0.0, 0.0),
                                             (0.9, 0.6, 0.25, 0.0), (0.9, 0.4, 0.0, 0.3),
                                             (1.0, 0.5, 0.2, 0.15)])
def test_two_by_two_theta_quadrature(beta, delta, h, h1):
    """Untruncated HOTRG on the 2x2 torus = direct lattice integral."""
    nmax = 3
    t = o.char_coeffs(beta, delta, nmax)
    r = untruncated(beta, delta, nmax, 2, h=h, h1=h1, imps=3)
    Z = theta_integral_2x2(t, beta, h, h1)
    assert 4 * r.lnz_per_site == pytest.approx(math.log(Z), rel=0, abs=1e-13)
    m1 = theta_integral_2x2(t, beta, h, h1, observable=np.cos) / Z
    m2 = theta_integral_2x2(t, beta, h, h1, observable=lambda a: np.cos(2 * a)) / Z
    assert r.m_cos1 == pytest.approx(m1, abs=1e-13)
    assert r.m_cos2 == pytest.approx(m2, abs=1e-13)


# --------------------------------------------------------------------------
# harmonic q >= 3 of the second coupling (eq. gXY_ham with general q)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("q", [3, 4, 5])
@pytest.mark.parametrize("beta,delta", [(0.6, 0.3), (1.2, 0.7), (1.5, 0.0)])
def test_harmonic_q_quadrature_equals_bessel_series(q, beta, delta):
    tq = o.char_coeffs(beta, delta, 12, q=q)
    tb = o.char_coeffs_bessel(beta, delta, 12, q=q)
    assert np.max(np.abs(tq - tb)) <= 1e-14 * math.exp(beta)


@pytest.mark.parametrize("q", [3, 4])
@pytest.mark.parametrize("beta,delta", [(0.5, 0.25), (1.0, 0.5), (1.5, 0.8)])
def test_harmonic_q_closed_sums(q, beta, delta):
    """w(0) = e^beta and w(pi) = e^{beta(-Delta + (1-Delta)(-1)^q)}."""
    t = o.char_coeffs(beta, delta, 40, q=q)
    n = np.arange(-40, 41)
    tol = 1e-13 * math.exp(beta)
    assert abs(t.sum() - math.exp(beta)) <= tol
    wpi = math.exp(beta * (-delta + (1.0 - delta) * (-1.0) ** q))
    assert abs(((-1.0) ** n * t).sum() - wpi) <= tol


@pytest.mark.parametrize("q", [3, 4])
def test_harmonic_q_delta_zero_is_bessel_of_n_over_q(q):
    """At Delta = 0, w = exp(beta cos q phi): t_n = I_{n/q}(beta) if q | n, else 0."""
    beta = 1.3
    t = o.char_coeffs(beta, 0.0, 12, q=q)
    n = np.arange(-12, 13)
    on = n % q == 0
    assert np.allclose(t[on], iv(n[on] // q, beta), rtol=1e-13, atol=1e-15 * math.exp(beta))
    assert np.max(np.abs(t[~on])) <= 1e-15 * math.exp(beta)


def test_harmonic_q_field_factors():
    """Zero field: cos q theta impurity at |Q| = q; with fields: Fourier
    coefficients of exp(bh cos th + bh1 cos q th) times 1, cos th, cos q th."""
    for q in (3, 4):
        F, FM, FM1 = o.field_factors(1.1, 0.0, 0.0, 8, q=q)
        Q = np.arange(-8, 9)
        assert np.array_equal(FM1, 0.5 * (np.abs(Q) == q))
        beta, h, h1 = 1.1, 0.3, 0.2
        F, FM, FM1 = o.field_factors(beta, h, h1, 6, q=q)
        K = 256
        th = 2 * np.pi * np.arange(K) / K
        s = np.exp(beta * h * np.cos(th) + beta * h1 * np.cos(q * th))
        for a, Qa in enumerate(range(-6, 7)):
            assert F[a] == pytest.approx(np.mean(s * np.cos(Qa * th)), abs=1e-15)
            assert FM[a] == pytest.approx(np.mean(np.cos(th) * s * np.cos(Qa * th)), abs=1e-15)
            assert FM1[a] == pytest.approx(np.mean(np.cos(q * th) * s * np.cos(Qa * th)),
                                           abs=1e-15)


@pytest.mark.parametrize("q", [3, 4])
@pytest.mark.parametrize("beta,delta,h,h1", [(0.9, 0.4, 0.0, 0.0), (1.0, 0.3, 0.0, 0.3),
                                             (0.8, 0.5, 0.2, 0.15)])
def test_harmonic_q_two_by_two_theta_quadrature(q, beta, delta, h, h1):
    """Untruncated HOTRG on the 2x2 torus (U(1), Z_q and no-symmetry
    sectors) = direct lattice integral with the cos q couplings."""
    nmax = 3
    t = o.char_coeffs(beta, delta, nmax, q=q)
    r = o.run_point(beta, delta, h=h, h1=h1, nmax=nmax, dcut=10 ** 9, nsteps=2,
                    impurities=3, q=q)
    # K = 60 nodes: the trapezoid rule is exact up to degree K - 1, and the
    # site weight's cos q theta series aliases at degree 16 + q l >= K only
    # for orders l whose I_l(beta h1) are below 1e-16
    K = 60
    Z = theta_integral_2x2(t, beta, h, h1, K=K, q=q)
    assert 4 * r.lnz_per_site == pytest.approx(math.log(Z), rel=0, abs=1e-13)
    m1 = theta_integral_2x2(t, beta, h, h1, K=K, observable=np.cos, q=q) / Z
    mq = theta_integral_2x2(t, beta, h, h1, K=K, observable=lambda a: np.cos(q * a), q=q) / Z
    assert r.m_cos1 == pytest.approx(m1, abs=1e-13)
    assert r.m_cos2 == pytest.approx(mq, abs=1e-13)


def test_harmonic_q_sectors_do_not_change_truncated_runs():
    """Z_q sectors (h = 0 != h1) against one dense block: the symmetry only
    splits the eigensolves, so a truncated run gives the same ln Z/V."""
    pt = dict(beta=1.0, delta=0.4, h1=0.2, nmax=3, dcut=9, nsteps=4, impurities=0)
    T, _ = o.initial_tensors(pt["beta"], pt["delta"], 0.0, pt["h1"], pt["nmax"], q=3)
    lab = o.leg_labels(pt["nmax"], o.SYM_Z2, 3)
    zq = o.hotrg_run(T, {}, lab, lab, o.SYM_Z2, pt["dcut"], pt["nsteps"], q=3)
    zero = np.zeros_like(lab)
    dense = o.hotrg_run(T, {}, zero, zero, o.SYM_NONE, pt["dcut"], pt["nsteps"], q=3)
    assert zq.lnz_per_site == pytest.approx(dense.lnz_per_site, abs=1e-12)


def test_two_by_two_full_characters_tail():
    """With untruncated characters the lattice integral differs by the tail."""
    beta, delta, nmax = 1.0, 0.5, 3
    r = untruncated(beta, delta, nmax, 2)
    K = 40
    th = 2 * np.pi * np.arange(K) / K
    A, B, C, D = np.meshgrid(th, th, th, th, indexing="ij")

    def w(p):
        return np.exp(beta * (delta * np.cos(p) + (1 - delta) * np.cos(2 * p)))
    Z = float(((w(A - B) * w(C - D) * w(A - C) * w(B - D)) ** 2).sum()) / K ** 4
    rel = abs(math.exp(4 * r.lnz_per_site) / Z - 1)
    t_tail = o.char_coeffs(beta, delta, nmax + 1)[-1] / o.char_coeffs(beta, delta, 0)[0]
    assert rel < 20 * t_tail


@pytest.mark.parametrize("first", ["y", "x"])
@pytest.mark.parametrize("h,h1", [(0.0, 0.0), (0.3, 0.2)])
def test_four_by_two_brute_force(first, h, h1):
    """N = 3 untruncated steps against a brute-force trace of 8 tensors."""
    beta, delta, nmax = 0.9, 0.4, 1
    r = untruncated(beta, delta, nmax, 3, h=h, h1=h1, imps=3, first=first)
    T, imps = o.initial_tensors(beta, delta, h, h1, nmax, impurities=3)
    Lx, Ly = (2, 4) if first == "y" else (4, 2)
    sites = {(x, y): T for x in range(Lx) for y in range(Ly)}
    Z = torus_trace(sites, Lx, Ly)
    assert 8 * r.lnz_per_site == pytest.approx(math.log(Z), abs=1e-13)
    for k, m in ((1, r.m_cos1), (2, r.m_cos2)):
        s2 = dict(sites)
        s2[(0, 0)] = imps[k]
        assert m == pytest.approx(torus_trace(s2, Lx, Ly) / Z, abs=1e-13)


def test_one_by_two_brute_force():
    beta, delta, nmax = 1.2, 0.6, 3
    r = untruncated(beta, delta, nmax, 1, imps=0)
    T, _ = o.initial_tensors(beta, delta, 0.0, 0.0, nmax)
    Z = torus_trace({(0, 0): T, (0, 1): T}, 1, 2)
    assert 2 * r.lnz_per_site == pytest.approx(math.log(Z), abs=1e-14)


def _ring_tensor(t):
    """T[l, r, u, d] = t_l delta_{lr}: horizontal rings, trivial vertical bond."""
    D = len(t)
    T = np.zeros((D, D, 1, 1))
    T[np.arange(D), np.arange(D), 0, 0] = t
    return T


@pytest.mark.parametrize("first,nsteps,Lx,Ly", [("y", 2, 2, 2), ("x", 3, 4, 2), ("x", 1, 2, 1)])
def test_decoupled_rings_closed_form(first, nsteps, Lx, Ly):
    """Z = (sum_n t_n^Lx)^Ly for rings of length Lx (1D closed form)."""
    nmax = 3
    t = o.char_coeffs(1.0, 0.5, nmax)
    lab = np.arange(-nmax, nmax + 1)
    r = o.hotrg_run(_ring_tensor(t), {}, lab, np.zeros(1, dtype=int), o.SYM_U1,
                    10 ** 6, nsteps, first=first)
    expect = Ly * math.log(np.sum(t ** Lx))
    assert Lx * Ly * r.lnz_per_site == pytest.approx(expect, abs=1e-13)


# --------------------------------------------------------------------------
# HOSVD pieces against an explicit M
# --------------------------------------------------------------------------

def test_environment_spectrum_is_hosvd_mode_spectrum():
    """|S_{i,:,:,:}|^2 = squared singular values of the explicit unfolding."""
    T, _ = o.initial_tensors(1.1, 0.6, 0.1, 0.05, 2)
    Dh, Dv = T.shape[0], T.shape[2]
    M = np.einsum("aeui,bfid->abefud", T, T).reshape(Dh * Dh, Dh * Dh, Dv, Dv)
    EL, ER = o.environments(T)
    sL = np.linalg.svd(M.reshape(Dh * Dh, -1), compute_uv=False) ** 2
    sR = np.linalg.svd(M.transpose(1, 0, 2, 3).reshape(Dh * Dh, -1), compute_uv=False) ** 2
    assert np.allclose(np.sort(np.linalg.eigvalsh(EL))[::-1], sL, atol=1e-14 * sL[0])
    assert np.allclose(np.sort(np.linalg.eigvalsh(ER))[::-1], sR, atol=1e-14 * sR[0])
    Mm = M.reshape(Dh * Dh, -1)
    assert np.allclose(EL, Mm @ Mm.T, atol=1e-15 * sL[0])


def test_projection_matches_explicit_sandwich():
    """T' = P^T M P with M from eq. Mtensor, contracted here by einsum."""
    rng = np.random.default_rng(5)
    Dh, Dv, Dn = 4, 3, 5
    A = rng.standard_normal((Dh, Dh, Dv, Dv))
    B = rng.standard_normal((Dh, Dh, Dv, Dv))
    P = np.linalg.qr(rng.standard_normal((Dh * Dh, Dn)))[0]
    M = np.einsum("aeui,bfid->abefud", A, B).reshape(Dh * Dh, Dh * Dh, Dv, Dv)
    ref = np.einsum("ia,ijud,jb->abud", P, M, P)
    assert np.allclose(o.project(P, A, B), ref, atol=1e-13)


def test_truncation_discarded_weight_identity():
    """eps = trace(E) - sum of kept eigenvalues, and P is an isometry."""
    T, _ = o.initial_tensors(1.0, 0.5, 0.0, 0.0, 3)
    EL, ER = o.environments(T)
    lab = o.fuse_labels(np.arange(-3, 4), np.arange(-3, 4), o.SYM_U1)
    sel = o.select_states(o.sector_eigh(EL, lab), o.sector_eigh(ER, lab), 12, 49)
    E = EL if sel.side == 0 else ER
    kept = np.trace(sel.P.T @ E @ sel.P)
    eps = sel.eps_l if sel.side == 0 else sel.eps_r
    assert eps == pytest.approx(np.trace(E) - kept, abs=1e-14 * np.trace(E))
    assert np.allclose(sel.P.T @ sel.P, np.eye(12), atol=1e-13)
    # the kept eigenvalues are the 12 largest of the whole spectrum
    lam = np.sort(np.linalg.eigvalsh(E))[::-1]
    assert kept == pytest.approx(lam[:12].sum(), rel=1e-13)


# --------------------------------------------------------------------------
# whole-run identities with truncation
# --------------------------------------------------------------------------

def test_beta_zero_gives_zero_free_energy():
    r = o.run_point(0.0, 0.5, nmax=3, dcut=12, nsteps=12)
    assert r.lnz_per_site == 0.0
    assert r.m_cos1 == 0.0 and r.m_cos2 == 0.0


def test_normalisation_choice_invariance():
    # a well-conditioned point: at beta=1, Delta=0.5, Dcut=12 the truncated
    # flow amplifies rounding-level differences to ~1e-10 (see
    # test_conditioning_spread_of_single_point)
    a = o.run_point(1.2, 0.7, nmax=3, dcut=12, nsteps=30, impurities=0, norm="fro")
    b = o.run_point(1.2, 0.7, nmax=3, dcut=12, nsteps=30, impurities=0, norm="maxabs")
    assert a.lnz_per_site == pytest.approx(b.lnz_per_site, abs=1e-13)


def test_high_temperature_series():
    beta, delta = 0.1, 0.5
    r = o.run_point(beta, delta, nmax=4, dcut=16, nsteps=20, impurities=0)
    t = o.char_coeffs(beta, delta, 4)
    t0 = t[4]
    series = 2 * math.log(t0) + 2 * np.sum((t[5:] / t0) ** 4)
    assert abs(r.lnz_per_site - series) <= 10 * (t[5] / t0) ** 6
    # the quartic term itself is resolved
    assert abs(r.lnz_per_site - 2 * math.log(t0)) > 100 * 10 * (t[5] / t0) ** 6


def test_zero_field_magnetisations_vanish_exactly():
    r = o.run_point(1.0, 0.5, nmax=3, dcut=12, nsteps=10)
    assert r.m_cos1 == 0.0 and r.m_cos2 == 0.0


@pytest.mark.parametrize("beta", [0.8, 1.2])
def test_delta0_equals_delta1_with_truncation(beta):
    """Z(beta, Delta=0) = Z(beta, Delta=1) on every torus (theta -> 2 theta)."""
    a = o.run_point(beta, 0.0, nmax=6, dcut=12, nsteps=14, impurities=0)
    b = o.run_point(beta, 1.0, nmax=3, dcut=12, nsteps=14, impurities=0)
    assert a.lnz_per_site == pytest.approx(b.lnz_per_site, abs=1e-13)


def test_delta0_nematic_equals_delta1_magnetisation():
    a = o.run_point(0.9, 0.0, h1=0.05, nmax=4, dcut=10, nsteps=8, impurities=2)
    b = o.run_point(0.9, 1.0, h=0.05, nmax=2, dcut=10, nsteps=8, impurities=1)
    assert a.lnz_per_site == pytest.approx(b.lnz_per_site, abs=1e-13)
    assert a.m_cos2 == pytest.approx(b.m_cos1, abs=1e-12)


def test_impurity_matches_field_derivative():
    """<cos theta> = (1/beta) d(ln Z/V)/dh, to truncation-level accuracy:
    the gap closes as Dcut grows."""
    beta, delta, h, dh = 0.5, 0.6, 0.1, 1e-4
    gaps = []
    for dcut in (8, 20):
        kw = dict(nmax=3, dcut=dcut, nsteps=14)
        r = o.run_point(beta, delta, h=h, impurities=1, **kw)
        rp = o.run_point(beta, delta, h=h + dh, impurities=0, **kw)
        rm = o.run_point(beta, delta, h=h - dh, impurities=0, **kw)
        fd = (rp.lnz_per_site - rm.lnz_per_site) / (2 * dh) / beta
        gaps.append(abs(r.m_cos1 - fd))
        assert r.m_cos1 > 0.05
    assert gaps[1] < 2e-6 and gaps[1] < gaps[0] / 5


def test_free_energy_plausible_against_thesis_table():
    """Table 2 prints F = -0.54360.. at Delta = 0.34, T = 0.694, D = 91 with
    an unstated h1 >= 0. A field only lowers F, so the zero-field F must not
    lie below the printed value by more than the truncation spread."""
    beta = 1 / 0.694
    r = o.run_point(beta, 0.34, nmax=10, dcut=16, nsteps=30, impurities=0)
    F = -r.lnz_per_site / beta
    assert F >= -0.5436066 - 1e-3
    assert abs(F - (-0.5436043)) < 0.03


def test_conditioning_spread_of_single_point():
    """At beta=1, Delta=0.5, Dcut=12 the truncated flow amplifies rounding:
    1-ulp relative perturbations of the initial tensor move ln Z/V by up to
    ~1e-10, which bounds any parity claim at this point (the GPU parity
    test compares it at 1e-9 and its first ten steps at 1e-11)."""
    T, _ = o.initial_tensors(1.0, 0.5, 0.0, 0.0, 3)
    lab = o.leg_labels(3, o.SYM_U1)
    base = o.hotrg_run(T, {}, lab, lab, o.SYM_U1, 12, 30).lnz_per_site
    rng = np.random.default_rng(1)
    spread = 0.0
    for _ in range(3):
        Tp = T * (1 + 2.0 ** -52 * rng.standard_normal(T.shape))
        spread = max(spread, abs(o.hotrg_run(Tp, {}, lab, lab, o.SYM_U1, 12, 30).lnz_per_site - base))
    assert 1e-12 < spread < 1e-9
