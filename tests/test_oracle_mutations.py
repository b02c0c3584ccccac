"""Plant plausible mistakes in the oracle (on the CPU) and check a pin fails.

Each mutation replaces one oracle function with a subtly wrong variant
(dropped factor, wrong sign or index, transposed operand) and runs a few of
the pins from test_oracle_pins; at least one must fail.
"""

import math

import numpy as np
import pytest

import oracle.hotrg as o
import tests.test_oracle_pins as pins


def _expect_some_pin_fails(checks):
    failed = 0
    for check in checks:
        try:
            check()
        except (AssertionError, FloatingPointError, ValueError, IndexError):
            failed += 1
    assert failed > 0, "mutation survived every pin"


def _small_pins():
    return [
        lambda: pins.test_one_by_one_torus(1.0, 0.5, 3),
        lambda: pins.test_two_by_two_theta_quadrature(0.9, 0.6, 0.25, 0.0),
        lambda: pins.test_two_by_two_theta_quadrature(1.1, 0.3, 0.0, 0.0),
        lambda: pins.test_four_by_two_brute_force("y", 0.3, 0.2),
        lambda: pins.test_decoupled_rings_closed_form("x", 3, 4, 2),
        pins.test_environment_spectrum_is_hosvd_mode_spectrum,
        pins.test_projection_matches_explicit_sandwich,
        pins.test_truncation_discarded_weight_identity,
        pins.test_high_temperature_series,
    ]


def _wrong_orientation(beta, delta, h, h1, nmax, nquad=4096, impurities=0, q=2):
    t = o.char_coeffs(beta, delta, nmax, nquad, q)
    n = np.arange(-nmax, nmax + 1)
    F, FM, FM1 = o.field_factors(beta, h, h1, 4 * nmax, q=q)
    l, r, u, d = np.meshgrid(n, n, n, n, indexing="ij")
    Q = u + d - r - l                      # mistake: l + r = u + d
    amp = np.sqrt(t[l + nmax] * t[r + nmax] * t[u + nmax] * t[d + nmax])
    imps = {}
    if impurities & 1:
        imps[1] = amp * FM[Q + 4 * nmax]
    if impurities & 2:
        imps[2] = amp * FM1[Q + 4 * nmax]
    return amp * F[Q + 4 * nmax], imps


def _no_sqrt(beta, delta, h, h1, nmax, nquad=4096, impurities=0, q=2):
    T, imps = _orig_initial(beta, delta, h, h1, nmax, nquad, impurities, q)
    return T * T, {k: v * v for k, v in imps.items()}   # mistake: prod t, not sqrt


_orig_initial = o.initial_tensors
_orig_env = o.environments
_orig_project = o.project
_orig_select = o.select_states
_orig_run = o.hotrg_run


def _env_transposed(T):
    Dh = T.shape[0]
    A = np.tensordot(T, T, axes=([1, 2], [1, 2]))
    B = np.tensordot(T, T, axes=([1, 3], [1, 3]))
    EL = np.tensordot(A, B, axes=([1, 3], [3, 1]))    # mistake: i paired with i'
    EL = EL.transpose(0, 2, 1, 3).reshape(Dh * Dh, Dh * Dh)
    return EL, _orig_env(T)[1]


def _project_wrong_leg(P, A, B):
    return _orig_project(P, A, B.transpose(0, 1, 3, 2))  # mistake: i <-> d


def _select_smallest(secL, secR, dcut, nfused):
    flip = [o.Sector(s.label, s.index, -s.lam, s.vec) for s in secL]
    sel = _orig_select(flip, flip, dcut, nfused)           # mistake: keeps the smallest
    return sel


def _run_wrong_lognorm(T, imps, lab_h, lab_v, sym, dcut, nsteps, first="y", norm="fro", **kw):
    r = _orig_run(T, imps, lab_h, lab_v, sym, dcut, nsteps, first, norm, **kw)
    # mistake: weight ln c_n by 2^-(n-1)
    extra = sum(s.lnc / 2.0 ** (i + 1) for i, s in enumerate(r.steps))
    r.lnz_per_site += extra
    return r


MUTATIONS = {
    "charge_orientation": ("initial_tensors", _wrong_orientation),
    "dropped_sqrt": ("initial_tensors", _no_sqrt),
    "env_transposed_operand": ("environments", _env_transposed),
    "projection_wrong_leg": ("project", _project_wrong_leg),
    "keeps_smallest": ("select_states", _select_smallest),
    "lognorm_weight": ("hotrg_run", _run_wrong_lognorm),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_mutation_is_caught(name, monkeypatch):
    attr, fn = MUTATIONS[name]
    monkeypatch.setattr(o, attr, fn)
    _expect_some_pin_fails(_small_pins())


def test_impurity_half_factor_is_caught(monkeypatch):
    orig = o.project

    def doubled(P, A, B):
        out = orig(P, A, B)
        return out if A is B else 2.0 * out      # mistake: impurity without the 1/2
    monkeypatch.setattr(o, "project", doubled)
    _expect_some_pin_fails([
        lambda: pins.test_two_by_two_theta_quadrature(0.9, 0.6, 0.25, 0.0),
        lambda: pins.test_four_by_two_brute_force("y", 0.3, 0.2),
    ])


_orig_cc = o.char_coeffs
_orig_ff = o.field_factors
_orig_ll = o.leg_labels
_orig_fl = o.fuse_labels

HARMONIC_MUTATIONS = {
    # mistake: the second coupling stays cos 2 phi whatever q is
    "coupling_harmonic_fixed": ("char_coeffs",
                                lambda beta, delta, nmax, nquad=4096, q=2:
                                _orig_cc(beta, delta, nmax, nquad, 2)),
    # mistake: h1 and the second impurity stay on cos 2 theta
    "field_harmonic_fixed": ("field_factors",
                             lambda beta, h, h1, qmax, lmax=50, q=2:
                             _orig_ff(beta, h, h1, qmax, lmax, 2)),
    # mistake: Z2 parities instead of charge mod q
    "sector_labels_mod_2": ("leg_labels", lambda nmax, sym, q=2: _orig_ll(nmax, sym, 2)),
}


def _harmonic_pins():
    return [
        lambda: pins.test_harmonic_q_quadrature_equals_bessel_series(3, 1.2, 0.7),
        lambda: pins.test_harmonic_q_closed_sums(3, 1.0, 0.5),
        pins.test_harmonic_q_field_factors,
        lambda: pins.test_harmonic_q_two_by_two_theta_quadrature(3, 1.0, 0.3, 0.0, 0.3),
        pins.test_harmonic_q_sectors_do_not_change_truncated_runs,
    ]


@pytest.mark.parametrize("name", sorted(HARMONIC_MUTATIONS))
def test_harmonic_mutation_is_caught(name, monkeypatch):
    attr, fn = HARMONIC_MUTATIONS[name]
    monkeypatch.setattr(o, attr, fn)
    _expect_some_pin_fails(_harmonic_pins())
