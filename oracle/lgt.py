"""FP64 CPU oracle of the configurational-temperature estimator for compact
U(1) lattice gauge theory.

TEST INFRASTRUCTURE ONLY. This module is the plain, slow reference the GPU
library's estimator is checked against. It shares no code with the HIP path.
Only the test suite and the CPU-baseline leg of the benchmark may import it.

What it computes, and where the thesis defines it:

* Link angles theta_mu(n) on a periodic d-dimensional lattice
  L_0 x ... x L_{d-1}, mu = 0..d-1 (Ch. 5, introduction: U_mu(n) =
  exp(i theta_mu(n))). Array layout: theta[mu, x_{d-1}, ..., x_1, x_0], so
  that x_0 runs fastest in memory; a batch of configurations adds a leading
  axis.
* Plaquette angles theta_{mu nu}(n) = theta_mu(n) + theta_nu(n + mu) -
  theta_mu(n + nu) - theta_nu(n) for mu < nu, and the Wilson action
  S = beta sum_{n, mu < nu} (1 - cos theta_{mu nu}(n)) (Ch. 5,
  introduction).
* Gradient and Hessian of the action scaled by 1/beta,
  g_l = (1/beta) dS/dtheta_l and h_lm = (1/beta) d^2 S / dtheta_l dtheta_m
  (Ch. 5, eq. grad_hess; the two-dimensional expressions of Sec.
  "Two-Dimensional Theory" are the case d = 2). Each plaquette P adds
  s_{P,l} sin theta_P to g_l and s_{P,l} s_{P,m} cos theta_P to h_lm for
  every pair of its four links, where s_{P,l} = +-1 is the sign of
  theta_l in theta_P.
* The estimator beta_hat = Tr h / |g|^2 - 2 g^T h g / |g|^4 (Ch. 4, eq.
  another-form, the divergence of g / |g|^2; Ch. 5, eq. beta_lat), its
  diagonal form Tr h / |g|^2 (Ch. 5, Sec. "Four-Dimensional Theory", which
  drops the Hessian's off-diagonal part) and the directional sums per link
  direction (Ch. 5, Sec. "Two-Dimensional Theory", beta_x). With the 1/beta
  scaling, beta_hat estimates the coupling itself.
* The plaquette average <P> = mean over the lattice of cos theta_{mu nu}
  (Ch. 5, Sec. "Four-Dimensional Theory").
* A heat-bath sweep that draws every link from its exact conditional
  distribution, used only by the tests to produce equilibrium
  configurations (not a method of the thesis, which uses HMC).

Pinned by tests/test_oracle_lgt.py: gauge invariance and known-flux
configurations (plaquette), finite differences of the action (gradient,
Hessian diagonal, g^T h g, and the divergence form of the estimator), the
exact identity <h_l> = beta <g_l^2> under a link's conditional distribution
(by quadrature), and equilibrium configurations against the closed form
<cos theta_P> = I_1(beta) / I_0(beta) of the two-dimensional theory (Ch. 5,
eq. plaq_2d) and against the exact ratio <Tr h> / <|g|^2> = beta.
"""

from __future__ import annotations

import itertools

import numpy as np
import scipy.sparse as sp


def _axis(d: int, mu: int) -> int:
    """Array axis of direction mu in a site array of a d-dimensional
    lattice (x_0 is the last axis)."""
    return d - 1 - mu


def shift(a: np.ndarray, d: int, mu: int, k: int = 1) -> np.ndarray:
    """b[n] = a[n + k mu] on the periodic lattice."""
    return np.roll(a, -k, axis=_axis(d, mu))


def plaquettes(theta: np.ndarray):
    """[(mu, nu, theta_{mu nu}(n) as a site array)] for mu < nu. Every
    extent must be at least 2, so that the four links of a plaquette are
    distinct (with an extent of 1, theta_nu(n + mu) is theta_nu(n) and the
    per-plaquette Hessian terms below would count a link twice)."""
    d = theta.shape[0]
    if min(theta.shape[1:]) < 2:
        raise ValueError("every lattice extent must be at least 2")
    out = []
    for mu, nu in itertools.combinations(range(d), 2):
        t = theta[mu] + shift(theta[nu], d, mu) - shift(theta[mu], d, nu) - theta[nu]
        out.append((mu, nu, t))
    return out


def action(theta: np.ndarray, beta: float) -> float:
    return float(beta * sum(np.sum(1.0 - np.cos(t)) for _, _, t in plaquettes(theta)))


def _plaquette_links(mu: int, nu: int):
    """The four links of theta_{mu nu}(n) as (direction, displacement from
    n, sign)."""
    return [(mu, {}, +1), (nu, {mu: 1}, +1), (mu, {nu: 1}, -1), (nu, {}, -1)]


def _back(a: np.ndarray, d: int, disp: dict) -> np.ndarray:
    """Move a plaquette quantity from its base site n to the site n + disp of
    one of its links: b[n + disp] = a[n]."""
    for ax, k in disp.items():
        a = np.roll(a, k, axis=_axis(d, ax))
    return a


def gradient_hdiag(theta: np.ndarray):
    """(g, hdiag) with the layout of theta: every plaquette adds
    s sin theta_P to g and cos theta_P to the Hessian diagonal of each of its
    links."""
    d = theta.shape[0]
    g = np.zeros_like(theta)
    hd = np.zeros_like(theta)
    for mu, nu, t in plaquettes(theta):
        s_t, c_t = np.sin(t), np.cos(t)
        for lmu, disp, sgn in _plaquette_links(mu, nu):
            g[lmu] += sgn * _back(s_t, d, disp)
            hd[lmu] += _back(c_t, d, disp)
    return g, hd


def hessian(theta: np.ndarray) -> sp.csr_matrix:
    """h as a sparse matrix over link indices l = mu V + (flat site): every
    plaquette adds s_l s_m cos theta_P at (l, m) for each pair of its links
    (including l = m)."""
    d = theta.shape[0]
    V = theta[0].size
    sites = np.arange(V).reshape(theta.shape[1:])
    rows, cols, vals = [], [], []
    for mu, nu, t in plaquettes(theta):
        c_t = np.cos(t).ravel()
        links = [(lmu * V + _site_of(sites, d, disp).ravel(), sgn)
                 for lmu, disp, sgn in _plaquette_links(mu, nu)]
        for (li, si), (lj, sj) in itertools.product(links, links):
            rows.append(li)
            cols.append(lj)
            vals.append(si * sj * c_t)
    n = d * V
    return sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(n, n)).tocsr()


def _site_of(sites: np.ndarray, d: int, disp: dict) -> np.ndarray:
    """Flat index of n + disp for every base site n."""
    out = sites
    for ax, k in disp.items():
        out = shift(out, d, ax, k)
    return out


def estimator_value(trace_h: float, sum_g2: float, ghg: float) -> float:
    """Tr h / |g|^2 - 2 g^T h g / |g|^4 (Ch. 4, eq. another-form)."""
    return trace_h / sum_g2 - 2.0 * ghg / sum_g2 ** 2


def estimator(theta: np.ndarray, full: bool = True) -> dict:
    """Sums and estimators of one configuration theta[mu, ...]."""
    d = theta.shape[0]
    g, hd = gradient_hdiag(theta)
    sum_g2 = float(np.sum(g * g))
    sum_h = float(np.sum(hd))
    plaq = [np.cos(t) for _, _, t in plaquettes(theta)]
    out = {
        "sum_g2": sum_g2,
        "sum_h": sum_h,
        "plaquette": float(np.mean(np.stack(plaq))),
        "beta_diag": sum_h / sum_g2,
        "sum_g2_dir": [float(np.sum(g[mu] ** 2)) for mu in range(d)],
        "sum_h_dir": [float(np.sum(hd[mu])) for mu in range(d)],
        "g_h_g": float("nan"),
        "beta_full": float("nan"),
    }
    if full:
        H = hessian(theta)
        gv = g.ravel()
        ghg = float(gv @ (H @ gv))
        out["g_h_g"] = ghg
        out["trace_h"] = float(H.diagonal().sum())
        out["beta_full"] = estimator_value(out["trace_h"], sum_g2, ghg)
    return out


def heatbath_sweep(theta: np.ndarray, beta: float, rng: np.random.Generator) -> None:
    """One sweep over every link, each drawn from its conditional
    distribution exp(-S) with the other links fixed (in place). With the
    other links fixed, sum over the link's plaquettes of cos theta_P as a
    function of the new angle t is Re(e^{i t} Z), Z = e^{-i theta_l}
    (h_l + i g_l), so t follows a von Mises law with mean -arg Z and
    concentration beta |Z|. Links of one direction whose coordinates
    transverse to it have the same parity share no plaquette and are drawn
    together."""
    d = theta.shape[0]
    if any(n % 2 for n in theta.shape[1:]):
        raise ValueError("the two-colour sweep needs even lattice extents")
    grids = np.meshgrid(*[np.arange(n) for n in theta.shape[1:]], indexing="ij")
    coord = {mu: grids[_axis(d, mu)] for mu in range(d)}
    for mu in range(d):
        par = sum(coord[nu] for nu in range(d) if nu != mu) % 2
        for color in (0, 1):
            g, hd = gradient_hdiag(theta)
            z = np.exp(-1j * theta[mu]) * (hd[mu] + 1j * g[mu])
            new = rng.vonmises(-np.angle(z), beta * np.abs(z))
            m = par == color
            theta[mu][m] = new[m]


def wrap(theta: np.ndarray) -> np.ndarray:
    """Angles mapped to (-pi, pi]."""
    return np.pi - np.mod(np.pi - theta, 2.0 * np.pi)
