"""Seeded synthetic parameter points for the gXY HOTRG workloads.

This module only builds parameter sets (inverse temperature, deformation,
fields, charge cutoff, bond dimension, step count). It holds none of the
method's arithmetic, so both the GPU path's tests and the CPU oracle's
tests can draw the same inputs from it.

Workload families (the thesis studies the gXY model of Ch. 3, eq. for the
gXY Hamiltonian with J = Delta, J1 = 1 - Delta, q = 2):

* ``single``   beta=1.0, Delta=0.5, nmax=3 (D0=7), Dcut=12, 30 steps.
* ``cv``       beta in {0.9,1.0,1.1} x {b-1e-3, b, b+1e-3}, Delta=0.3,
               nmax=10 (D0=21), Dcut=48, 40 steps, both impurity chains.
* ``precision`` beta=1.2, Delta=0.7, nmax=10, Dcut in {64,96}, 40 steps.
* ``grid``     16x16 (beta, Delta) grid, beta in [0.5,1.5], Delta in [0,1]
               (endpoints included), nmax=10, 40 steps, Dcut per point drawn
               from {24,32,48,64} by SplitMix64 (seed 20536).
* ``lgt``      link configurations of compact U(1) lattice gauge theory for
               the configurational-temperature estimator (Ch. 4-5): seeded
               uniform or gauge-transformed Gaussian angles; the throughput
               batch is 16 configurations of 32^4.
"""

from __future__ import annotations

from dataclasses import dataclass, field, asdict, replace
from typing import List

IMP_COS1 = 1
IMP_COS2 = 2
IMP_COS1_SQ = 4
IMP_COS2_SQ = 8

PREC_FP64 = 0
PREC_FP32 = 1
PREC_BF16X3 = 2

# Finite-difference steps and central field values used for C_v, chi, chi_n.
BETA_FD_STEP = 1e-3
FIELD_CENTER = 1e-3
FIELD_FD_STEP = 1e-4


@dataclass
class Point:
    """One HOTRG run: model parameters plus numerical cutoffs."""

    beta: float
    delta: float
    h: float = 0.0
    h1: float = 0.0
    nmax: int = 3
    dcut: int = 12
    nsteps: int = 30
    nquad: int = 4096
    impurities: int = IMP_COS1 | IMP_COS2
    prec: int = PREC_FP64
    fp64_steps: int = 0
    q: int = 2

    def as_dict(self):
        return asdict(self)

    def with_(self, **kw) -> "Point":
        return replace(self, **kw)


def single_point() -> Point:
    """beta=1, Delta=0.5, |n|<=3, Dcut=12, 30 steps, cos and cos2 chains."""
    return Point(beta=1.0, delta=0.5, nmax=3, dcut=12, nsteps=30)


def cv_points() -> List[Point]:
    """Specific-heat triplets around beta in {0.9,1.0,1.1} at Delta=0.3."""
    pts = []
    for b in (0.9, 1.0, 1.1):
        for s in (-1, 0, 1):
            pts.append(Point(beta=b + s * BETA_FD_STEP, delta=0.3, nmax=10,
                             dcut=48, nsteps=40))
    return pts


def precision_point(dcut: int = 64, prec: int = PREC_FP64,
                    fp64_steps: int = 0, impurities: int = IMP_COS1 | IMP_COS2,
                    beta: float = 1.2) -> Point:
    """beta=1.2, Delta=0.7, |n|<=10, Dcut in {64, 96}, 40 steps."""
    return Point(beta=beta, delta=0.7, nmax=10, dcut=dcut, nsteps=40,
                 impurities=impurities, prec=prec, fp64_steps=fp64_steps)


def splitmix64(state: int):
    """SplitMix64 (Steele, Lea, Flood 2014): returns (next_state, output)."""
    mask = (1 << 64) - 1
    state = (state + 0x9E3779B97F4A7C15) & mask
    z = state
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & mask
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & mask
    z = z ^ (z >> 31)
    return state, z


GRID_DCUTS = (24, 32, 48, 64)
GRID_SEED = 20536


def grid_dcuts(n: int = 256, seed: int = GRID_SEED) -> List[int]:
    """Dcut of grid point k: {24,32,48,64}[top two bits of the k-th output]."""
    out = []
    s = seed
    for _ in range(n):
        s, z = splitmix64(s)
        out.append(GRID_DCUTS[z >> 62])
    return out


@dataclass
class GridPoint:
    beta: float
    delta: float
    dcut: int
    index: int


def grid_points(nb: int = 16, nd: int = 16, nmax: int = 10,
                nsteps: int = 40) -> List[GridPoint]:
    """beta_i = 0.5 + i/(nb-1), Delta_j = j/(nd-1), k = nd*i + j."""
    dc = grid_dcuts(nb * nd)
    pts = []
    for i in range(nb):
        for j in range(nd):
            k = nd * i + j
            pts.append(GridPoint(beta=0.5 + i / (nb - 1), delta=j / (nd - 1),
                                 dcut=dc[k], index=k))
    return pts


def observable_runs(beta: float, delta: float, dcut: int, nmax: int = 10,
                    nsteps: int = 40, prec: int = PREC_FP64,
                    fp64_steps: int = 0, db: float = BETA_FD_STEP) -> List[Point]:
    """The seven runs behind (f, C_v, chi, chi_n) at one (beta, Delta).

    Order: beta-db, beta, beta+db (zero field, no chains);
    h = hc-dh, hc+dh (cos chain); h1 = hc-dh, hc+dh (cos2 chain).
    """
    base = Point(beta=beta, delta=delta, nmax=nmax, dcut=dcut, nsteps=nsteps,
                 impurities=0, prec=prec, fp64_steps=fp64_steps)
    hc, dh = FIELD_CENTER, FIELD_FD_STEP
    return [
        base.with_(beta=beta - db),
        base,
        base.with_(beta=beta + db),
        base.with_(h=hc - dh, impurities=IMP_COS1),
        base.with_(h=hc + dh, impurities=IMP_COS1),
        base.with_(h1=hc - dh, impurities=IMP_COS2),
        base.with_(h1=hc + dh, impurities=IMP_COS2),
    ]


def zero_field_runs(beta: float, delta: float, dcut: int, nmax: int = 10,
                    nsteps: int = 40, prec: int = PREC_FP64,
                    fp64_steps: int = 0, db: float = BETA_FD_STEP) -> List[Point]:
    """The three runs behind (f, C_v, chi, chi_n) at one (beta, Delta) by the
    zero-field route: beta-db and beta+db without chains, and beta with the
    second-moment chains of cos theta and cos 2 theta (chi, chi_n at h = 0).

    Order: beta-db, beta (chains), beta+db.
    """
    base = Point(beta=beta, delta=delta, nmax=nmax, dcut=dcut, nsteps=nsteps,
                 impurities=0, prec=prec, fp64_steps=fp64_steps)
    return [
        base.with_(beta=beta - db),
        base.with_(impurities=IMP_COS1_SQ | IMP_COS2_SQ),
        base.with_(beta=beta + db),
    ]


# ---------------------------------------------------------------------------
# Learned surrogate: seeded initial weights and train/validation split.
# ---------------------------------------------------------------------------

MLP_SEED = 20536
MLP_LAYERS = ((128, 2), (128, 128), (4, 128))   # (fan_out, fan_in) per layer
MLP_NPARAM = sum(o * i + o for o, i in MLP_LAYERS)  # 17412


def mlp_init_params(seed: int = MLP_SEED) -> List[float]:
    """Xavier-uniform weights, zero biases, as one flat vector.

    Layout: W1[128][2], b1[128], W2[128][128], b2[128], W3[4][128], b3[4]
    (row-major). Weight w of a layer with limit a = sqrt(6 / (fan_in +
    fan_out)) is (2u - 1) a with u = (z >> 11) 2^-53 from consecutive
    SplitMix64 outputs z of one stream seeded with ``seed`` (weights of W1,
    then W2, then W3; biases draw nothing).
    """
    import math
    out: List[float] = []
    s = seed
    for fo, fi in MLP_LAYERS:
        a = math.sqrt(6.0 / (fi + fo))
        for _ in range(fo * fi):
            s, z = splitmix64(s)
            u = (z >> 11) * 2.0 ** -53
            out.append((2.0 * u - 1.0) * a)
        out.extend([0.0] * fo)
    return out


def mlp_split(n: int, seed: int = MLP_SEED, train_frac: float = 0.9):
    """Seeded 90/10 split of n samples: Fisher-Yates with SplitMix64, the
    first round(train_frac n) indices of the permutation train."""
    perm = list(range(n))
    s = seed
    for i in range(n - 1, 0, -1):
        s, z = splitmix64(s)
        j = z % (i + 1)
        perm[i], perm[j] = perm[j], perm[i]
    ntr = int(round(train_frac * n))
    return perm[:ntr], perm[ntr:]


# ---------------------------------------------------------------------------
# compact U(1) lattice gauge theory: link configurations for the
# configurational-temperature estimator (include/gxy_lgt.h)
# ---------------------------------------------------------------------------
# The thesis's four-dimensional study runs on 8^4 lattices (Ch. 5, Sec.
# "Four-Dimensional Theory"); the throughput workload is a batch of larger
# lattices of the same theory.
LGT_BENCH_DIMS = (32, 32, 32, 32)
LGT_BENCH_CONF = 16
LGT_SEED = 0x5EED_1A77


def lgt_configs(nconf: int, dims, seed: int = LGT_SEED, kind: str = "gauge_noise",
                sigma: float = 0.52):
    """Seeded link angles as a numpy array of shape (nconf, d, L_{d-1}, ...,
    L_0) (x_0 fastest, the library's layout), d = len(dims).

    kind "uniform": independent angles uniform on (-pi, pi] (the
    configurations of infinite temperature, beta = 0).
    kind "gauge_noise": theta_mu(x) = alpha(x) + eps_mu(x) - alpha(x + mu),
    alpha uniform on (-pi, pi] and eps Gaussian of width sigma, mapped to
    (-pi, pi]: every link looks uniformly random while the plaquettes stay
    near e^{-2 sigma^2} on average (0.58 at sigma = 0.52, the thesis's 8^4
    plaquette near beta = 1), a synthetic stand-in for thermalised
    configurations (no Monte Carlo is run)."""
    import numpy as np

    rng = np.random.default_rng(seed)
    d = len(dims)
    shape = (nconf, d) + tuple(reversed(dims))
    if kind == "uniform":
        th = rng.uniform(-np.pi, np.pi, size=shape)
    elif kind == "gauge_noise":
        alpha = rng.uniform(-np.pi, np.pi, size=(nconf,) + tuple(reversed(dims)))
        eps = rng.normal(0.0, sigma, size=shape)
        th = np.empty(shape)
        for mu in range(d):
            # alpha(x + mu): x_mu is array axis 1 + (d - 1 - mu) of alpha
            th[:, mu] = alpha + eps[:, mu] - np.roll(alpha, -1, axis=1 + (d - 1 - mu))
    else:
        raise ValueError(kind)
    return np.pi - np.mod(np.pi - th, 2.0 * np.pi)
