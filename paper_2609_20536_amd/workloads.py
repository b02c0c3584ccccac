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
"""

from __future__ import annotations

from dataclasses import dataclass, field, asdict, replace
from typing import List

IMP_COS1 = 1
IMP_COS2 = 2

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
                    fp64_steps: int = 0) -> List[Point]:
    """The seven runs behind (f, C_v, chi, chi_n) at one (beta, Delta).

    Order: beta-db, beta, beta+db (zero field, no chains);
    h = hc-dh, hc+dh (cos chain); h1 = hc-dh, hc+dh (cos2 chain).
    """
    base = Point(beta=beta, delta=delta, nmax=nmax, dcut=dcut, nsteps=nsteps,
                 impurities=0, prec=prec, fp64_steps=fp64_steps)
    db, hc, dh = BETA_FD_STEP, FIELD_CENTER, FIELD_FD_STEP
    return [
        base.with_(beta=beta - db),
        base,
        base.with_(beta=beta + db),
        base.with_(h=hc - dh, impurities=IMP_COS1),
        base.with_(h=hc + dh, impurities=IMP_COS1),
        base.with_(h1=hc - dh, impurities=IMP_COS2),
        base.with_(h1=hc + dh, impurities=IMP_COS2),
    ]
