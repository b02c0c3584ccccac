"""FP64 CPU oracle of HOTRG for the 2D generalized XY model.

TEST INFRASTRUCTURE ONLY. This module is the plain, slow reference the GPU
library is checked against. It shares no code with the HIP path. Only the
test suite, the smoke check and the CPU-baseline leg of the benchmark may
import it.

What it computes, and where the thesis defines it:

* Character coefficients t_n of the bond weight
  w(phi) = exp(beta [Delta cos phi + (1 - Delta) cos q phi]) (Ch. 3, Sec.
  "Tensor Formulation", eq. for a_n): t_n = (1/2pi) int w(phi) cos(n phi).
  The normative evaluation is the periodic trapezoid rule on nquad points;
  the Bessel-product series of that equation is the cross-check. The thesis
  writes the Hamiltonian (Ch. 3, Sec. "The Generalized XY Model", eq.
  gXY_ham) for a general harmonic q and studies q = 2, the default here;
  q >= 3 is the extension its conclusions name.
* Site tensor T_{n1 n2 n3 n4} = sqrt(prod a_nk) * sum_l I_{Q+ql}(beta h)
  I_l(beta h1), Q = n1 + n2 - n3 - n4, legs (top, right, bottom, left)
  (Ch. 3, Sec. "Derivation of Tensors", final site-tensor equation, written
  there for q = 2), and the impurity tensors for <cos theta> and
  <cos q theta> (Ch. 3, Sec. "Numerical Results", the two impure-tensor
  equations). The field h1 couples to cos q theta (for q = 2 the thesis's
  nematic field).
* HOTRG coarse graining (Ch. 2, Sec. "Higher-Order Tensor Renormalization
  Group Method"): the fused two-site tensor M (eq. Mtensor), the mode
  unfoldings' Gram matrices whose eigenvectors are the HOSVD factors U, V
  (eq. hosvd), the discarded weights eps_1, eps_2 and the side choice, the
  projector built from the leading Dcut vectors, and the renormalised tensor
  P^T M P (eq. renormalizedT); directions alternate.
* Normalisation after every step (Ch. 2, Sec. "Computational Cost") with the
  running log-norm, the final tensor trace on the periodic 1x1 torus, the
  impurity ratio M = P/Z, and finite-difference observables C_v, chi
  (Ch. 3, eqs. spech, susc, mag).
* Zero-field susceptibility from summed insertions (a variant of the
  impurity method of Ch. 3 that the thesis does not use): besides the
  one-insertion tensor, the tensor with two insertions averaged over ordered
  pairs of sites is carried through the steps, so <m^2> = Tr T2 / Tr T for
  the site average m, and chi = beta V (<m^2> - <m>^2) (eq. susc by the
  fluctuation relation) from one zero-field run.

Readings where the thesis is silent or garbled (each is restated in the
design notes):

* Leg order T[l, r, u, d]; charge law q_l + q_d = q_r + q_u (the thesis's
  n1 + n2 - n3 - n4 with (n1, n2, n3, n4) = (u, r, d, l)).
* Every step contracts the vertical bond of two vertically adjacent
  tensors ("y-step"); an x-step is the y-step applied to the transposed
  tensor T[u, d, l, r] and transposed back. The first step is a y-step.
* The eigendecomposition is done per symmetry sector (U(1) charge at
  h = h1 = 0, Z_q label (charge mod q) at h = 0 != h1, one dense block
  otherwise).
* Truncation keeps Dcut states chosen greedily: repeatedly take, among the
  remaining eigenvalues within TIE_REL * lambda_max of the largest
  remaining one, the state with the smallest (|q|, q, rank in its sector).
  eps = sum of the eigenvalues not kept. The right side is used only if
  eps_R < eps_L - SIDE_TOL * lambda_max; ties go to the left side. The
  model's reflection symmetry makes eps_L = eps_R exactly at many steps, and
  two FP64 evaluations of these sums over ~Dh^2 eigenvalues differ by up to
  ~Dh^2 eps lambda_max, so SIDE_TOL (1e-10) sits well above that level.
* The impurity tensor is updated as 1/2 [Proj(T_X, T) + Proj(T, T_X)] with
  the pure tensor's projector and norm.
* The normalisation constant is the Frobenius norm.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

TIE_REL = 1e-12
SIDE_TOL = 1e-10

IMP_COS1 = 1
IMP_COS2 = 2
# second moments of the site-averaged insertions (zero-field susceptibilities)
IMP_COS1_SQ = 4
IMP_COS2_SQ = 8
SECOND_OF = {IMP_COS1_SQ: IMP_COS1, IMP_COS2_SQ: IMP_COS2}

SYM_U1 = 0     # integer charges, fused by addition
SYM_NONE = 1   # a single sector (all labels 0)
SYM_Z2 = 2     # Z_q labels (charge mod q; parities for q = 2), fused by addition mod q


# --------------------------------------------------------------------------
# Special functions and character coefficients
# --------------------------------------------------------------------------

def bessel_i(k: int, x: float) -> float:
    """Modified Bessel function I_k(x) of integer order by its power series.

    I_k(x) = sum_j (x/2)^(2j+k) / (j! (j+k)!), with I_{-k} = I_k. All terms
    are positive, so the sum is accurate to rounding for the arguments used
    here. Pinned by comparison with scipy.special.iv in the tests.
    """
    k = abs(int(k))
    if x == 0.0:
        return 1.0 if k == 0 else 0.0
    half = 0.5 * x
    # first term (x/2)^k / k!, built by products to avoid overflow in k!
    term = 1.0
    for j in range(1, k + 1):
        term *= half / j
    total = term
    j = 0
    while True:
        j += 1
        term *= half * half / (j * (j + k))
        total += term
        if term <= 1e-18 * total:
            break
    return total


def char_coeffs(beta: float, delta: float, nmax: int,
                nquad: int = 4096, q: int = 2) -> np.ndarray:
    """t_n for n = -nmax..nmax by the periodic trapezoid rule on nquad points.

    t_n = (1/Q) sum_{k<Q} w(phi_k) cos(n phi_k), phi_k = 2 pi k / Q,
    w(phi) = exp(beta [Delta cos phi + (1-Delta) cos q phi]) (Ch. 3, the
    character-expansion coefficient a_n written as a Fourier integral).
    The negative orders are mirrored (t_{-n} = t_n holds exactly since w is
    even) and the values are clamped at 0 (the exact coefficients are
    non-negative; odd orders at Delta = 0 come out at rounding level).

    Pinned by: Bessel-product series, closed sums sum t_n = e^beta,
    sum (-1)^n t_n = e^(beta(-Delta + (1-Delta)(-1)^q)), Parseval
    sum t_n^2 = t_0(2 beta), the Delta = 1 and Delta = 0 reductions, beta = 0.
    """
    if nquad <= 2 * nmax:
        raise ValueError("nquad must exceed 2*nmax")
    phi = 2.0 * np.pi * np.arange(nquad, dtype=np.float64) / nquad
    w = np.exp(beta * (delta * np.cos(phi) + (1.0 - delta) * np.cos(q * phi)))
    half = np.array([np.sum(w * np.cos(n * phi)) / nquad
                     for n in range(nmax + 1)])
    half = np.maximum(half, 0.0)
    return np.concatenate([half[:0:-1], half])


def char_coeffs_bessel(beta: float, delta: float, nmax: int,
                       mmax: int = 50, q: int = 2) -> np.ndarray:
    """a_n = sum_{|m|<=mmax} I_{n-qm}(beta Delta) I_m(beta (1-Delta)).

    The thesis's Bessel-product form (Ch. 3, eq. a_n, there with q = 2),
    truncated at |m| <= mmax as the thesis does. Used as an independent check
    of char_coeffs.
    """
    out = []
    for n in range(-nmax, nmax + 1):
        s = 0.0
        for m in range(-mmax, mmax + 1):
            s += bessel_i(n - q * m, beta * delta) * bessel_i(m, beta * (1.0 - delta))
        out.append(s)
    return np.array(out)


def field_factors(beta: float, h: float, h1: float, qmax: int,
                  lmax: int = 50, q: int = 2) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Field factors of the pure and the two impure site tensors.

    For Q in [-qmax, qmax] (array index Q + qmax):
      F(Q)   = sum_l I_{Q+ql}(beta h) I_l(beta h1)
      F_M(Q) = sum_l I_l(beta h1) [I_{Q+ql-1}(beta h) + I_{Q+ql+1}(beta h)]/2
      F_M1(Q)= sum_l I_{Q+ql}(beta h) [I_{l+1}(beta h1) + I_{l-1}(beta h1)]/2
    with |l| <= lmax (Ch. 3, final site-tensor equation and the two
    impure-tensor equations, there with q = 2: the Fourier coefficients of
    exp(beta h cos th + beta h1 cos q th) times 1, cos th, cos q th). At
    h = h1 = 0 these are exactly delta_{Q,0}, (delta_{Q,1} + delta_{Q,-1})/2,
    (delta_{Q,q} + delta_{Q,-q})/2.
    """
    qs = np.arange(-qmax, qmax + 1)
    F = np.zeros(len(qs))
    FM = np.zeros(len(qs))
    FM1 = np.zeros(len(qs))
    if h == 0.0 and h1 == 0.0:
        F[qs == 0] = 1.0
        FM[np.abs(qs) == 1] = 0.5
        FM1[np.abs(qs) == q] = 0.5
        return F, FM, FM1
    x, x1 = beta * h, beta * h1
    for a, Q in enumerate(qs):
        f = fm = fm1 = 0.0
        for l in range(-lmax, lmax + 1):
            il1 = bessel_i(l, x1)
            iq = bessel_i(Q + q * l, x)
            f += iq * il1
            fm += il1 * 0.5 * (bessel_i(Q + q * l - 1, x) + bessel_i(Q + q * l + 1, x))
            fm1 += iq * 0.5 * (bessel_i(l + 1, x1) + bessel_i(l - 1, x1))
        F[a], FM[a], FM1[a] = f, fm, fm1
    return F, FM, FM1


def square_factors(qmax: int, q: int = 2) -> Tuple[np.ndarray, np.ndarray]:
    """Zero-field factors of the site tensors with cos^2 theta and cos^2 q theta
    inserted: the Fourier coefficients (1/2pi) int cos^2(k th) e^{-i Q th} dth
    = delta_{Q,0}/2 + (delta_{Q,2k} + delta_{Q,-2k})/4 for k = 1 and k = q
    (index Q + qmax), the same integral over the site angle that gives the
    impure tensors of Ch. 3 (Sec. Numerical Results) with cos^2 in place of
    cos. Pinned by: beta = 0 (<m^2> V = 1/2 exactly) and the 2x2 / 4x2 tori.
    """
    qs = np.arange(-qmax, qmax + 1)
    out = []
    for k in (1, q):
        f = np.zeros(len(qs))
        f[qs == 0] += 0.5
        f[np.abs(qs) == 2 * k] += 0.25
        out.append(f)
    return out[0], out[1]


def symmetry_of(h: float, h1: float) -> int:
    """Symmetry left by the fields: U(1) at h = h1 = 0, Z_q at h = 0, else none."""
    if h == 0.0 and h1 == 0.0:
        return SYM_U1
    if h == 0.0:
        return SYM_Z2
    return SYM_NONE


def leg_labels(nmax: int, sym: int, q: int = 2) -> np.ndarray:
    n = np.arange(-nmax, nmax + 1)
    if sym == SYM_U1:
        return n.copy()
    if sym == SYM_Z2:
        return np.mod(n, q)
    return np.zeros_like(n)


def fuse_labels(qa: np.ndarray, qb: np.ndarray, sym: int, q: int = 2) -> np.ndarray:
    """Label of the fused index (a, b) -> a * len(qb) + b."""
    s = qa[:, None] + qb[None, :]
    if sym == SYM_Z2:
        s = np.mod(s, q)
    elif sym == SYM_NONE:
        s = np.zeros_like(s)
    return s.reshape(-1)


def initial_tensors(beta: float, delta: float, h: float, h1: float,
                    nmax: int, nquad: int = 4096,
                    impurities: int = 0, q: int = 2) -> Tuple[np.ndarray, Dict[int, np.ndarray]]:
    """Site tensor T[l, r, u, d] and the requested impurity tensors.

    T[l,r,u,d] = sqrt(t_l t_r t_u t_d) F(n_u + n_r - n_d - n_l); the cos
    impurity uses F_M and the cos q impurity F_M1 in place of F.
    Pinned by: the 1x1-torus trace (sum t)^2, tiny-torus brute force and
    theta quadrature (pure and with fields).
    """
    t = char_coeffs(beta, delta, nmax, nquad, q)
    n = np.arange(-nmax, nmax + 1)
    F, FM, FM1 = field_factors(beta, h, h1, 4 * nmax, q=q)
    l, r, u, d = np.meshgrid(n, n, n, n, indexing="ij")
    Q = u + r - d - l
    amp = np.sqrt(t[l + nmax] * t[r + nmax] * t[u + nmax] * t[d + nmax])
    T = amp * F[Q + 4 * nmax]
    imps = {}
    if impurities & IMP_COS1:
        imps[IMP_COS1] = amp * FM[Q + 4 * nmax]
    if impurities & IMP_COS2:
        imps[IMP_COS2] = amp * FM1[Q + 4 * nmax]
    if impurities & (IMP_COS1_SQ | IMP_COS2_SQ):
        if h != 0.0 or h1 != 0.0:
            raise ValueError("second-moment insertions are defined at zero field only")
        F2, F2q = square_factors(4 * nmax, q)
        if impurities & IMP_COS1_SQ:
            imps[IMP_COS1_SQ] = amp * F2[Q + 4 * nmax]
        if impurities & IMP_COS2_SQ:
            imps[IMP_COS2_SQ] = amp * F2q[Q + 4 * nmax]
    return T, imps


# --------------------------------------------------------------------------
# One coarse-graining step (vertical bond contracted)
# --------------------------------------------------------------------------

def environments(T: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """Gram matrices of the left and right mode unfoldings of M.

    M[(l1 l2),(r1 r2),u,d] = sum_i T[l1,r1,u,i] T[l2,r2,i,d] (eq. Mtensor).
    E_L = M_(l) M_(l)^T and E_R = M_(r) M_(r)^T; their eigenvectors are the
    HOSVD factors U and V of eq. hosvd, and their eigenvalues the squared
    mode singular values |S_{i,:,:,:}|^2 that enter eps_1 and eps_2.
    Evaluated as E_L = sum_{i,i'} A[l1,i,l1',i'] B[l2,i,l2',i'] with
    A = sum_{r1,u} T T and B = sum_{r2,d} T T. Fused index (x, y) -> x*Dh + y.
    """
    Dh = T.shape[0]
    A = np.tensordot(T, T, axes=([1, 2], [1, 2]))      # [l1, i, l1', i']
    B = np.tensordot(T, T, axes=([1, 3], [1, 3]))      # [l2, i, l2', i']
    EL = np.tensordot(A, B, axes=([1, 3], [1, 3]))     # [l1, l1', l2, l2']
    EL = EL.transpose(0, 2, 1, 3).reshape(Dh * Dh, Dh * Dh)
    A = np.tensordot(T, T, axes=([0, 2], [0, 2]))      # [r1, i, r1', i']
    B = np.tensordot(T, T, axes=([0, 3], [0, 3]))      # [r2, i, r2', i']
    ER = np.tensordot(A, B, axes=([1, 3], [1, 3]))     # [r1, r1', r2, r2']
    ER = ER.transpose(0, 2, 1, 3).reshape(Dh * Dh, Dh * Dh)
    return EL, ER


@dataclass
class Sector:
    label: int
    index: np.ndarray      # positions in the fused index
    lam: np.ndarray        # eigenvalues, descending
    vec: np.ndarray        # eigenvectors as columns, same order


def sector_eigh(E: np.ndarray, labels: np.ndarray,
                basis_rng: Optional[np.random.Generator] = None) -> List[Sector]:
    """Eigendecomposition of the symmetric E restricted to each label sector.

    E commutes with the symmetry, so it is block diagonal in the fused label;
    each block is diagonalised by LAPACK's symmetric solver and sorted by
    decreasing eigenvalue. Eigenvector signs are fixed so the entry of
    largest magnitude is positive (a gauge choice that does not enter any
    output).

    basis_rng (test option): diagonalise Q^T E_s Q for a random orthogonal Q
    and rotate back. This is an equally valid backward-stable FP64 eigensolve
    with a different rounding pattern; comparing runs with and without it
    measures how far the run is fixed by FP64 eigensolver rounding at all
    (near-degenerate eigenvalues at the cut make the kept vectors
    ill-determined).
    """
    out = []
    for s in np.unique(labels):
        idx = np.nonzero(labels == s)[0]
        Es = E[np.ix_(idx, idx)]
        if basis_rng is not None and len(idx) > 1:
            Q = np.linalg.qr(basis_rng.standard_normal((len(idx), len(idx))))[0]
            w, v = np.linalg.eigh(Q.T @ Es @ Q)
            v = Q @ v
        else:
            w, v = np.linalg.eigh(Es)
        order = np.argsort(-w, kind="stable")
        w, v = w[order], v[:, order]
        big = np.argmax(np.abs(v), axis=0)
        sgn = np.sign(v[big, np.arange(v.shape[1])])
        sgn[sgn == 0] = 1.0
        out.append(Sector(int(s), idx, w, v * sgn))
    return out


def _greedy_pick(sectors: List[Sector], dcut: int) -> Tuple[List[Tuple[int, int]], int]:
    """Choose dcut (sector, rank) pairs by the tie rule; returns picks, #ties."""
    cand = []
    for si, s in enumerate(sectors):
        for k, lam in enumerate(s.lam):
            cand.append((float(lam), s.label, k, si))
    lam1 = max(c[0] for c in cand)
    tol = TIE_REL * abs(lam1)
    remaining = list(cand)
    picks = []
    ties = 0
    for _ in range(dcut):
        top = max(c[0] for c in remaining)
        group = [c for c in remaining if c[0] >= top - tol]
        if len(group) > 1:
            ties += 1
        best = min(group, key=lambda c: (abs(c[1]), c[1], c[2]))
        picks.append((best[3], best[2]))
        remaining.remove(best)
    return picks, ties


@dataclass
class Selection:
    P: np.ndarray             # isometry [Dh*Dh, D']
    labels: np.ndarray        # labels of the new bond states
    eps_l: float
    eps_r: float
    side: int                 # 0 = left (U), 1 = right (V)
    lam_max: float
    cut_gap: float
    ties: int
    sector_gap: float = math.inf   # smallest within-sector gap at the cut


def select_states(secL: List[Sector], secR: List[Sector], dcut: int,
                  nfused: int) -> Selection:
    """Truncation of the fused bond to dcut states and the choice of side.

    eps_side is the discarded weight (sum of eigenvalues not kept) of that
    side's environment (Ch. 2, HOTRG: eps_1, eps_2 and the rule that the
    side with the smaller discarded weight is truncated). The projector is
    the kept eigenvectors of that side, ordered by (label, rank).
    """
    res = {}
    for side, secs in ((0, secL), (1, secR)):
        picks, ties = _greedy_pick(secs, dcut)
        kept = {(si, k) for si, k in picks}
        eps = 0.0
        for si, s in enumerate(secs):
            for k, lam in enumerate(s.lam):
                if (si, k) not in kept:
                    eps += float(lam)
        lam1 = max(float(s.lam[0]) for s in secs)
        kept_l = [float(secs[si].lam[k]) for si, k in picks]
        disc_l = [float(lam) for si, s in enumerate(secs)
                  for k, lam in enumerate(s.lam) if (si, k) not in kept]
        # cut gap: smallest kept minus largest discarded eigenvalue
        gap = (min(kept_l) - max(disc_l)) / lam1 if lam1 > 0 else 0.0
        # the same within each sector that has both kept and discarded
        # states (a diagnostic: a small value means the kept directions of
        # that sector are fixed only to eps ||E|| / gap; a small cut gap
        # between different sectors is settled exactly by the tie rule)
        sgap = math.inf
        for si, s in enumerate(secs):
            kin = [float(lam) for k, lam in enumerate(s.lam) if (si, k) in kept]
            kout = [float(lam) for k, lam in enumerate(s.lam) if (si, k) not in kept]
            if kin and kout and lam1 > 0:
                sgap = min(sgap, (min(kin) - max(kout)) / lam1)
        res[side] = (picks, eps, lam1, gap, ties, sgap)
    epsL, epsR = res[0][1], res[1][1]
    lam_max = max(res[0][2], res[1][2])
    side = 1 if epsR < epsL - SIDE_TOL * lam_max else 0
    secs = secL if side == 0 else secR
    picks, _, _, gap, ties, sgap = res[side]
    picks = sorted(picks, key=lambda p: (secs[p[0]].label, p[1]))
    P = np.zeros((nfused, dcut))
    labels = np.zeros(dcut, dtype=np.int64)
    for j, (si, k) in enumerate(picks):
        s = secs[si]
        P[s.index, j] = s.vec[:, k]
        labels[j] = s.label
    return Selection(P, labels, epsL, epsR, side, lam_max, gap, ties, sgap)


def project(P: np.ndarray, A: np.ndarray, B: np.ndarray) -> np.ndarray:
    """T'[a,b,u,d] = sum P[(l1 l2),a] P[(r1 r2),b] A[l1,r1,u,i] B[l2,r2,i,d].

    The renormalised tensor of eq. renormalizedT with M built from A on top
    and B below (eq. Mtensor). Looped over the output index a so that only
    O(D^4) data is live: X_a = P_a . A, Y_a = X_a . B, T'_a = Y_a . P.
    """
    Dh, _, Dv, _ = A.shape
    Dn = P.shape[1]
    P3 = P.reshape(Dh, Dh, Dn)
    B2 = B.transpose(0, 2, 1, 3).reshape(Dh * Dv, Dh * Dv)   # [(l2,i),(r2,d)]
    out = np.empty((Dn, Dn, Dv, Dv))
    for a in range(Dn):
        Xa = np.tensordot(P3[:, :, a], A, axes=([0], [0]))   # [l2, r1, u, i]
        Xa = Xa.transpose(1, 2, 0, 3).reshape(Dh * Dv, Dh * Dv)  # [(r1,u),(l2,i)]
        Ya = (Xa @ B2).reshape(Dh, Dv, Dh, Dv)               # [r1, u, r2, d]
        Ta = np.tensordot(Ya, P3, axes=([0, 2], [0, 1]))     # [u, d, b]
        out[a] = Ta.transpose(2, 0, 1)
    return out


def second_moment_update(P: np.ndarray, x2: np.ndarray, T: np.ndarray,
                         x1: np.ndarray) -> np.ndarray:
    """Two insertions averaged over the ordered pairs of sites of the merged
    block: pairs inside the upper or the lower half, and the pairs split
    between the halves (both orders): (X2 (x) T + T (x) X2 + 2 X1 (x) X1) / 4,
    with X1 the one-insertion tensor of the step's input."""
    return 0.25 * (project(P, x2, T) + project(P, T, x2) + 2.0 * project(P, x1, x1))


# --------------------------------------------------------------------------
# Full run
# --------------------------------------------------------------------------

@dataclass
class StepLog:
    lnc: float
    eps_l: float
    eps_r: float
    side: int
    dh: int
    dv: int
    lam_max: float
    cut_gap: float
    ties: int
    truncated: bool
    sector_gap: float = math.inf


@dataclass
class RunResult:
    lnz_per_site: float
    m_cos1: float
    m_cos2: float
    steps: List[StepLog] = field(default_factory=list)
    lnc0: float = 0.0
    trace: float = 0.0
    msq_cos1: float = float("nan")   # <m^2>, m = (1/V) sum_i cos theta_i
    msq_cos2: float = float("nan")   # the same for cos q theta
    chi0: float = float("nan")       # beta V (<m^2> - <m>^2), cos theta
    chi0_n: float = float("nan")     # the same for cos q theta
    # (keep_tensor) the final normalised tensor and its leg labels
    tensor: Optional[np.ndarray] = None
    labels_hv: Optional[Tuple[np.ndarray, np.ndarray]] = None


def _norm(T: np.ndarray, kind: str) -> float:
    if kind == "fro":
        return float(np.sqrt(np.sum(T * T)))
    if kind == "maxabs":
        return float(np.max(np.abs(T)))
    raise ValueError(kind)


def hotrg_run(T: np.ndarray, imps: Dict[int, np.ndarray], lab_h: np.ndarray,
              lab_v: np.ndarray, sym: int, dcut: int, nsteps: int,
              first: str = "y", norm: str = "fro",
              basis_seed: Optional[int] = None, q: int = 2,
              keep_tensor: bool = False) -> RunResult:
    """Coarse-grain T (and impurity tensors) nsteps times; ln Z per site.

    ln Z / 2^N = ln c_0 + sum_n ln c_n / 2^n + ln Tr T_N / 2^N, where c_n is
    the norm divided out after step n and Tr T = sum_{l,u} T[l,l,u,u] closes
    the periodic 1x1 torus (Ch. 2 tensor-trace definition of Z).
    Impurity expectation value = Tr T_X / Tr T (M = P/Z of Ch. 3).
    Pinned by: tiny tori against brute-force traces and theta quadrature,
    decoupled-ring closed form, beta = 0, high-temperature series,
    normalisation and rotation invariance, the Delta = 0 / Delta = 1 map.
    """
    T = np.array(T, dtype=np.float64)
    imps = {k: np.array(v, dtype=np.float64) for k, v in imps.items()}
    brng = None if basis_seed is None else np.random.default_rng(basis_seed)
    lab_h = np.asarray(lab_h)
    lab_v = np.asarray(lab_v)
    c0 = _norm(T, norm)
    T /= c0
    for k in imps:
        imps[k] /= c0
    acc = math.log(c0)
    logs = []
    for n in range(1, nsteps + 1):
        is_y = ((n % 2 == 1) == (first == "y"))
        if not is_y:
            T = np.ascontiguousarray(T.transpose(2, 3, 0, 1))
            imps = {k: np.ascontiguousarray(v.transpose(2, 3, 0, 1)) for k, v in imps.items()}
            lab_h, lab_v = lab_v, lab_h
        Dh, Dv = T.shape[0], T.shape[2]
        fused = fuse_labels(lab_h, lab_h, sym, q)
        if Dh * Dh <= dcut:
            P = np.eye(Dh * Dh)
            new_h = fused
            sel = Selection(P, fused, 0.0, 0.0, 0, 0.0, 0.0, 0)
            truncated = False
        else:
            EL, ER = environments(T)
            sel = select_states(sector_eigh(EL, fused, brng), sector_eigh(ER, fused, brng),
                                dcut, Dh * Dh)
            P = sel.P
            new_h = sel.labels
            truncated = True
        Tn = project(P, T, T)
        # one insertion averaged over the sites of the doubled block:
        # (X (x) T + T (x) X) / 2; two insertions averaged over ordered pairs
        # of sites: (X2 (x) T + T (x) X2 + 2 X (x) X) / 4, with the step's
        # input X (the pairs split between the two halves count twice)
        new_imps = {}
        for k, v in imps.items():
            if k in SECOND_OF:
                new_imps[k] = second_moment_update(P, v, T, imps[SECOND_OF[k]])
            else:
                new_imps[k] = 0.5 * (project(P, v, T) + project(P, T, v))
        c = _norm(Tn, norm)
        Tn /= c
        for k in new_imps:
            new_imps[k] /= c
        acc += math.log(c) / 2.0 ** n
        T, imps, lab_h = Tn, new_imps, new_h
        if not is_y:
            T = np.ascontiguousarray(T.transpose(2, 3, 0, 1))
            imps = {k: np.ascontiguousarray(v.transpose(2, 3, 0, 1)) for k, v in imps.items()}
            lab_h, lab_v = lab_v, lab_h
        logs.append(StepLog(math.log(c), sel.eps_l, sel.eps_r, sel.side,
                            T.shape[0], T.shape[2], sel.lam_max, sel.cut_gap,
                            sel.ties, truncated, sel.sector_gap))
    Dh, Dv = T.shape[0], T.shape[2]
    tr = float(np.einsum("llUU->", T)) if Dh and Dv else 0.0
    if not (tr > 0.0) or not math.isfinite(tr):
        raise FloatingPointError("non-positive or non-finite final trace")
    lnz = acc + math.log(tr) / 2.0 ** nsteps
    m = {k: float(np.einsum("llUU->", v)) / tr for k, v in imps.items()}
    nan = float("nan")
    out = RunResult(lnz, m.get(IMP_COS1, nan), m.get(IMP_COS2, nan),
                    logs, math.log(c0), tr, m.get(IMP_COS1_SQ, nan), m.get(IMP_COS2_SQ, nan))
    if keep_tensor:
        out.tensor, out.labels_hv = T, (lab_h, lab_v)
    return out


def run_point(beta: float, delta: float, h: float = 0.0, h1: float = 0.0,
              nmax: int = 3, dcut: int = 12, nsteps: int = 30,
              nquad: int = 4096, impurities: int = IMP_COS1 | IMP_COS2,
              first: str = "y", norm: str = "fro", basis_seed: Optional[int] = None,
              q: int = 2, keep_tensor: bool = False, **_ignored) -> RunResult:
    """One HOTRG run from the gXY parameters (the full problem statement)."""
    q = 2 if q == 0 else int(q)
    sym = symmetry_of(h, h1)
    # a second moment carries its first moment along
    if impurities & IMP_COS1_SQ:
        impurities |= IMP_COS1
    if impurities & IMP_COS2_SQ:
        impurities |= IMP_COS2
    T, imps = initial_tensors(beta, delta, h, h1, nmax, nquad, impurities, q)
    lab = leg_labels(nmax, sym, q)
    r = hotrg_run(T, imps, lab, lab, sym, dcut, nsteps, first=first, norm=norm,
                  basis_seed=basis_seed, q=q, keep_tensor=keep_tensor)
    # susceptibility from the fluctuation of the site average (Ch. 3, eq. susc
    # as beta V (<m^2> - <m>^2) at the field of the run), V = 2^nsteps
    V = 2.0 ** nsteps
    if impurities & IMP_COS1_SQ:
        r.chi0 = beta * V * (r.msq_cos1 - r.m_cos1 ** 2)
    if impurities & IMP_COS2_SQ:
        r.chi0_n = beta * V * (r.msq_cos2 - r.m_cos2 ** 2)
    return r


def observables_from_runs(beta: float, lnz: Sequence[float], m_h: Sequence[float],
                          m_h1: Sequence[float], dbeta: float, dh: float,
                          dh1: float) -> Dict[str, float]:
    """f, C_v, chi, chi_n from the seven runs of one (beta, Delta) point.

    lnz = ln Z/V at beta - db, beta, beta + db; m_h = <cos theta> at
    h = hc -/+ dh; m_h1 = <cos q theta> at h1 = hc -/+ dh1.
    f = -lnZ/(beta V) (F = -T ln Z), C_v = beta^2 d^2(lnZ/V)/d beta^2 by the
    central difference (eq. spech), chi = d<cos theta>/dh and
    chi_n = d<cos q theta>/dh1 by central differences (eqs. susc, mag).
    """
    f = -lnz[1] / beta
    cv = beta * beta * (lnz[2] - 2.0 * lnz[1] + lnz[0]) / (dbeta * dbeta)
    chi = (m_h[1] - m_h[0]) / (2.0 * dh)
    chin = (m_h1[1] - m_h1[0]) / (2.0 * dh1)
    return {"f": f, "cv": cv, "chi": chi, "chi_n": chin}
