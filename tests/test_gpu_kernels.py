"""Single-kernel GPU checks through the C ABI (MFMA layout, GEMM, eigensolver,
coefficients, initial tensors) against numpy / LAPACK / the oracle."""

import math

import numpy as np
import pytest

import oracle.hotrg as o

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2609_20536_amd import hotrg as H
    c = H.Context(0)
    yield c
    c.close()


def test_mfma_f64_register_layout(ctx):
    """A[i][k] = a[i + 16k], B[k][j] = b[j + 16k]; acc r of lane l = D[l/16 + 4r][l%16]."""
    rng = np.random.default_rng(3)
    a = rng.integers(-4, 5, 64).astype(float)
    b = rng.integers(-4, 5, 64).astype(float)
    out = ctx.test_mfma_layout(a, b)
    A = np.zeros((16, 4))
    B = np.zeros((4, 16))
    for l in range(64):
        A[l % 16, l // 16] = a[l]
        B[l // 16, l % 16] = b[l]
    D = A @ B
    for l in range(64):
        for r in range(4):
            assert out[l, r] == D[l // 16 + 4 * r, l % 16]


@pytest.mark.parametrize("M,N,K", [(1, 1, 1), (16, 16, 4), (37, 29, 13), (64, 64, 16),
                                   (130, 70, 45), (257, 300, 129), (1100, 1030, 77),
                                   (8, 2000, 3)])
@pytest.mark.parametrize("at,bt", [(0, 0), (0, 1), (1, 0), (1, 1)])
def test_gemm_matches_numpy(ctx, M, N, K, at, bt):
    rng = np.random.default_rng(M * 7 + N * 3 + K)
    A = rng.standard_normal((M, K))
    B = rng.standard_normal((K, N))
    C = ctx.test_gemm(A, B, at, bt)
    ref = A @ B
    assert np.max(np.abs(C - ref)) <= 1e-13 * max(1.0, math.sqrt(K)) * np.max(np.abs(ref) + 1)


def test_gemm_exact_on_integers(ctx):
    rng = np.random.default_rng(11)
    A = rng.integers(-8, 9, (200, 96)).astype(float)
    B = rng.integers(-8, 9, (96, 150)).astype(float)
    assert np.array_equal(ctx.test_gemm(A, B), A @ B)


def _check_eig(A, w, V, tol=None):
    n = A.shape[0]
    if tol is None:
        tol = 5e-15 * max(n, 32)
    scale = max(np.max(np.abs(np.linalg.eigvalsh(A))), 1e-300)
    wr = np.sort(np.linalg.eigvalsh(A))
    assert np.max(np.abs(np.sort(w) - wr)) <= tol * scale
    assert np.max(np.abs(A @ V - V * w)) <= 10 * tol * scale
    assert np.max(np.abs(V.T @ V - np.eye(n))) <= 10 * tol * max(1, n / 100)


@pytest.mark.parametrize("n", [1, 2, 5, 16, 31, 32, 33, 64, 100, 257])
def test_eigh_psd(ctx, n):
    rng = np.random.default_rng(n)
    X = rng.standard_normal((n, n + 3))
    A = X @ X.T
    w, V = ctx.test_eigh(A)
    _check_eig(A, w, V)


def test_eigh_rank_deficient_and_degenerate(ctx):
    rng = np.random.default_rng(7)
    Q = np.linalg.qr(rng.standard_normal((70, 70)))[0]
    lam = np.concatenate([np.full(10, 3.0), np.full(20, 1e-3), np.zeros(40)])
    A = (Q * lam) @ Q.T
    A = 0.5 * (A + A.T)
    w, V = ctx.test_eigh(A)
    _check_eig(A, w, V)
    assert np.sum(np.abs(w - 3.0) < 1e-12) == 10


def test_eigh_diagonal_and_block(ctx):
    A = np.diag(np.arange(40, dtype=float)[::-1])
    w, V = ctx.test_eigh(A)
    assert np.array_equal(np.sort(w), np.arange(40, dtype=float))


@pytest.mark.parametrize("beta,delta,nmax", [(0.0, 0.5, 3), (0.5, 0.0, 10), (1.0, 0.5, 10),
                                             (1.5, 1.0, 20), (1.2, 0.7, 45)])
def test_char_coeffs_match_oracle(ctx, beta, delta, nmax):
    t = ctx.char_coeffs(beta, delta, nmax)
    assert np.max(np.abs(t - o.char_coeffs(beta, delta, nmax))) <= 1e-15 * math.exp(beta)


@pytest.mark.parametrize("h,h1", [(0.0, 0.0), (0.0, 0.3), (0.4, 0.0), (0.3, 0.2)])
@pytest.mark.parametrize("which", [0, 1, 2])
def test_initial_tensors_match_oracle(ctx, h, h1, which):
    nmax = 4
    Tg = ctx.initial_tensor(dict(beta=1.1, delta=0.6, h=h, h1=h1, nmax=nmax, dcut=8,
                                 nsteps=0), which)
    T, imps = o.initial_tensors(1.1, 0.6, h, h1, nmax, impurities=3)
    ref = T if which == 0 else imps[which]
    assert np.max(np.abs(Tg - ref)) <= 1e-15 * max(1.0, np.max(np.abs(ref)))
    if h == 0.0 and h1 == 0.0:
        assert np.array_equal(Tg == 0.0, ref == 0.0)   # exact charge structure
