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


def test_gemm_large_tile_path(ctx):
    """Shapes with >= 512 output tiles of 128 x 128 take the 8-wave 128-tile kernel."""
    rng = np.random.default_rng(5)
    A = rng.standard_normal((3000, 40))
    B = rng.standard_normal((40, 3001))
    for at, bt in [(0, 0), (1, 1)]:
        C = ctx.test_gemm(A, B, at, bt)
        ref = A @ B
        assert np.max(np.abs(C - ref)) <= 1e-13 * math.sqrt(40) * np.max(np.abs(ref) + 1)


@pytest.mark.parametrize("kind", [0, 1])
def test_mfma_fp32_accumulating_register_layout(ctx, kind):
    """FP32-output 16x16 instructions: acc r of lane l = D[4(l/16) + r][l%16].

    kind 0 (FP32, 16x16x4): A[i][k] = a[i + 16k], B[k][j] = b[j + 16k].
    kind 1 (BF16, 16x16x32): lane l holds row l%16 of A and column l%16 of B
    with k = 8(l/16) + j for its eight values j (integers, exact in BF16).
    """
    rng = np.random.default_rng(4 + kind)
    n = 64 if kind == 0 else 512
    a = rng.integers(-4, 5, n).astype(np.float32)
    b = rng.integers(-4, 5, n).astype(np.float32)
    out = ctx.test_mfma_layout32(kind, a, b)
    kdim = 4 if kind == 0 else 32
    A = np.zeros((16, kdim))
    B = np.zeros((kdim, 16))
    for l in range(64):
        if kind == 0:
            A[l % 16, l // 16] = a[l]
            B[l // 16, l % 16] = b[l]
        else:
            for j in range(8):
                A[l % 16, 8 * (l // 16) + j] = a[8 * l + j]
                B[8 * (l // 16) + j, l % 16] = b[8 * l + j]
    D = A @ B
    for l in range(64):
        for r in range(4):
            assert out[l, r] == D[4 * (l // 16) + r, l % 16]


def _bf16_rne(x32):
    """Round float32 values to bfloat16 (round to nearest even), as float32."""
    u = x32.astype(np.float32).view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000).astype(np.uint32)
    return r.view(np.float32)


GEMM_PREC_SHAPES = [(37, 29, 13), (130, 70, 45), (257, 300, 129), (3000, 300, 40)]


@pytest.mark.parametrize("M,N,K", GEMM_PREC_SHAPES)
@pytest.mark.parametrize("at,bt", [(0, 0), (1, 1), (0, 1)])
def test_gemm_fp32_form(ctx, M, N, K, at, bt):
    """FP32 form = exact product of the FP32-rounded operands, up to FP32
    accumulation (|err| <= 2 K u32 (|A32||B32|)), and measurably not FP64."""
    rng = np.random.default_rng(M + 5 * N + 11 * K + at)
    A = rng.standard_normal((M, K))
    B = rng.standard_normal((K, N))
    C = ctx.test_gemm(A, B, at, bt, prec=1)
    A32 = A.astype(np.float32).astype(np.float64)
    B32 = B.astype(np.float32).astype(np.float64)
    ref = A32 @ B32
    bound = 2.0 * K * 2.0 ** -24 * (np.abs(A32) @ np.abs(B32)) + 1e-300
    assert np.all(np.abs(C - ref) <= bound)
    assert np.max(np.abs(C - A @ B)) > 1e-12


@pytest.mark.parametrize("M,N,K", GEMM_PREC_SHAPES)
@pytest.mark.parametrize("at,bt", [(0, 0), (1, 1), (1, 0)])
def test_gemm_bf16x3_form(ctx, M, N, K, at, bt):
    """BF16X3 form = hi*hi + hi*lo + lo*hi of the bfloat16 split of the
    FP32-rounded operands (products exact in FP32), up to FP32 accumulation;
    against the FP64 product it is within the split's 2^-16 relative bound."""
    rng = np.random.default_rng(3 * M + N + 7 * K + bt)
    A = rng.standard_normal((M, K))
    B = rng.standard_normal((K, N))
    C = ctx.test_gemm(A, B, at, bt, prec=2)
    def split(X):
        f = X.astype(np.float32)
        hi = _bf16_rne(f)
        lo = _bf16_rne(f - hi)
        return hi.astype(np.float64), lo.astype(np.float64)
    ah, al = split(A)
    bh, bl = split(B)
    ref = ah @ bh + ah @ bl + al @ bh
    absAB = np.abs(A) @ np.abs(B)
    assert np.all(np.abs(C - ref) <= 4.0 * K * 2.0 ** -24 * absAB + 1e-300)
    assert np.all(np.abs(C - A @ B) <= (2.0 ** -15 + 4.0 * K * 2.0 ** -24) * absAB + 1e-300)
    assert np.max(np.abs(C - A @ B)) > 1e-12


def _check_eig(A, w, V, tol=None):
    n = A.shape[0]
    if tol is None:
        tol = 5e-15 * max(n, 32)
    scale = max(np.max(np.abs(np.linalg.eigvalsh(A))), 1e-300)
    wr = np.sort(np.linalg.eigvalsh(A))
    assert np.max(np.abs(np.sort(w) - wr)) <= tol * scale
    assert np.max(np.abs(A @ V - V * w)) <= 10 * tol * scale
    assert np.max(np.abs(V.T @ V - np.eye(n))) <= 10 * tol * max(1, n / 100)


EIG_METHODS = [1, 2]   # block Jacobi, Householder + bisection + inverse iteration


@pytest.mark.parametrize("method", EIG_METHODS)
@pytest.mark.parametrize("n", [1, 2, 3, 5, 16, 31, 32, 33, 40, 64, 65, 100, 127, 128, 257])
def test_eigh_psd(ctx, n, method):
    rng = np.random.default_rng(n)
    X = rng.standard_normal((n, n + 3))
    A = X @ X.T
    w, V = ctx.test_eigh(A, method)
    _check_eig(A, w, V)


def test_eigh_above_tridiagonal_limit_uses_jacobi(ctx):
    rng = np.random.default_rng(513)
    X = rng.standard_normal((129, 140))
    A = X @ X.T
    w, V = ctx.test_eigh(A, 2)
    _check_eig(A, w, V)
    assert ctx.last_sweeps > 0


def test_eigh_above_2048_rows_uses_jacobi(ctx):
    rng = np.random.default_rng(2049)
    X = rng.standard_normal((2049, 2060))
    A = X @ X.T
    w, V = ctx.test_eigh(A, 2, kmax=32)
    assert ctx.last_sweeps > 0
    wr = np.sort(np.linalg.eigvalsh(A))[::-1]
    assert np.max(np.abs(np.sort(w)[::-1] - wr)) <= 5e-15 * 2049 * wr[0]


@pytest.mark.parametrize("method", EIG_METHODS)
def test_eigh_graded_spectrum(ctx, method):
    """Spectrum over 14 decades, like the HOTRG environments: eigenvalues to
    eps * lambda_max, residuals and orthogonality to the same class."""
    rng = np.random.default_rng(17)
    n = 120
    Q = np.linalg.qr(rng.standard_normal((n, n)))[0]
    lam = np.exp(-np.linspace(0.0, 32.0, n))
    A = (Q * lam) @ Q.T
    A = 0.5 * (A + A.T)
    w, V = ctx.test_eigh(A, method)
    _check_eig(A, w, V)


@pytest.mark.parametrize("method", EIG_METHODS)
def test_eigh_rank_deficient_and_degenerate(ctx, method):
    rng = np.random.default_rng(7)
    Q = np.linalg.qr(rng.standard_normal((70, 70)))[0]
    lam = np.concatenate([np.full(10, 3.0), np.full(20, 1e-3), np.zeros(40)])
    A = (Q * lam) @ Q.T
    A = 0.5 * (A + A.T)
    w, V = ctx.test_eigh(A, method)
    _check_eig(A, w, V)
    assert np.sum(np.abs(w - 3.0) < 1e-12) == 10


@pytest.mark.parametrize("method", EIG_METHODS)
def test_eigh_diagonal_and_block(ctx, method):
    A = np.diag(np.arange(40, dtype=float)[::-1])
    w, V = ctx.test_eigh(A, method)
    if method == 1:   # rotations never start: exact
        assert np.array_equal(np.sort(w), np.arange(40, dtype=float))
    else:             # bisection: to eps ||A||
        assert np.max(np.abs(np.sort(w) - np.arange(40.0))) <= 4e-16 * 39
    B = np.zeros((45, 45))
    B[:20, :20] = 2.0 * np.eye(20) + 0.5
    B[20:, 20:] = np.diag(np.linspace(0.1, 1.0, 25))
    w, V = ctx.test_eigh(B, method)
    _check_eig(B, w, V)


@pytest.mark.parametrize("n,kmax", [(300, 64), (513, 48), (777, 128), (1024, 64), (1025, 96),
                                    (1500, 96), (2048, 128)])
def test_tridiagonal_leading_vectors_of_large_sectors(ctx, n, kmax):
    """Sector sizes of Dcut = 64 and 96 runs (above 1024 rows the kernels'
    2048-row instantiation): all eigenvalues, the kmax leading eigenvectors
    (residual and orthogonality at eps ||A||), graded spectrum."""
    rng = np.random.default_rng(n)
    Q = np.linalg.qr(rng.standard_normal((n, n)))[0]
    lam = np.exp(-np.linspace(0.0, 30.0, n))
    lam[n // 3: n // 3 + 2] = lam[n // 3]                      # a degenerate pair
    A = (Q * lam) @ Q.T
    A = 0.5 * (A + A.T)
    w, V = ctx.test_eigh(A, 2, kmax=kmax)
    assert ctx.last_sweeps == 0                                # tridiagonal path taken
    wr = np.sort(np.linalg.eigvalsh(A))[::-1]
    scale = wr[0]
    assert np.max(np.abs(w - wr)) <= 5e-15 * n * scale
    Vk = V[:, :kmax]
    assert np.max(np.abs(A @ Vk - Vk * w[:kmax])) <= 5e-14 * n ** 0.5 * scale
    assert np.max(np.abs(Vk.T @ Vk - np.eye(kmax))) <= 1e-12
    assert not np.any(V[:, kmax:])


@pytest.mark.parametrize("n", [800, 1024, 1600])
@pytest.mark.parametrize("other", ["GXY_TRI_MULTI", "GXY_TRI_COOP"])
def test_tridiagonal_shared_reduction_same_bits(ctx, n, other, monkeypatch):
    """Sectors of at least 384 rows are reduced by several workgroups of one
    cooperative launch (a barrier of the matrix's workgroups per column); the
    matrix-vector sums are
    grouped the same way as when one workgroup runs the groups in turn, so
    both give the same eigenvalues and vectors bit for bit; so does the same
    grid launched as a regular (not cooperative) one."""
    rng = np.random.default_rng(n + 1)
    X = rng.standard_normal((n, n + 7))
    A = X @ X.T
    w1, V1 = ctx.test_eigh(A, 2, kmax=64)
    monkeypatch.setenv(other, "0")
    w0, V0 = ctx.test_eigh(A, 2, kmax=64)
    assert np.array_equal(w0, w1)
    assert np.array_equal(V0, V1)


def test_tridiagonal_eigenvalues_sorted_decreasing(ctx):
    rng = np.random.default_rng(3)
    X = rng.standard_normal((90, 95))
    w, V = ctx.test_eigh(X @ X.T, 2)
    assert np.all(np.diff(w) <= 0.0)


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


@pytest.mark.parametrize("q", [3, 5])
@pytest.mark.parametrize("h,h1", [(0.0, 0.0), (0.0, 0.3), (0.3, 0.2)])
@pytest.mark.parametrize("which", [0, 1, 2])
def test_initial_tensors_harmonic_q_match_oracle(ctx, q, h, h1, which):
    nmax = 4
    Tg = ctx.initial_tensor(dict(beta=1.1, delta=0.6, h=h, h1=h1, nmax=nmax, dcut=8,
                                 nsteps=0, q=q), which)
    T, imps = o.initial_tensors(1.1, 0.6, h, h1, nmax, impurities=3, q=q)
    ref = T if which == 0 else imps[which]
    assert np.max(np.abs(Tg - ref)) <= 1e-15 * max(1.0, np.max(np.abs(ref)))
    if h == 0.0 and h1 == 0.0:
        assert np.array_equal(Tg == 0.0, ref == 0.0)
