"""ctypes binding of libgxyhotrg.so (include/gxy_hotrg.h).

Argument marshalling only: every step of a run executes in the library's
HIP kernels. torch supplies the device workspace and the HIP stream. There
is no CPU fallback: if the library is missing, loading raises.
"""

from __future__ import annotations

import ctypes as C
import math
import os
from dataclasses import dataclass
from typing import List, Optional, Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgxyhotrg.so")

GXY_OK = 0
STATUS = {0: "ok", 1: "EINVAL", 2: "ENOMEM", 3: "EDEVICE", 4: "ENUMERIC",
          5: "EUNSUPPORTED", 6: "EPARTIAL"}


class GxyError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Point(C.Structure):
    _fields_ = [("beta", C.c_double), ("delta", C.c_double), ("h", C.c_double),
                ("h1", C.c_double), ("nmax", C.c_int32), ("dcut", C.c_int32),
                ("nsteps", C.c_int32), ("nquad", C.c_int32),
                ("impurities", C.c_uint32), ("prec", C.c_int32),
                ("fp64_steps", C.c_int32), ("q", C.c_int32)]


class Result(C.Structure):
    _fields_ = [("lnz_per_site", C.c_double), ("m_cos1", C.c_double),
                ("m_cos2", C.c_double), ("max_trunc_err", C.c_double),
                ("min_cut_gap", C.c_double), ("near_ties", C.c_int32),
                ("status", C.c_int32), ("fail_step", C.c_int32),
                ("nsteps_done", C.c_int32), ("msq_cos1", C.c_double),
                ("msq_cos2", C.c_double), ("chi0", C.c_double), ("chi0_n", C.c_double)]


class LgtResult(C.Structure):
    """gxy_lgt_result (include/gxy_lgt.h)."""
    _fields_ = [("sum_g2", C.c_double), ("sum_h", C.c_double), ("g_h_g", C.c_double),
                ("plaquette", C.c_double), ("beta_diag", C.c_double),
                ("beta_full", C.c_double), ("sum_g2_dir", C.c_double * 4),
                ("sum_h_dir", C.c_double * 4)]

    def as_dict(self, ndim: int = 4) -> dict:
        out = {f: getattr(self, f) for f, _ in self._fields_[:6]}
        out["sum_g2_dir"] = list(self.sum_g2_dir)[:ndim]
        out["sum_h_dir"] = list(self.sum_h_dir)[:ndim]
        return out


LGT_FULL = 1


class StepInfo(C.Structure):
    _fields_ = [("lnc", C.c_double), ("eps_l", C.c_double), ("eps_r", C.c_double),
                ("lam_max", C.c_double), ("cut_gap", C.c_double), ("side", C.c_int32),
                ("dh", C.c_int32), ("dv", C.c_int32), ("truncated", C.c_int32),
                ("ties", C.c_int32), ("eig_sweeps", C.c_int32)]


_lib = None


class TrainCfg(C.Structure):
    _fields_ = [("epochs", C.c_int32), ("lr", C.c_float), ("beta1", C.c_float),
                ("beta2", C.c_float), ("eps", C.c_float), ("log_targets", C.c_uint32),
                ("standardize", C.c_int32)]


class ProposeCfg(C.Structure):
    _fields_ = [("nbeta", C.c_int32), ("ndelta", C.c_int32), ("beta_lo", C.c_double),
                ("beta_hi", C.c_double), ("delta_lo", C.c_double), ("delta_hi", C.c_double),
                ("seed", C.c_uint64), ("jitter", C.c_double), ("cv_col", C.c_int32),
                ("chi_col", C.c_int32)]


def load_library(path: str = LIB_PATH):
    """Load the HIP library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with __graft_entry__.build()")
    lib = C.CDLL(path)
    P = C.POINTER
    sigs = {
        "gxy_create": [P(C.c_void_p), C.c_int, C.c_void_p],
        "gxy_destroy": [C.c_void_p],
        "gxy_workspace_bytes": [C.c_void_p, P(Point), C.c_int32, P(C.c_size_t)],
        "gxy_set_workspace": [C.c_void_p, C.c_void_p, C.c_size_t],
        "gxy_char_coeffs": [C.c_void_p, C.c_double, C.c_double, C.c_int32, C.c_int32,
                            P(C.c_double)],
        "gxy_initial_tensor": [C.c_void_p, P(Point), C.c_int32, P(C.c_double)],
        "gxy_run": [C.c_void_p, P(Point), P(Result)],
        "gxy_run_batch": [C.c_void_p, P(Point), C.c_int32, P(Result)],
        "gxy_run_noalloc": [C.c_void_p, P(Point), P(Result)],
        "gxy_set_batch_workers": [C.c_void_p, C.c_int32],
        "gxy_autotune": [C.c_void_p, P(Point), P(C.c_int32), C.c_int32, P(C.c_int32),
                         P(C.c_double)],
        "gxy_step_log": [C.c_void_p, C.c_int32, P(StepInfo), C.c_int32, P(C.c_int32)],
        "gxy_observables": [C.c_void_p, C.c_int32, P(C.c_double), P(C.c_double),
                            P(C.c_double), P(C.c_double), C.c_double, C.c_double,
                            C.c_double, P(C.c_double)],
        "gxy_phase_times": [C.c_void_p, P(C.c_double)],
        "gxy_lgt_workspace_bytes": [C.c_int32, P(C.c_int32), C.c_int64, C.c_uint32,
                                    P(C.c_size_t)],
        "gxy_lgt_estimator": [C.c_void_p, C.c_void_p, C.c_int32, P(C.c_int32), C.c_int64,
                              C.c_uint32, P(LgtResult)],
        "gxy_mlp_create": [C.c_void_p, C.c_uint64, P(C.c_void_p)],
        "gxy_mlp_destroy": [C.c_void_p],
        "gxy_mlp_params": [C.c_void_p, P(C.c_float), P(C.c_float)],
        "gxy_mlp_train": [C.c_void_p, P(C.c_double), P(C.c_double), C.c_int32, P(TrainCfg),
                          P(C.c_float)],
        "gxy_mlp_grad": [C.c_void_p, P(C.c_float), P(C.c_float), C.c_int32, P(C.c_float),
                         P(C.c_float)],
        "gxy_mlp_predict": [C.c_void_p, P(C.c_double), C.c_int32, C.c_int32, P(C.c_double)],
        "gxy_mlp_scaling": [C.c_void_p, P(C.c_double), P(C.c_uint32)],
        "gxy_mlp_propose": [C.c_void_p, P(ProposeCfg), P(C.c_double)],
        "gxy_hot_kernel_stats": [C.c_void_p, P(C.c_double), C.c_int32],
        "gxy_test_gemm_f64": [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, P(C.c_double),
                              C.c_int32, P(C.c_double), C.c_int32, P(C.c_double)],
        "gxy_test_gemm": [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                          P(C.c_double), C.c_int32, P(C.c_double), C.c_int32, P(C.c_double)],
        "gxy_test_eigh_method": [C.c_void_p, C.c_int32, C.c_int32, P(C.c_double),
                                 P(C.c_double), P(C.c_double), P(C.c_int32)],
        "gxy_test_eigh_top": [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, P(C.c_double),
                              P(C.c_double), P(C.c_double), P(C.c_int32)],
        "gxy_test_eigh": [C.c_void_p, C.c_int32, P(C.c_double), P(C.c_double),
                          P(C.c_double), P(C.c_int32)],
        "gxy_test_mfma_layout": [C.c_void_p, P(C.c_double), P(C.c_double), P(C.c_double)],
        "gxy_test_mfma_layout32": [C.c_void_p, C.c_int32, P(C.c_float), P(C.c_float),
                                   P(C.c_float)],
    }
    for name, args in sigs.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = C.c_int
    lib.gxy_status_string.argtypes = [C.c_int]
    lib.gxy_status_string.restype = C.c_char_p
    lib.gxy_last_error.argtypes = [C.c_void_p]
    lib.gxy_last_error.restype = C.c_char_p
    _lib = lib
    return lib


def make_point(beta, delta, h=0.0, h1=0.0, nmax=3, dcut=12, nsteps=30, nquad=4096,
               impurities=3, prec=0, fp64_steps=0, q=2, **_ignored) -> Point:
    return Point(float(beta), float(delta), float(h), float(h1), int(nmax), int(dcut),
                 int(nsteps), int(nquad), int(impurities), int(prec), int(fp64_steps),
                 int(q))


def point_from(obj) -> Point:
    if isinstance(obj, Point):
        return obj
    if isinstance(obj, dict):
        return make_point(**obj)
    return make_point(**obj.as_dict())


@dataclass
class RunResult:
    lnz_per_site: float
    m_cos1: float
    m_cos2: float
    max_trunc_err: float
    min_cut_gap: float
    near_ties: int
    status: int
    steps: list
    msq_cos1: float = float("nan")
    msq_cos2: float = float("nan")
    chi0: float = float("nan")
    chi0_n: float = float("nan")
    fail_step: int = -1


class Context:
    """A library context bound to a device and torch's current stream."""

    def __init__(self, device: int = 0, stream=None, torch_workspace: bool = True):
        import torch
        self.torch = torch
        self.lib = load_library()
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device visible")
        self.device = device
        torch.cuda.set_device(device)
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        h = C.c_void_p()
        self._check(self.lib.gxy_create(C.byref(h), device, C.c_void_p(stream.cuda_stream)),
                    None)
        self.handle = h
        self.torch_workspace = torch_workspace
        self._ws = None

    def _check(self, st, handle=None):
        if st != GXY_OK:
            msg = self.lib.gxy_last_error(handle if handle is not None else getattr(self, "handle", None))
            raise GxyError(st, (msg or b"").decode())

    def close(self):
        if getattr(self, "handle", None):
            self.lib.gxy_destroy(self.handle)
            self.handle = None
            self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- workspace -------------------------------------------------------
    def reserve(self, points: Sequence) -> int:
        """Allocate (through torch) the device workspace for these points."""
        arr = (Point * len(points))(*[point_from(p) for p in points])
        nb = C.c_size_t()
        self._check(self.lib.gxy_workspace_bytes(self.handle, arr, len(points), C.byref(nb)),
                    self.handle)
        self._reserve_bytes(nb.value)
        return nb.value

    def _reserve_bytes(self, nbytes: int):
        if not self.torch_workspace:
            return
        if self._ws is None or self._ws.numel() < nbytes:
            self.lib.gxy_set_workspace(self.handle, None, 0)
            self._ws = None
            self._ws = self.torch.empty(int(nbytes), dtype=self.torch.uint8,
                                        device=f"cuda:{self.device}")
            self._check(self.lib.gxy_set_workspace(self.handle, C.c_void_p(self._ws.data_ptr()),
                                                   int(nbytes)), self.handle)

    # -- calls ---------------------------------------------------------------
    def char_coeffs(self, beta, delta, nmax, nquad=4096):
        import numpy as np
        out = (C.c_double * (2 * nmax + 1))()
        self.reserve([make_point(beta, delta, nmax=nmax, dcut=1, nsteps=0, nquad=nquad,
                                 impurities=0)])
        self._check(self.lib.gxy_char_coeffs(self.handle, beta, delta, nmax, nquad, out),
                    self.handle)
        return np.array(out[:])

    def initial_tensor(self, point, which=0):
        import numpy as np
        p = point_from(point)
        D = 2 * p.nmax + 1
        out = np.empty(D ** 4, dtype=np.float64)
        self.reserve([p])
        self._check(self.lib.gxy_initial_tensor(self.handle, C.byref(p), which,
                                                out.ctypes.data_as(C.POINTER(C.c_double))),
                    self.handle)
        return out.reshape(D, D, D, D)

    def run(self, point) -> RunResult:
        p = point_from(point)
        self.reserve([p])
        r = Result()
        st = self.lib.gxy_run(self.handle, C.byref(p), C.byref(r))
        if st != GXY_OK and r.status == 0:
            self._check(st, self.handle)
        return self._result(r, 0)

    def run_noalloc(self, point) -> RunResult:
        """gxy_run_noalloc: the run in the library's fixed device scratch
        array (no device allocation, no workspace reservation here)."""
        p = point_from(point)
        r = Result()
        st = self.lib.gxy_run_noalloc(self.handle, C.byref(p), C.byref(r))
        if st != GXY_OK and r.status == 0:
            self._check(st, self.handle)
        return self._result(r, 0)

    def run_batch(self, points, workers: int = 1) -> List[RunResult]:
        """Runs of all points; workers > 1 runs them concurrently on worker
        contexts (own streams and library-allocated workspaces)."""
        pts = [point_from(p) for p in points]
        self._check(self.lib.gxy_set_batch_workers(self.handle, int(workers)), self.handle)
        if workers <= 1:
            self.reserve(pts)
        arr = (Point * len(pts))(*pts)
        res = (Result * len(pts))()
        st = self.lib.gxy_run_batch(self.handle, arr, len(pts), res)
        if st not in (GXY_OK, 6):
            self._check(st, self.handle)
        return [self._result(res[i], i) for i in range(len(pts))]

    def autotune(self, point, dcuts):
        """Pick the fastest projection tile per Dcut (see gxy_autotune);
        returns {dcut: (tile, ms64, ms128, ms256)}."""
        import numpy as np
        pt = point_from(point)
        d = np.ascontiguousarray(dcuts, dtype=np.int32)
        copies = []
        for x in d:
            q = Point()
            C.memmove(C.byref(q), C.byref(pt), C.sizeof(Point))
            q.dcut = int(x)
            copies.append(q)
        self.reserve(copies)
        tiles = np.empty(d.size, dtype=np.int32)
        ms = np.empty(3 * d.size)
        self._check(self.lib.gxy_autotune(self.handle, C.byref(pt),
                                          d.ctypes.data_as(C.POINTER(C.c_int32)), d.size,
                                          tiles.ctypes.data_as(C.POINTER(C.c_int32)),
                                          ms.ctypes.data_as(C.POINTER(C.c_double))),
                    self.handle)
        return {int(x): (int(t), float(ms[3 * i]), float(ms[3 * i + 1]), float(ms[3 * i + 2]))
                for i, (x, t) in enumerate(zip(d, tiles))}

    def step_log(self, run=0):
        cnt = C.c_int32()
        self._check(self.lib.gxy_step_log(self.handle, run, None, 0, C.byref(cnt)), self.handle)
        arr = (StepInfo * max(cnt.value, 1))()
        self._check(self.lib.gxy_step_log(self.handle, run, arr, cnt.value, C.byref(cnt)),
                    self.handle)
        return [dict((f, getattr(arr[i], f)) for f, _ in StepInfo._fields_)
                for i in range(cnt.value)]

    def _result(self, r: Result, run: int) -> RunResult:
        steps = self.step_log(run) if r.status == 0 else []
        return RunResult(r.lnz_per_site, r.m_cos1, r.m_cos2, r.max_trunc_err,
                         r.min_cut_gap, r.near_ties, r.status, steps, r.msq_cos1,
                         r.msq_cos2, r.chi0, r.chi0_n, r.fail_step)

    def observables(self, beta, lnz, m_h, m_h1, dbeta, dh, dh1):
        import numpy as np
        beta = np.ascontiguousarray(beta, dtype=np.float64)
        lnz = np.ascontiguousarray(lnz, dtype=np.float64)
        m_h = np.ascontiguousarray(m_h, dtype=np.float64)
        m_h1 = np.ascontiguousarray(m_h1, dtype=np.float64)
        n = len(beta)
        out = np.empty((n, 4))
        self._reserve_bytes(8 * 12 * n + 4096)
        dp = lambda a: a.ctypes.data_as(C.POINTER(C.c_double))  # noqa: E731
        self._check(self.lib.gxy_observables(self.handle, n, dp(beta), dp(lnz), dp(m_h),
                                             dp(m_h1), dbeta, dh, dh1, dp(out)), self.handle)
        return out

    def lgt_estimator(self, theta, full: bool = True):
        """Configurational-temperature estimator (include/gxy_lgt.h) of a batch
        of link configurations: theta is a float64 device tensor of shape
        (nconf, d, L_{d-1}, ..., L_0) (x_0 fastest), on this context's
        device; returns one gxy_lgt_result dict per configuration."""
        t = self.torch
        if not (isinstance(theta, t.Tensor) and theta.is_cuda and theta.dtype == t.float64):
            raise TypeError("theta must be a float64 device tensor")
        if not theta.is_contiguous():
            raise ValueError("theta must be contiguous")
        nconf, d = theta.shape[0], theta.shape[1]
        if theta.dim() != d + 2:
            raise ValueError("theta must have shape (nconf, d, L_{d-1}, ..., L_0)")
        dims = (C.c_int32 * d)(*[int(n) for n in reversed(theta.shape[2:])])
        flags = LGT_FULL if full else 0
        nb = C.c_size_t()
        self._check(self.lib.gxy_lgt_workspace_bytes(d, dims, nconf, flags, C.byref(nb)))
        self._reserve_bytes(nb.value)
        out = (LgtResult * max(nconf, 1))()
        self._check(self.lib.gxy_lgt_estimator(self.handle, C.c_void_p(theta.data_ptr()), d,
                                               dims, nconf, flags, out), self.handle)
        return [out[i].as_dict(d) for i in range(nconf)]

    # -- single-kernel checks (include/gxy_hotrg_testing.h) -------------------
    def test_gemm(self, A, B, a_trans=False, b_trans=False, prec=None):
        """C = A @ B through the matrix-core GEMM; A (M,K), B (K,N) as numpy.

        prec None calls the FP64 entry point; otherwise a gxy_precision value.
        """
        import numpy as np
        M, K = A.shape
        K2, N = B.shape
        assert K == K2
        Ah = np.ascontiguousarray(A.T if a_trans else A, dtype=np.float64)
        Bh = np.ascontiguousarray(B.T if b_trans else B, dtype=np.float64)
        out = np.empty((M, N))
        self._reserve_bytes(8 * (M * K + K * N + M * N) + 4096)
        dp = lambda a: a.ctypes.data_as(C.POINTER(C.c_double))  # noqa: E731
        if prec is None:
            rc = self.lib.gxy_test_gemm_f64(self.handle, M, N, K, dp(Ah), int(a_trans),
                                            dp(Bh), int(b_trans), dp(out))
        else:
            rc = self.lib.gxy_test_gemm(self.handle, int(prec), M, N, K, dp(Ah), int(a_trans),
                                        dp(Bh), int(b_trans), dp(out))
        self._check(rc, self.handle)
        return out

    def test_eigh(self, A, method=0, kmax=None):
        """Eigenpairs of one symmetric matrix by the batched sector solver
        (method 0: as a run chooses, 1: block Jacobi, 2: tridiagonal path);
        kmax: only the leading kmax eigenvectors are required."""
        import numpy as np
        A = np.ascontiguousarray(A, dtype=np.float64)
        n = A.shape[0]
        w = np.empty(n)
        V = np.empty((n, n))
        npad = (n + 31) // 32 * 32
        q = npad // 32
        self._reserve_bytes(8 * (2 * n * n + 8 * npad * npad + 2 * q * 1024 + 2048 + 8 * npad)
                            + 4 * (n + 16 * q * q + 256) + (1 << 20))
        dp = lambda a: a.ctypes.data_as(C.POINTER(C.c_double))  # noqa: E731
        sw = C.c_int32(0)
        k = n if kmax is None else int(kmax)
        self._check(self.lib.gxy_test_eigh_top(self.handle, int(method), n, k, dp(A), dp(w),
                                               dp(V), C.byref(sw)), self.handle)
        self.last_sweeps = sw.value
        return w, V

    def test_mfma_layout(self, a, b):
        import numpy as np
        a = np.ascontiguousarray(a, dtype=np.float64)
        b = np.ascontiguousarray(b, dtype=np.float64)
        out = np.empty(256)
        self._reserve_bytes(8 * 384 + 4096)
        dp = lambda x: x.ctypes.data_as(C.POINTER(C.c_double))  # noqa: E731
        self._check(self.lib.gxy_test_mfma_layout(self.handle, dp(a), dp(b), dp(out)),
                    self.handle)
        return out.reshape(64, 4)

    def hot_kernel_stats(self, reset=True):
        """(launches, total ms, algorithmic flops, algorithmic bytes) of the D^7 GEMM."""
        out = (C.c_double * 4)()
        self._check(self.lib.gxy_hot_kernel_stats(self.handle, out, int(reset)), self.handle)
        return list(out)

    def test_mfma_layout32(self, kind, a, b):
        import numpy as np
        a = np.ascontiguousarray(a, dtype=np.float32)
        b = np.ascontiguousarray(b, dtype=np.float32)
        out = np.empty(256, dtype=np.float32)
        self._reserve_bytes(4 * (2 * 512 + 256) + 4096)
        fp = lambda x: x.ctypes.data_as(C.POINTER(C.c_float))  # noqa: E731
        self._check(self.lib.gxy_test_mfma_layout32(self.handle, int(kind), fp(a), fp(b),
                                                    fp(out)), self.handle)
        return out.reshape(64, 4)

    def phase_times(self):
        out = (C.c_double * 6)()
        self._check(self.lib.gxy_phase_times(self.handle, out), self.handle)
        return list(out)


NPARAM = 17412


class Surrogate:
    """The 2 -> 128 -> 128 -> 4 surrogate MLP on a context's device.

    Thin marshalling over gxy_mlp_*: every computation (initialisation,
    scaling, training, inference, proposals) runs in the library's kernels.
    """

    def __init__(self, ctx: "Context", seed: int = 20536):
        self.ctx = ctx
        self.lib = ctx.lib
        h = C.c_void_p()
        ctx._check(self.lib.gxy_mlp_create(ctx.handle, C.c_uint64(seed), C.byref(h)),
                   ctx.handle)
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            self.lib.gxy_mlp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _chk(self, st):
        self.ctx._check(st, self.ctx.handle)

    @staticmethod
    def _f(a):
        return a.ctypes.data_as(C.POINTER(C.c_float))

    @staticmethod
    def _d(a):
        return a.ctypes.data_as(C.POINTER(C.c_double))

    def get_params(self):
        import numpy as np
        out = np.empty(NPARAM, dtype=np.float32)
        self._chk(self.lib.gxy_mlp_params(self.handle, self._f(out), None))
        return out

    def set_params(self, theta):
        import numpy as np
        a = np.ascontiguousarray(theta, dtype=np.float32)
        assert a.shape == (NPARAM,)
        self._chk(self.lib.gxy_mlp_params(self.handle, None, self._f(a)))

    def train(self, X, Y, epochs=5000, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8,
              log_targets=0b1100, standardize=True):
        import numpy as np
        X = np.ascontiguousarray(X, dtype=np.float64)
        Y = np.ascontiguousarray(Y, dtype=np.float64)
        n = X.shape[0]
        assert X.shape == (n, 2) and Y.shape == (n, 4)
        cfg = TrainCfg(int(epochs), lr, beta1, beta2, eps, int(log_targets), int(standardize))
        hist = np.empty(max(int(epochs), 1), dtype=np.float32)
        self._chk(self.lib.gxy_mlp_train(self.handle, self._d(X), self._d(Y), n,
                                         C.byref(cfg), self._f(hist)))
        return hist[:int(epochs)]

    def grad(self, Xs, Ys):
        import numpy as np
        Xs = np.ascontiguousarray(Xs, dtype=np.float32)
        Ys = np.ascontiguousarray(Ys, dtype=np.float32)
        n = Xs.shape[0]
        g = np.empty(NPARAM, dtype=np.float32)
        loss = np.empty(1, dtype=np.float32)
        self._chk(self.lib.gxy_mlp_grad(self.handle, self._f(Xs), self._f(Ys), n,
                                        self._f(g), self._f(loss)))
        return float(loss[0]), g

    def predict(self, X, bf16=False):
        import numpy as np
        X = np.ascontiguousarray(X, dtype=np.float64)
        n = X.shape[0]
        y = np.empty((n, 4))
        self._chk(self.lib.gxy_mlp_predict(self.handle, self._d(X), n, int(bool(bf16)),
                                           self._d(y)))
        return y

    def scaling(self):
        import numpy as np
        out = np.empty(12)
        mask = C.c_uint32()
        self._chk(self.lib.gxy_mlp_scaling(self.handle, self._d(out), C.byref(mask)))
        return out[0:2], out[6:8], out[2:6], out[8:12], int(mask.value)

    def propose(self, nbeta=256, ndelta=256, beta_lo=0.5, beta_hi=1.5, delta_lo=0.0,
                delta_hi=1.0, seed=20536, jitter=0.5, cv_col=1, chi_col=2):
        import numpy as np
        cfg = ProposeCfg(int(nbeta), int(ndelta), beta_lo, beta_hi, delta_lo, delta_hi,
                         C.c_uint64(seed), jitter, int(cv_col), int(chi_col))
        out = np.empty((2 * int(ndelta), 2))
        self._chk(self.lib.gxy_mlp_propose(self.handle, C.byref(cfg), self._d(out)))
        return out
