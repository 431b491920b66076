"""ctypes front end of the plain C oracle (oracle.c), plus the parity metrics built from it.

Test infrastructure only (tests, smoke check, CPU-baseline timing); never on the product path.
Inputs are promoted exactly to FP64 before they reach the C code.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

CONVERGED, MAXITER, BREAKDOWN, NONFINITE = 0, 1, 2, 3

_dp = ctypes.POINTER(ctypes.c_double)
_lp = ctypes.POINTER(ctypes.c_int64)
_ip = ctypes.POINTER(ctypes.c_int32)
_i64 = ctypes.c_int64


def build(plant: int = 0, out: str | None = None) -> str:
    """Compile oracle.c with gcc (OpenMP).  plant != 0 builds a deliberately broken variant for
    the pin-strength test."""
    if out is None:
        out = _LIB_PATH if plant == 0 else os.path.join(_HERE, "_build", f"liboracle_plant{plant}.so")
    os.makedirs(os.path.dirname(out), exist_ok=True)
    tmp = out + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", f"-DPLANT={plant}",
           _SRC, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


class Oracle:
    """Handle on one build of the oracle library."""

    def __init__(self, path: str):
        lib = ctypes.CDLL(path)
        lib.oracle_gram.argtypes = [_i64, _i64, _i64, _dp, _dp, _dp, _dp, ctypes.c_int]
        lib.oracle_gram.restype = None
        lib.oracle_rescale.argtypes = [_i64, _i64, _dp, _dp, _dp, _dp, _dp]
        lib.oracle_rescale.restype = None
        lib.oracle_nqp.argtypes = [_i64, _dp, _dp, _dp, ctypes.c_double, _i64, _dp, _lp, _dp, _dp]
        lib.oracle_nqp.restype = ctypes.c_int
        lib.oracle_nnls.argtypes = [_i64, _i64, _i64, _dp, _dp, _dp, ctypes.c_double, _i64, _dp,
                                    _lp, _dp, _ip, _dp, _dp, _dp, ctypes.c_int]
        lib.oracle_nnls.restype = None
        lib.oracle_kkt_x.argtypes = [_i64, _i64, _i64, _dp, _dp, _dp, _dp, _dp, ctypes.c_int]
        lib.oracle_kkt_x.restype = None
        lib.oracle_num_threads.argtypes = []
        lib.oracle_num_threads.restype = ctypes.c_int
        self.lib = lib
        self.path = path

    @staticmethod
    def _f64(a) -> np.ndarray:
        return np.ascontiguousarray(np.asarray(a, dtype=np.float64))

    @staticmethod
    def _ptr(a: np.ndarray):
        return a.ctypes.data_as(_dp)

    def num_threads(self) -> int:
        return int(self.lib.oracle_num_threads())

    def gram(self, A, B=None, nthreads: int = 0):
        """H = A^T A and h = -A^T B (Problem (2))."""
        A = self._f64(A)
        d, n = A.shape
        if B is None:
            B = np.zeros((d, 0))
        B = self._f64(B).reshape(d, -1)
        k = B.shape[1]
        H = np.zeros((n, n))
        h = np.zeros((n, k))
        self.lib.oracle_gram(d, n, k, self._ptr(A), self._ptr(B), self._ptr(H), self._ptr(h),
                             nthreads)
        return H, h

    def rescale(self, H, h):
        """(s, Q, q) of Algorithm 1 from (H, h)."""
        H = self._f64(H)
        n = H.shape[0]
        h = self._f64(h).reshape(n, -1)
        k = h.shape[1]
        s = np.zeros(n)
        Q = np.zeros((n, n))
        q = np.zeros((n, k))
        self.lib.oracle_rescale(n, k, self._ptr(H), self._ptr(h), self._ptr(s), self._ptr(Q),
                                self._ptr(q))
        return s, Q, q

    def prepare(self, A, B, nthreads: int = 0):
        H, h = self.gram(A, B, nthreads)
        return self.rescale(H, h)

    def nqp(self, Q, q, tol: float, max_iter: int, y0=None, trace: bool = False):
        """Algorithm 2 on one column.  Returns (y, iters, kkt, status[, trace])."""
        Q = self._f64(Q)
        n = Q.shape[0]
        q = self._f64(q).reshape(n)
        y = np.zeros(n)
        it = ctypes.c_int64(0)
        kkt = ctypes.c_double(0.0)
        y0p = self._ptr(self._f64(y0).reshape(n)) if y0 is not None else None
        y0keep = y0p  # keep the buffer alive during the call
        tr = np.full(max_iter + 1, np.nan) if trace else None
        st = self.lib.oracle_nqp(n, self._ptr(Q), self._ptr(q), y0keep, tol, max_iter,
                                 self._ptr(y), ctypes.byref(it), ctypes.byref(kkt),
                                 self._ptr(tr) if trace else None)
        out = (y, int(it.value), float(kkt.value), int(st))
        if trace:
            out = out + (tr[: int(it.value) + 1],)
        return out

    def nnls(self, A, B, tol: float, max_iter: int = 0, Y0=None, nthreads: int = 0,
             want_problem: bool = False):
        """Algorithm 1 for every column of B.  max_iter 0 means 5 n (the paper's cap).
        Returns dict(X, iters, kkt, status[, Q, q, s])."""
        A = self._f64(A)
        d, n = A.shape
        B = self._f64(B).reshape(d, -1)
        k = B.shape[1]
        if max_iter <= 0:
            max_iter = 5 * n
        X = np.zeros((n, k))
        iters = np.zeros(k, dtype=np.int64)
        kkt = np.zeros(k)
        status = np.zeros(k, dtype=np.int32)
        Y0a = self._f64(Y0).reshape(n, k) if Y0 is not None else None
        Qo = np.zeros((n, n)) if want_problem else None
        qo = np.zeros((n, k)) if want_problem else None
        so = np.zeros(n) if want_problem else None
        self.lib.oracle_nnls(d, n, k, self._ptr(A), self._ptr(B),
                             self._ptr(Y0a) if Y0a is not None else None, tol, max_iter,
                             self._ptr(X), iters.ctypes.data_as(_lp), self._ptr(kkt),
                             status.ctypes.data_as(_ip),
                             self._ptr(Qo) if want_problem else None,
                             self._ptr(qo) if want_problem else None,
                             self._ptr(so) if want_problem else None, nthreads)
        out = dict(X=X, iters=iters, kkt=kkt, status=status)
        if want_problem:
            out.update(Q=Qo, q=qo, s=so)
        return out

    def kkt_x(self, A, B, X, nthreads: int = 0):
        """(r, F) per column: relative KKT residual and 1/2||Ax-b||^2 against the original data."""
        A = self._f64(A)
        d, n = A.shape
        B = self._f64(B).reshape(d, -1)
        k = B.shape[1]
        X = self._f64(X).reshape(n, k)
        r = np.zeros(k)
        F = np.zeros(k)
        self.lib.oracle_kkt_x(d, n, k, self._ptr(A), self._ptr(B), self._ptr(X), self._ptr(r),
                              self._ptr(F), nthreads)
        return r, F


def refine_candidate(A, B, X, out_dtype=np.float64) -> np.ndarray:
    """One step of Algorithm 2 taken from x in FP64 against the original data (the refinement
    step of the FP64 check): y = s x, gradient of Problem (5) g_y = A^T (A x - b) / s, masked
    gradient p on the passive set, exact step alpha = ||p||^2 / ||A (p / s)||^2, projection
    x' = [x - alpha p / s]_+, rounded to the output type.  Plain numpy, one column at a time."""
    A = np.asarray(A, dtype=np.float64)
    d, n = A.shape
    B = np.asarray(B, dtype=np.float64).reshape(d, -1)
    X = np.asarray(X, dtype=np.float64).reshape(n, -1)
    s = np.sqrt(np.sum(A * A, axis=0))
    s = np.where(s > 0, s, 1.0)
    out = np.zeros_like(X)
    for c in range(X.shape[1]):
        x = X[:, c]
        gy = (A.T @ (A @ x - B[:, c])) / s
        y = s * x
        p = np.where((y > 0) | (gy < 0), gy, 0.0)
        D = p / s
        den = np.sum((A @ D) ** 2)
        alpha = np.sum(p * p) / den if den > 0 else 0.0
        out[:, c] = np.maximum(x - alpha * D, 0.0)
    return out.astype(out_dtype).astype(np.float64)


_default: Oracle | None = None


def load(path: str | None = None) -> Oracle:
    """The default oracle build, compiled on first use if nothing is built yet."""
    global _default
    if path is not None:
        return Oracle(path)
    if _default is None:
        if not os.path.exists(_LIB_PATH):
            build()
        _default = Oracle(_LIB_PATH)
    return _default


@dataclass
class Reference:
    """Tight solve of one instance used as the yardstick of the parity metrics."""
    X: np.ndarray
    F: np.ndarray          # 1/2 ||A x* - b||^2 per column
    half_bb: np.ndarray    # 1/2 ||b||^2 per column
    iters: np.ndarray
    kkt: np.ndarray


def reference_solution(A, B, tight: float = 1e-12, max_iter: int = 200000, nthreads: int = 0,
                       orc: Oracle | None = None) -> Reference:
    """The oracle run to a tight residual: its objective serves as F* for the gap metric."""
    orc = orc or load()
    B = np.asarray(B, dtype=np.float64).reshape(A.shape[0], -1)
    out = orc.nnls(A, B, tight, max_iter, nthreads=nthreads)
    bad = out["kkt"] > tight
    if np.any(bad):
        # Stalled at rounding level: accept 1e-10 as the reference accuracy.
        assert np.all(out["kkt"] <= 1e-10), f"reference solve stalled at {out['kkt'].max():.3e}"
    _, F = orc.kkt_x(A, B, out["X"], nthreads)
    half_bb = 0.5 * np.sum(B * B, axis=0)
    return Reference(out["X"], F, half_bb, out["iters"], out["kkt"])


def relative_gap(F, ref: Reference) -> np.ndarray:
    """(f(y) - f*) / |f*| with f = F - 1/2||b||^2, evaluated from residual-based objectives.
    Where f* = 0 (x* = 0) the absolute gap is returned."""
    F = np.asarray(F, dtype=np.float64)
    fstar = ref.F - ref.half_bb
    denom = np.where(np.abs(fstar) > 0, np.abs(fstar), 1.0)
    return (F - ref.F) / denom
