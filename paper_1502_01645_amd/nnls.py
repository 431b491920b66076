"""Thin Python binding of libnnls (include/nnls.h): argument marshalling only.

Tensors are PyTorch device tensors; their data pointers and torch's current HIP stream are
handed to the C ABI unchanged.  Every step of the method runs in the library's HIP kernels;
there is no fallback: if libnnls.so is missing or fails to load, every call raises.
"""
from __future__ import annotations

import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnnls.so")

# enums of nnls.h
OK, E_ARG, E_WORKSPACE, E_HIP, E_UNSUPPORTED, E_IO = 0, -1, -2, -3, -4, -5
CONVERGED, MAXITER, BREAKDOWN, NONFINITE, FELL_BACK = 0, 1, 2, 3, 4
GRAM_FP64, GRAM_FP32, GRAM_BF16X3 = 0, 1, 2
F32, F64 = 0, 1
OP_PREPARE, OP_SOLVE, OP_REFINE, OP_SCALES, OP_GRAM = 0, 1, 2, 3, 4
TUNE_BATCHED = 1
NOALLOC_SCRATCH_BYTES = 8 << 20   # NNLS_NOALLOC_SCRATCH_BYTES

_ERRORS = {E_ARG: "invalid argument", E_WORKSPACE: "workspace too small",
           E_HIP: "HIP runtime error", E_UNSUPPORTED: "unsupported shape",
           E_IO: "file error or not a checkpoint of this network"}

_lib = None
_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_i32 = ctypes.c_int32
_sz = ctypes.c_size_t


class NNLSError(RuntimeError):
    pass


class ProblemDesc(ctypes.Structure):
    """nnls_problem_desc of nnls.h (element offsets into the pools)."""
    _fields_ = [(f, ctypes.c_int64) for f in ("d", "n", "offA", "offB", "offQ", "offq", "offX")]


def lib():
    """The loaded libnnls.so (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise NNLSError(f"libnnls.so not built at {LIB_PATH}; run paper_1502_01645_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        L.nnls_workspace_bytes.argtypes = [ctypes.c_int, _i64, _i64, _i64, ctypes.c_int, ctypes.c_int]
        L.nnls_workspace_bytes.restype = _sz
        L.nnls_prepare.argtypes = [_i64, _i64, _i64, _vp, _i64, _vp, _i64, ctypes.c_int, ctypes.c_int,
                                   _vp, _vp, _vp, _vp, _sz, _vp]
        L.nnls_prepare.restype = ctypes.c_int
        L.nnls_solve.argtypes = [_i64, _i64, ctypes.c_int, _vp, _vp, _vp, ctypes.c_double, _i32, _vp,
                                 _vp, _vp, _vp, _vp, _vp, _vp, _i32, _vp, _sz, _vp]
        L.nnls_solve_noalloc.argtypes = [_i64, _i64, ctypes.c_int, _vp, _vp, _vp, ctypes.c_double,
                                         _i32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _i32, _vp]
        L.nnls_solve_noalloc.restype = ctypes.c_int
        L.nnls_prepare_split.argtypes = [_i64, _i64, _i64, _vp, _i64, _vp, _i64, _vp, _vp, _sz,
                                         _vp]
        L.nnls_prepare_split.restype = ctypes.c_int
        L.nnls_prepare_product.argtypes = [_i64, _i64, _i64, _vp, _vp, _vp, _vp, _sz, _vp]
        L.nnls_prepare_product.restype = ctypes.c_int
        L.nnls_column_scales.argtypes = [_i64, _i64, _vp, _i64, ctypes.c_int, _vp, _vp, _sz, _vp]
        L.nnls_column_scales.restype = ctypes.c_int
        L.nnls_gram_rescaled.argtypes = [_i64, _i64, _i64, _vp, _i64, _vp, _i64, ctypes.c_int,
                                         ctypes.c_int, _vp, _vp, _vp, _vp, _sz, _vp]
        L.nnls_gram_rescaled.restype = ctypes.c_int
        L.nnls_gram.argtypes = [_i64, _i64, _i64, _vp, _i64, _vp, _i64, ctypes.c_int, ctypes.c_int,
                                _vp, _vp, _vp, _sz, _vp]
        L.nnls_gram.restype = ctypes.c_int
        L.nnls_transpose.argtypes = [_i64, _i64, _vp, _i64, _vp, _i64, _vp]
        L.nnls_transpose.restype = ctypes.c_int
        L.nnls_rescale_start.argtypes = [_i64, _i64, _vp, _vp, _vp, _vp]
        L.nnls_rescale_start.restype = ctypes.c_int
        L.nnls_solve.restype = ctypes.c_int
        L.nnls_refine.argtypes = [_i64, _i64, _i64, _vp, _i64, _vp, _i64, ctypes.c_int, _vp, _vp, _vp,
                                  _vp, _sz, _vp]
        L.nnls_refine.restype = ctypes.c_int
        L.nnls_batched_workspace_bytes.argtypes = [ctypes.POINTER(ProblemDesc), _i64]
        L.nnls_batched_workspace_bytes.restype = _sz
        L.nnls_batched_plan_create.argtypes = [ctypes.POINTER(ProblemDesc), _i64, ctypes.c_double,
                                               _i32, ctypes.c_char_p] + [_vp] * 11 + [_sz, _vp,
                                               ctypes.POINTER(ctypes.c_void_p)]
        L.nnls_autotune.argtypes = [ctypes.c_char_p, ctypes.c_int, ctypes.POINTER(_i64), _i64, _vp]
        L.nnls_autotune.restype = ctypes.c_int
        L.nnls_batched_plan_create.restype = ctypes.c_int
        L.nnls_batched_plan_launch.argtypes = [_vp, _vp]
        L.nnls_batched_plan_launch.restype = ctypes.c_int
        L.nnls_batched_plan_destroy.argtypes = [_vp]
        L.nnls_batched_plan_destroy.restype = None
        L.nnls_mlp_param_count.argtypes = []
        L.nnls_mlp_param_count.restype = _i64
        L.nnls_mlp_blob_bytes.argtypes = []
        L.nnls_mlp_blob_bytes.restype = _sz
        L.nnls_mlp_workspace_bytes.argtypes = [_i64, ctypes.c_int]
        L.nnls_mlp_workspace_bytes.restype = _sz
        L.nnls_mlp_reset_state.argtypes = [_vp, _vp]
        L.nnls_mlp_reset_state.restype = ctypes.c_int
        L.nnls_mlp_fit_input_workspace_bytes.argtypes = []
        L.nnls_mlp_fit_input_workspace_bytes.restype = _sz
        L.nnls_mlp_fit_input.argtypes = [_i64, _vp, _vp, _vp, _sz, _vp]
        L.nnls_mlp_fit_input.restype = ctypes.c_int
        L.nnls_mlp_forward.argtypes = [_i64, _vp, _vp, _vp, _vp, _sz, _vp]
        L.nnls_mlp_forward.restype = ctypes.c_int
        L.nnls_mlp_gradients.argtypes = [_i64, _vp, _vp, _vp, ctypes.c_float, _vp, _vp, _vp, _sz,
                                         _vp]
        L.nnls_mlp_gradients.restype = ctypes.c_int
        L.nnls_mlp_train_step.argtypes = [_i64, _vp, _vp, _vp, ctypes.c_float, _i64,
                                          ctypes.c_float, _vp, _vp, _sz, _vp]
        L.nnls_mlp_train_step.restype = ctypes.c_int
        L.nnls_mlp_save.argtypes = [_vp, _i64, ctypes.c_char_p, _vp]
        L.nnls_mlp_save.restype = ctypes.c_int
        L.nnls_mlp_load.argtypes = [_vp, ctypes.POINTER(_i64), ctypes.c_char_p, _vp]
        L.nnls_mlp_load.restype = ctypes.c_int
        L.nnls_mlp_inputs.argtypes = [_i64, _i64, _vp, _vp, _vp, _vp, _vp]
        L.nnls_mlp_inputs.restype = ctypes.c_int
        L.nnls_warm_start_workspace_bytes.argtypes = [_i64, _i64]
        L.nnls_warm_start_workspace_bytes.restype = _sz
        L.nnls_warm_start.argtypes = [_i64, _i64, _vp, _vp, _vp, _vp, _vp, _vp, _sz, _vp]
        L.nnls_warm_start.restype = ctypes.c_int
        L.nnls_solver_name.argtypes = [_i64, _i64, ctypes.c_int]
        L.nnls_solver_name.restype = ctypes.c_char_p
        L.nnls_last_hip_error.argtypes = []
        L.nnls_last_hip_error.restype = ctypes.c_char_p
        L.nnls_version.argtypes = []
        L.nnls_version.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _check(rc: int, what: str):
    if rc != OK:
        msg = _ERRORS.get(rc, f"error {rc}")
        if rc == E_HIP:
            msg += ": " + lib().nnls_last_hip_error().decode()
        raise NNLSError(f"{what}: {msg}")


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _dtype_code(t: torch.Tensor) -> int:
    if t.dtype == torch.float32:
        return F32
    if t.dtype == torch.float64:
        return F64
    raise NNLSError(f"unsupported dtype {t.dtype}")


def solver_name(n: int, k: int, dtype: int = F32) -> str:
    """The solver nnls_solve picks for this shape on the current device."""
    return lib().nnls_solver_name(n, k, dtype).decode()


def workspace_bytes(op: int, d: int, n: int, k: int, mode: int, dtype: int) -> int:
    return int(lib().nnls_workspace_bytes(op, d, n, k, mode, dtype))


def _workspace(nbytes: int, device, ws=None):
    if nbytes == 0:
        return None
    if ws is not None and ws.numel() >= nbytes:
        return ws
    return torch.empty(nbytes, dtype=torch.uint8, device=device)


def prepare(A: torch.Tensor, B: torch.Tensor | None = None, mode: int | None = None, out=None,
            ws=None):
    """Gram product and rescale (Algorithm 1).  Returns (Q, q, s)."""
    assert A.dim() == 2 and A.stride(1) == 1
    d, n = A.shape
    dt = _dtype_code(A)
    if mode is None:
        mode = GRAM_FP64 if dt == F64 else GRAM_BF16X3
    if B is not None:
        if B.dim() == 1:
            B = B.reshape(d, 1)
        assert B.shape[0] == d and B.stride(1) == 1 and B.dtype == A.dtype
        k = B.shape[1]
    else:
        k = 0
    if out is None:
        Q = torch.empty((n, n), dtype=A.dtype, device=A.device)
        q = torch.empty((n, max(k, 1)), dtype=A.dtype, device=A.device)[:, :k]
        s = torch.empty(n, dtype=torch.float64, device=A.device)
    else:
        Q, q, s = out
    wsb = workspace_bytes(OP_PREPARE, d, n, k, mode, dt)
    ws = _workspace(wsb, A.device, ws)
    rc = lib().nnls_prepare(d, n, k, _ptr(A), A.stride(0), _ptr(B), B.stride(0) if B is not None else 0,
                            mode, dt, _ptr(Q), _ptr(q) if k > 0 else None, _ptr(s), _ptr(ws), wsb,
                            _stream(A.device))
    _check(rc, "nnls_prepare")
    return Q, q, s


def prepare_split(A: torch.Tensor, B: torch.Tensor, s: torch.Tensor, ws: torch.Tensor):
    """nnls_prepare_split (FP32, BF16x3): the operand split into ws and the scales s."""
    d, n = A.shape
    if B is None or B.numel() == 0:
        B, k, ldb = None, 0, 1
    else:
        B = B.reshape(d, -1)
        k, ldb = B.shape[1], B.stride(0)
        assert B.stride(1) == 1
    assert A.dtype == torch.float32 and A.stride(1) == 1
    wsb = workspace_bytes(OP_PREPARE, d, n, k, GRAM_BF16X3, F32)
    assert ws.numel() >= wsb
    _check(lib().nnls_prepare_split(d, n, k, _ptr(A), A.stride(0), _ptr(B), ldb, _ptr(s),
                                    _ptr(ws), ws.numel(), _stream(A.device)),
           "nnls_prepare_split")


def prepare_product(d: int, s: torch.Tensor, Q: torch.Tensor, q: torch.Tensor, ws: torch.Tensor):
    """nnls_prepare_product: Q, q from the split planes a prepare_split call left in ws."""
    n = Q.shape[0]
    k = 0 if q is None else (q.shape[1] if q.dim() == 2 else 1)
    _check(lib().nnls_prepare_product(d, n, k, _ptr(s), _ptr(Q), _ptr(q if k else None),
                                      _ptr(ws), ws.numel(), _stream(Q.device)),
           "nnls_prepare_product")


def column_scales(A: torch.Tensor, out=None, ws=None):
    """s_i = ||A_i|| in FP64 (1 for a zero column): the scale of the rescaling (4)."""
    d, n = A.shape
    dt = _dtype_code(A)
    s = out if out is not None else torch.empty(n, dtype=torch.float64, device=A.device)
    wsb = workspace_bytes(OP_SCALES, d, n, 0, 0, dt)
    ws = _workspace(wsb, A.device, ws)
    rc = lib().nnls_column_scales(d, n, _ptr(A), A.stride(0), dt, _ptr(s), _ptr(ws), wsb,
                                  _stream(A.device))
    _check(rc, "nnls_column_scales")
    return s


def gram_rescaled(A: torch.Tensor, B: torch.Tensor | None, s: torch.Tensor, mode: int | None = None,
                  out=None, ws=None):
    """Gram product with the rescale epilogue, given s.  Returns (Q, q)."""
    d, n = A.shape
    dt = _dtype_code(A)
    if mode is None:
        mode = GRAM_FP64 if dt == F64 else GRAM_BF16X3
    k = 0 if B is None else B.reshape(d, -1).shape[1]
    if B is not None:
        B = B.reshape(d, k)
    if out is None:
        Q = torch.empty((n, n), dtype=A.dtype, device=A.device)
        q = torch.empty((n, max(k, 1)), dtype=A.dtype, device=A.device)[:, :k]
    else:
        Q, q = out
    wsb = workspace_bytes(OP_GRAM, d, n, k, mode, dt)
    ws = _workspace(wsb, A.device, ws)
    rc = lib().nnls_gram_rescaled(d, n, k, _ptr(A), A.stride(0), _ptr(B),
                                  B.stride(0) if B is not None else 0, mode, dt, _ptr(s), _ptr(Q),
                                  _ptr(q) if k > 0 else None, _ptr(ws), wsb, _stream(A.device))
    _check(rc, "nnls_gram_rescaled")
    return Q, q


def gram(A: torch.Tensor, B: torch.Tensor | None = None, mode: int | None = None, out=None,
         ws=None):
    """H = A^T A and h = -A^T B without the rescale (Problem (2)).  Returns (H, h)."""
    d, n = A.shape
    dt = _dtype_code(A)
    if mode is None:
        mode = GRAM_FP64 if dt == F64 else GRAM_BF16X3
    k = 0 if B is None else B.reshape(d, -1).shape[1]
    if B is not None:
        B = B.reshape(d, k)
    if out is None:
        H = torch.empty((n, n), dtype=A.dtype, device=A.device)
        h = torch.empty((n, max(k, 1)), dtype=A.dtype, device=A.device)[:, :k]
    else:
        H, h = out
    wsb = workspace_bytes(OP_GRAM, d, n, k, mode, dt)
    ws = _workspace(wsb, A.device, ws)
    rc = lib().nnls_gram(d, n, k, _ptr(A), A.stride(0), _ptr(B), B.stride(0) if B is not None else 0,
                         mode, dt, _ptr(H), _ptr(h) if k > 0 else None, _ptr(ws), wsb,
                         _stream(A.device))
    _check(rc, "nnls_gram")
    return H, h


def transpose(src: torch.Tensor, out=None) -> torch.Tensor:
    """dst = src^T for an FP32 matrix (row-major, unit column stride)."""
    assert src.dim() == 2 and src.stride(1) == 1 and src.dtype == torch.float32
    rows, cols = src.shape
    dst = out if out is not None else torch.empty((cols, rows), dtype=src.dtype, device=src.device)
    assert dst.shape == (cols, rows) and dst.stride(1) == 1
    rc = lib().nnls_transpose(rows, cols, _ptr(src), src.stride(0), _ptr(dst), dst.stride(0),
                              _stream(src.device))
    _check(rc, "nnls_transpose")
    return dst


def rescale_start(s: torch.Tensor, X: torch.Tensor, out=None) -> torch.Tensor:
    """Y0 = s .* X: a start in the original variables mapped to the rescaled ones."""
    assert X.dim() == 2 and X.is_contiguous() and X.dtype == torch.float32
    n, k = X.shape
    Y0 = out if out is not None else torch.empty_like(X)
    rc = lib().nnls_rescale_start(n, k, _ptr(s), _ptr(X), _ptr(Y0), _stream(X.device))
    _check(rc, "nnls_rescale_start")
    return Y0


def solve(Q: torch.Tensor, q: torch.Tensor, s: torch.Tensor | None = None, tol: float = 1e-5,
          max_iter: int = 0, Y0: torch.Tensor | None = None, out=None, ws=None, rows_read=None,
          trace=None):
    """Algorithm 2 on every column of q, then x = y / s.  Returns (X, iters, kkt, status).
    rows_read (optional int64 [k] tensor) receives the rows of Q the products read; trace
    (optional FP32 [k, T, 2] tensor) the per-update record (r, ||gbar||^2) for t < T."""
    n = Q.shape[0]
    if q.dim() == 1:
        q = q.reshape(n, 1)
    k = q.shape[1]
    dt = _dtype_code(Q)
    assert Q.is_contiguous() and q.is_contiguous() and q.dtype == Q.dtype
    if Y0 is not None:
        Y0 = Y0.reshape(n, k)
        assert Y0.is_contiguous() and Y0.dtype == Q.dtype
    if out is None:
        X = torch.empty((n, k), dtype=Q.dtype, device=Q.device)
        iters = torch.empty(k, dtype=torch.int32, device=Q.device)
        kkt = torch.empty(k, dtype=torch.float64, device=Q.device)
        status = torch.empty(k, dtype=torch.int32, device=Q.device)
    else:
        X, iters, kkt, status = out
    wsb = workspace_bytes(OP_SOLVE, 0, n, k, 0, dt)
    ws = _workspace(wsb, Q.device, ws)
    tl = _trace_len(trace, k)
    rc = lib().nnls_solve(n, k, dt, _ptr(Q), _ptr(q), _ptr(s), float(tol), int(max_iter), _ptr(Y0),
                          _ptr(X), _ptr(iters), _ptr(kkt), _ptr(status), _ptr(rows_read),
                          _ptr(trace), tl, _ptr(ws), wsb, _stream(Q.device))
    _check(rc, "nnls_solve")
    return X, iters, kkt, status


def _trace_len(trace, k):
    if trace is None:
        return 0
    assert trace.dtype == torch.float32 and trace.is_contiguous()
    assert trace.dim() == 3 and trace.shape[0] == k and trace.shape[2] == 2
    return int(trace.shape[1])


def solve_noalloc(Q: torch.Tensor, q: torch.Tensor, s: torch.Tensor | None, tol: float,
                  max_iter: int, Y0: torch.Tensor | None, out, rows_read=None, trace=None):
    """nnls_solve_noalloc: as solve(), with the solver state in the library's fixed device
    array instead of a workspace.  The caller passes every output (out = (X, iters, kkt,
    status)); nothing is allocated here or in the library."""
    n = Q.shape[0]
    if q.dim() == 1:
        q = q.reshape(n, 1)
    k = q.shape[1]
    dt = _dtype_code(Q)
    assert Q.is_contiguous() and q.is_contiguous() and q.dtype == Q.dtype
    if Y0 is not None:
        Y0 = Y0.reshape(n, k)
        assert Y0.is_contiguous() and Y0.dtype == Q.dtype
    X, iters, kkt, status = out
    rc = lib().nnls_solve_noalloc(n, k, dt, _ptr(Q), _ptr(q), _ptr(s), float(tol), int(max_iter),
                                  _ptr(Y0), _ptr(X), _ptr(iters), _ptr(kkt), _ptr(status),
                                  _ptr(rows_read), _ptr(trace), _trace_len(trace, k),
                                  _stream(Q.device))
    _check(rc, "nnls_solve_noalloc")
    return X, iters, kkt, status


def refine(A: torch.Tensor, B: torch.Tensor, X: torch.Tensor, out=None, ws=None,
           objective: bool = True):
    """FP64 check + one refinement step against (A, B); X is updated in place.
    Returns (kkt64, obj64); obj64 is None when objective is False (or out[1] is None)."""
    d, n = A.shape
    if B.dim() == 1:
        B = B.reshape(d, 1)
    k = B.shape[1]
    dt = _dtype_code(A)
    assert X.shape == (n, k) and X.is_contiguous() and X.dtype == A.dtype
    if out is None:
        kkt64 = torch.empty(k, dtype=torch.float64, device=A.device)
        obj64 = torch.empty(k, dtype=torch.float64, device=A.device) if objective else None
    else:
        kkt64, obj64 = out
    wsb = workspace_bytes(OP_REFINE, d, n, k, 0, dt)
    ws = _workspace(wsb, A.device, ws)
    rc = lib().nnls_refine(d, n, k, _ptr(A), A.stride(0), _ptr(B), B.stride(0), dt, _ptr(X),
                           _ptr(kkt64), _ptr(obj64), _ptr(ws), wsb, _stream(A.device))
    _check(rc, "nnls_refine")
    return kkt64, obj64


def nnls(A: torch.Tensor, B: torch.Tensor, tol: float = 1e-5, max_iter: int = 0,
         mode: int | None = None, refine_step: bool = True, inner_tol: float | None = None):
    """Algorithm 1 end to end on the GPU: prepare, solve, FP64 refine.
    Returns dict(X, iters, kkt, status, kkt64, obj64)."""
    Q, q, s = prepare(A, B, mode)
    X, iters, kkt, status = solve(Q, q, s, tol if inner_tol is None else inner_tol, max_iter)
    res = dict(X=X, iters=iters, kkt=kkt, status=status, Q=Q, q=q, s=s)
    if refine_step:
        kkt64, obj64 = refine(A, B, X)
        res.update(kkt64=kkt64, obj64=obj64)
    return res


def pack_problems(problems, device):
    """Lay out a list of (A_i [d_i, n_i], b_i [d_i]) host FP32 arrays as the A / B pools of a
    batched plan.  Returns (A_pool, B_pool, descriptors)."""
    import numpy as np
    descs = (ProblemDesc * len(problems))()
    offA = offB = offQ = offq = 0
    a_parts, b_parts = [], []
    for i, (A, b) in enumerate(problems):
        d, n = A.shape
        descs[i] = ProblemDesc(d, n, offA, offB, offQ, offq, offq)
        a_parts.append(np.ascontiguousarray(A, dtype=np.float32).reshape(-1))
        b_parts.append(np.ascontiguousarray(b, dtype=np.float32).reshape(-1))
        offA += d * n
        offB += d
        offQ += n * n
        offq += n
    A_pool = torch.from_numpy(np.concatenate(a_parts)).to(device)
    B_pool = torch.from_numpy(np.concatenate(b_parts)).to(device)
    return A_pool, B_pool, descs


def autotune(cache_path, shapes, device=None, op=TUNE_BATCHED):
    """nnls_autotune: measure the per-size-class parameters for problems of the given shapes
    ((d, n) pairs) on the device and record them in the JSON cache at cache_path."""
    flat = (_i64 * (2 * len(shapes)))()
    for i, (d, n) in enumerate(shapes):
        flat[2 * i], flat[2 * i + 1] = int(d), int(n)
    dev = torch.device("cuda") if device is None else device
    rc = lib().nnls_autotune(os.fsencode(cache_path), op, flat, len(shapes), _stream(dev))
    _check(rc, "nnls_autotune")


class BatchedPlan:
    """An uneven batch captured as one graph (nnls_batched_plan_*).  Outputs: Q, q, s, X pools
    and per-problem iters, kkt, status, rows_read."""

    def __init__(self, A_pool, B_pool, descs, tol=1e-5, max_iter=0, tune_cache=None):
        dev = A_pool.device
        count = len(descs)
        sum_n = sum(int(descs[i].n) for i in range(count))
        sum_nn = sum(int(descs[i].n) ** 2 for i in range(count))
        self.descs = descs
        self.A_pool, self.B_pool = A_pool, B_pool
        self.Q_pool = torch.empty(sum_nn, dtype=torch.float32, device=dev)
        self.q_pool = torch.empty(sum_n, dtype=torch.float32, device=dev)
        self.s_pool = torch.empty(sum_n, dtype=torch.float64, device=dev)
        self.X_pool = torch.empty(sum_n, dtype=torch.float32, device=dev)
        self.iters = torch.empty(count, dtype=torch.int32, device=dev)
        self.kkt = torch.empty(count, dtype=torch.float64, device=dev)
        self.status = torch.empty(count, dtype=torch.int32, device=dev)
        self.rows_read = torch.zeros(count, dtype=torch.int64, device=dev)
        wsb = int(lib().nnls_batched_workspace_bytes(descs, count))
        self.ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
        self._capture = torch.cuda.Stream(device=dev)
        torch.cuda.synchronize(dev)
        handle = ctypes.c_void_p()
        rc = lib().nnls_batched_plan_create(
            descs, count, float(tol), int(max_iter),
            None if tune_cache is None else os.fsencode(tune_cache), _ptr(A_pool), _ptr(B_pool),
            _ptr(self.Q_pool), _ptr(self.q_pool), _ptr(self.s_pool), _ptr(self.X_pool),
            _ptr(self.iters), _ptr(self.kkt), _ptr(self.status), _ptr(self.rows_read),
            _ptr(self.ws), wsb, ctypes.c_void_p(self._capture.cuda_stream), ctypes.byref(handle))
        _check(rc, "nnls_batched_plan_create")
        self.handle = handle

    def launch(self):
        rc = lib().nnls_batched_plan_launch(self.handle, _stream(self.A_pool.device))
        _check(rc, "nnls_batched_plan_launch")

    def x(self, i):
        d = self.descs[i]
        return self.X_pool[d.offX:d.offX + d.n]

    def close(self):
        if getattr(self, "handle", None):
            lib().nnls_batched_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


MLP_IN = 256


def mlp_inputs(q, Y=None):
    """(U, T): network inputs q / ||q|| and targets Y / ||q||, one row per column of q."""
    n, k = q.shape
    assert q.is_contiguous() and q.dtype == torch.float32
    U = torch.empty((k, n), dtype=torch.float32, device=q.device)
    T = None
    if Y is not None:
        assert Y.shape == q.shape and Y.is_contiguous() and Y.dtype == torch.float32
        T = torch.empty((k, n), dtype=torch.float32, device=q.device)
    _check(lib().nnls_mlp_inputs(n, k, _ptr(q), _ptr(Y), _ptr(U), _ptr(T), _stream(q.device)),
           "nnls_mlp_inputs")
    return U, T


class WarmStartNet:
    """The warm-start network's parameter blob (nnls_mlp_* / nnls_warm_start of nnls.h).
    `params` are the initial FP32 master weights in the library's layout; shift and scale the
    input standardisation (default 0 and 1; nnls_mlp_fit_input fits them with fit_input)."""

    def _alloc(self, device):
        L = lib()
        self.P = int(L.nnls_mlp_param_count())
        self.device = torch.device(device)
        self.blob = torch.empty(int(L.nnls_mlp_blob_bytes()), dtype=torch.uint8, device=device)
        self.master = self.blob[:4 * self.P].view(torch.float32)
        norm = self.blob[14 * self.P:14 * self.P + 8 * MLP_IN].view(torch.float32)
        self.shift, self.scale = norm[:MLP_IN], norm[MLP_IN:]
        self.step = 0
        self._ws = {}

    def __init__(self, params, device, shift=None, scale=None):
        L = lib()
        self._alloc(device)
        p = torch.as_tensor(params, dtype=torch.float32).reshape(-1)
        if p.numel() != self.P:
            raise NNLSError(f"expected {self.P} parameters, got {p.numel()}")
        self.master.copy_(p.to(device))
        self.shift.copy_(torch.as_tensor(0.0 if shift is None else shift, dtype=torch.float32)
                         .expand(MLP_IN).to(device))
        self.scale.copy_(torch.as_tensor(1.0 if scale is None else scale, dtype=torch.float32)
                         .expand(MLP_IN).to(device))
        _check(L.nnls_mlp_reset_state(_ptr(self.blob), _stream(self.device)), "nnls_mlp_reset_state")

    def _wsb(self, key, nbytes):
        ws = self._ws.get(key)
        if ws is None or ws.numel() < nbytes:
            ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            self._ws[key] = ws
        return ws

    def fit_input(self, U):
        """shift, scale = per-feature mean and 1 / std of the rows of U [count, 256]."""
        nb = int(lib().nnls_mlp_fit_input_workspace_bytes())
        ws = self._wsb("fit", nb)
        _check(lib().nnls_mlp_fit_input(U.shape[0], _ptr(self.blob), _ptr(U), _ptr(ws), nb,
                                        _stream(self.device)), "nnls_mlp_fit_input")

    def forward(self, u):
        b = u.shape[0]
        z = torch.empty((b, MLP_IN), dtype=torch.float32, device=self.device)
        nb = int(lib().nnls_mlp_workspace_bytes(b, 0))
        ws = self._wsb(("f", b), nb)
        _check(lib().nnls_mlp_forward(b, _ptr(self.blob), _ptr(u), _ptr(z), _ptr(ws), nb,
                                      _stream(self.device)), "nnls_mlp_forward")
        return z

    def gradients(self, u, target, lam):
        b = u.shape[0]
        grad = torch.empty(self.P, dtype=torch.float32, device=self.device)
        loss = torch.empty(1, dtype=torch.float32, device=self.device)
        nb = int(lib().nnls_mlp_workspace_bytes(b, 1))
        ws = self._wsb(("t", b), nb)
        _check(lib().nnls_mlp_gradients(b, _ptr(self.blob), _ptr(u), _ptr(target), float(lam),
                                        _ptr(grad), _ptr(loss), _ptr(ws), nb, _stream(self.device)),
               "nnls_mlp_gradients")
        return loss, grad

    def train_step(self, u, target, lr, lam, loss=None):
        """One Adam step; returns the device loss tensor (the batch loss before the step)."""
        b = u.shape[0]
        if loss is None:
            loss = torch.empty(1, dtype=torch.float32, device=self.device)
        nb = int(lib().nnls_mlp_workspace_bytes(b, 1))
        ws = self._wsb(("t", b), nb)
        self.step += 1
        _check(lib().nnls_mlp_train_step(b, _ptr(self.blob), _ptr(u), _ptr(target), float(lr),
                                         self.step, float(lam), _ptr(loss), _ptr(ws), nb,
                                         _stream(self.device)), "nnls_mlp_train_step")
        return loss

    def save(self, path):
        """Writes the whole blob and the Adam step count to a checkpoint file (nnls_mlp_save)."""
        _check(lib().nnls_mlp_save(_ptr(self.blob), self.step, os.fsencode(path),
                                   _stream(self.device)), "nnls_mlp_save")

    def load(self, path):
        """Replaces the blob and the step count by a checkpoint's (nnls_mlp_load); training
        continues where the checkpointed run stopped."""
        step = _i64(0)
        _check(lib().nnls_mlp_load(_ptr(self.blob), ctypes.byref(step), os.fsencode(path),
                                   _stream(self.device)), "nnls_mlp_load")
        self.step = int(step.value)

    @classmethod
    def from_checkpoint(cls, path, device):
        """A network restored from a checkpoint file."""
        net = cls.__new__(cls)
        net._alloc(device)
        net.load(path)
        return net

    def warm_start(self, Q, q, out=None):
        """(Y0 [256, k], fell_back [k] int32) for the rescaled problem (Q, q)."""
        n = Q.shape[0]
        if q.dim() == 1:
            q = q.reshape(n, 1)
        k = q.shape[1]
        assert Q.is_contiguous() and q.is_contiguous() and Q.dtype == torch.float32
        if out is None:
            Y0 = torch.empty((n, k), dtype=torch.float32, device=self.device)
            fb = torch.empty(k, dtype=torch.int32, device=self.device)
        else:
            Y0, fb = out
        nb = int(lib().nnls_warm_start_workspace_bytes(n, k))
        ws = self._wsb(("w", k), max(nb, 1))
        _check(lib().nnls_warm_start(n, k, _ptr(Q), _ptr(q), _ptr(self.blob), _ptr(Y0), _ptr(fb),
                                     _ptr(ws), nb, _stream(self.device)), "nnls_warm_start")
        return Y0, fb
