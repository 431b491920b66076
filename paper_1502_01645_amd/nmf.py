"""Alternating NNLS for a nonnegative matrix factorisation V ~ W H (the use of NNLS that the
Introduction motivates), built only from the library's calls.

Each half of an outer step is one NNLS problem with many right-hand sides sharing its matrix:
    H <- argmin_{H >= 0} ||V - W H||:      matrix W [m, r], right-hand sides the p columns of V;
    W <- argmin_{W >= 0} ||V^T - H^T W^T||: matrix H^T [p, r], right-hand sides the m columns of
                                            V^T, the transposes made by nnls_transpose.
Each half runs nnls_prepare (Gram and rescale, Algorithm 1), nnls_solve (Algorithm 2 on the
matrix cores; after the first step started from the half's previous factor, mapped to the
rescaled variables by nnls_rescale_start) and nnls_refine, whose FP64 objectives give
1/2 ||V - W H||_F^2 exactly.  This
module only orders the calls and owns the buffers; every arithmetic step runs in the library.
"""
from __future__ import annotations

import torch

from . import nnls as N


class AlternatingNNLS:
    """Buffers and workspaces for repeated outer steps on V [m, p] with rank r (FP32, device).
    max_iter caps the updates per column (the paper's 5 n is far too few at a small rank r)."""

    def __init__(self, V: torch.Tensor, W0: torch.Tensor, tol: float = 1e-5,
                 inner_tol: float = 8e-6, max_iter: int = 100000, warm: bool = True):
        assert V.dim() == 2 and V.dtype == torch.float32 and V.stride(1) == 1
        m, p = V.shape
        r = W0.shape[1]
        assert W0.shape == (m, r) and W0.dtype == torch.float32
        dev = V.device
        self.m, self.p, self.r = m, p, r
        self.tol, self.inner_tol, self.max_iter = tol, inner_tol, max_iter
        self.warm = warm
        self.steps_done = 0
        self.V = V
        self.Vt = N.transpose(V)
        self.W = W0.contiguous().clone()
        self.H = torch.empty((r, p), dtype=torch.float32, device=dev)
        self.Ht = torch.empty((p, r), dtype=torch.float32, device=dev)
        self.Wt = torch.empty((r, m), dtype=torch.float32, device=dev)

        def half(d, k):
            f32, f64, i32 = torch.float32, torch.float64, torch.int32

            def ws(op, mode=0):
                return torch.empty(max(N.workspace_bytes(op, d, r, k, mode, N.F32), 1),
                                   dtype=torch.uint8, device=dev)
            return dict(Q=torch.empty((r, r), dtype=f32, device=dev),
                        q=torch.empty((r, k), dtype=f32, device=dev),
                        Y0=torch.empty((r, k), dtype=f32, device=dev),
                        s=torch.empty(r, dtype=f64, device=dev),
                        iters=torch.empty(k, dtype=i32, device=dev),
                        kkt=torch.empty(k, dtype=f64, device=dev),
                        status=torch.empty(k, dtype=i32, device=dev),
                        rows=torch.zeros(k, dtype=torch.int64, device=dev),
                        kkt64=torch.empty(k, dtype=f64, device=dev),
                        obj64=torch.empty(k, dtype=f64, device=dev),
                        ws_p=ws(N.OP_PREPARE, N.GRAM_BF16X3), ws_v=ws(N.OP_SOLVE),
                        ws_r=ws(N.OP_REFINE))
        self.hh = half(m, p)    # H half: d = m, k = p
        self.hw = half(p, m)    # W half: d = p, k = m

    def _solve(self, h, A, B, X, mark):
        N.prepare(A, B, N.GRAM_BF16X3, out=(h["Q"], h["q"], h["s"]), ws=h["ws_p"])
        # after the first step, X holds this half's previous factor: start from it
        warm = self.warm and self.steps_done > 0
        if warm:
            N.rescale_start(h["s"], X, out=h["Y0"])
        mark()
        h["rows"].zero_()
        N.solve(h["Q"], h["q"], h["s"], tol=self.inner_tol, max_iter=self.max_iter,
                Y0=h["Y0"] if warm else None, out=(X, h["iters"], h["kkt"], h["status"]),
                ws=h["ws_v"], rows_read=h["rows"])
        mark()
        N.refine(A, B, X, out=(h["kkt64"], h["obj64"]), ws=h["ws_r"])
        mark()

    def step(self, events=None):
        """One outer step: the H half, then the W half.  Asynchronous on the current stream;
        objective() / stats() read the results.  events (optional, 9 timing events) are recorded
        at the start and after each of: H prepare, solve, check; transpose; W prepare, solve,
        check; transpose."""
        it = iter(events or [])

        def mark():
            e = next(it, None)
            if e is not None:
                e.record()
        mark()
        self._solve(self.hh, self.W, self.V, self.H, mark)
        N.transpose(self.H, out=self.Ht)
        mark()
        self._solve(self.hw, self.Ht, self.Vt, self.Wt, mark)
        N.transpose(self.Wt, out=self.W)
        mark()
        self.steps_done += 1

    def objective(self):
        """(1/2 ||V - W H||^2 after the H half, after the W half), FP64."""
        return float(self.hh["obj64"].sum().item()), float(self.hw["obj64"].sum().item())

    def stats(self):
        out = {}
        for name, h in (("H", self.hh), ("W", self.hw)):
            it = h["iters"]
            out[name] = {"updates_mean": float(it.double().mean().item()),
                         "updates_max": int(it.max().item()),
                         "kkt64_max": float(h["kkt64"].max().item()),
                         "not_converged": int((h["status"] != N.CONVERGED).sum().item()),
                         "rows_read": int(h["rows"].sum().item())}
        return out
