"""The per-update trace of nnls_solve (the record Figures 3 and 4 of Section 5 plot): for every
solver, entry t of a column is r and ||gbar||^2 of the iterate after t updates.  Checked at
t = 0 against the closed form for the cold start (y = 0, gradient q), for the first updates
against an FP64 evaluation at the solver's own iterate (a solve stopped after t updates returns
it), at t = iters against the returned residual, and past the last update for entries left
unwritten.  (The FP32 trajectory itself drifts from the FP64 oracle's within a few updates where
an entry sits on the edge of the passive set, so the iterates are taken from the solver.)"""
import numpy as np
import pytest
import torch

from gpu_common import dev, host, say
from paper_1502_01645_amd import nnls as N

pytestmark = pytest.mark.gpu


def _case(seed, d, n, k):
    rng = np.random.default_rng(seed)
    A = rng.random((d, n)).astype(np.float32)
    X = np.where(rng.random((n, k)) < 0.6, 0.0, rng.random((n, k)))
    B = (A.astype(np.float64) @ X + 0.01 * rng.standard_normal((d, k))).astype(np.float32)
    return A, B


def _r_num(Q, q, y):
    """r(y) and ||gbar||^2 of Algorithm 2's iterate y, in FP64."""
    g = Q @ y + q
    p = np.where((y > 0) | (g < 0), g, 0.0)
    m = np.minimum(y, g)
    qn = np.linalg.norm(q)
    return np.linalg.norm(m) / (qn if qn > 0 else 1.0), float(p @ p)


@pytest.mark.parametrize("solver,n,k", [("wg", 100, 3), ("mrhs", 96, 20), ("regq", 2000, 1),
                                        ("persistent", 2000, 1)])
def test_trace_records_every_update(solver, n, k, monkeypatch):
    monkeypatch.setenv("NNLS_SOLVER", solver)
    assert N.solver_name(n, k) == solver
    A, B = _case(90 + n, 3 * n, n, k)
    Q, q, s = N.prepare(dev(A), dev(B))
    T = 400
    trace = torch.full((k, T, 2), float("nan"), dtype=torch.float32, device="cuda")
    X, it, kkt, st = N.solve(Q, q, s, tol=1e-5, max_iter=T - 1, trace=trace)
    tr, it, kkt, st = host(trace), host(it), host(kkt), host(st)
    Qh, qh = host(Q).astype(np.float64), host(q).astype(np.float64)
    say(f"{solver} n={n} k={k}: updates {it.tolist()[:8]}")
    assert np.all(st == N.CONVERGED)
    for c in range(k):
        m = int(it[c])
        assert m >= 3
        # written for t <= m, untouched after
        assert np.all(np.isfinite(tr[c, :m + 1]))
        assert np.all(np.isnan(tr[c, m + 1:]))
        # the last entry is the returned (exactly recomputed) residual
        assert tr[c, m, 0] == np.float32(kkt[c])
        # t = 0: y = 0, gradient q: r = ||min(q, 0)|| / ||q||, gbar = q on {q < 0}
        qc = qh[:, c]
        r0 = np.linalg.norm(np.minimum(qc, 0.0)) / np.linalg.norm(qc)
        np.testing.assert_allclose(tr[c, 0], [r0, np.sum(np.minimum(qc, 0.0) ** 2)], rtol=1e-5)
    # first updates: FP64 evaluation at the iterate after t updates
    for t in range(1, 5):
        tr_t = torch.full((k, T, 2), float("nan"), dtype=torch.float32, device="cuda")
        Yt, it_t, _, _ = N.solve(Q, q, None, tol=1e-5, max_iter=t, trace=tr_t)
        Yt, it_t, tr_t = host(Yt).astype(np.float64), host(it_t), host(tr_t)
        for c in range(k):
            if t > int(it[c]):
                continue
            assert it_t[c] == t
            want = _r_num(Qh, qh[:, c], Yt[:, c])
            # the stopped solve recomputed the gradient at t; the long one carried it
            np.testing.assert_allclose(tr_t[c, t], want, rtol=1e-4)
            np.testing.assert_allclose(tr[c, t], want, rtol=1e-3)
