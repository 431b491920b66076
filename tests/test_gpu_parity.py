"""HIP path against the FP64 oracle, element by element where the result is unique.

Every call goes through the C ABI (paper_1502_01645_amd.nnls is only ctypes marshalling).
Sizes span several 128-wide Gram tiles with ragged tails; the end-to-end cases check the
method's own tolerances: relative KKT residual in FP64 against the original data (the metric
the oracle computes) and the relative objective gap against the oracle's tight solution.
"""
import numpy as np
import pytest
import torch

from gpu_common import DEV, dev, gram_abs_tol, host, orc, say
from oracle import oracle as O
from paper_1502_01645_amd import nnls as N
from paper_1502_01645_amd import workloads as W

pytestmark = pytest.mark.gpu


def _uniform_case(seed, d, n, k, dtype=np.float32):
    rng = np.random.default_rng(seed)
    A = rng.random((d, n)).astype(dtype)
    X = np.where(rng.random((n, k)) < 0.6, 0.0, rng.random((n, k)))
    B = (A.astype(np.float64) @ X + 0.01 * rng.standard_normal((d, k))).astype(dtype)
    return A, B


# ---------------------------------------------------------------------------- prepare ---------
@pytest.mark.parametrize("d,n,k", [(300, 300, 3), (1000, 130, 1), (257, 129, 0), (64, 5, 2),
                                   (1, 7, 1), (513, 384, 130)])
@pytest.mark.parametrize("mode", ["bf16x3", "fp32"])
def test_prepare_fp32_parity(d, n, k, mode):
    say(f"prepare {mode} d={d} n={n} k={k}")
    rng = np.random.default_rng(d * 7 + n)
    A = (rng.standard_normal((d, n)) * rng.random(n)[None, :] * 3).astype(np.float32)
    B = rng.standard_normal((d, k)).astype(np.float32) if k else None
    m = N.GRAM_BF16X3 if mode == "bf16x3" else N.GRAM_FP32
    Q, q, s = N.prepare(dev(A), dev(B) if k else None, mode=m)
    s_o, Q_o, q_o = orc().prepare(A, B if k else np.zeros((d, 0)))
    tol = gram_abs_tol(d, mode)
    assert np.allclose(host(s), s_o, rtol=1e-12, atol=0)
    Qh = host(Q).astype(np.float64)
    assert np.abs(Qh - Q_o).max() <= tol
    assert np.array_equal(Qh, Qh.T)
    assert np.all(np.diag(Qh) == 1.0)
    if k:
        bn = np.linalg.norm(B.astype(np.float64), axis=0)
        err = np.abs(host(q).astype(np.float64) - q_o) / bn[None, :]
        assert err.max() <= tol


def test_prepare_splitk_parity():
    d, n, k = 20000, 100, 20
    say(f"prepare split-K d={d} n={n} k={k}")
    rng = np.random.default_rng(3)
    A = np.abs(rng.standard_normal((d, n))).astype(np.float32)
    B = rng.random((d, k)).astype(np.float32)
    Q, q, s = N.prepare(dev(A), dev(B))
    s_o, Q_o, q_o = orc().prepare(A, B)
    tol = gram_abs_tol(d, "bf16x3")
    assert np.abs(host(Q) - Q_o).max() <= tol
    bn = np.linalg.norm(B.astype(np.float64), axis=0)
    assert (np.abs(host(q) - q_o) / bn[None, :]).max() <= tol


@pytest.mark.parametrize("d,n,k", [(1000, 130, 1), (513, 384, 130)])
def test_split_calls_match_prepare(d, n, k):
    """nnls_column_scales + nnls_gram_rescaled (s computed by its own pass, then given to the
    Gram) against the one-call nnls_prepare (s formed inside the operand split): the same s to
    rounding, and Q, q within the BF16x3 bound of the oracle."""
    say(f"split calls d={d} n={n} k={k}")
    A, B = _uniform_case(d + n, d, n, k)
    Q1, q1, s1 = N.prepare(dev(A), dev(B))
    s2 = N.column_scales(dev(A))
    Q2, q2 = N.gram_rescaled(dev(A), dev(B), s2)
    s_o, Q_o, q_o = orc().prepare(A, B)
    assert np.allclose(host(s1), s_o, rtol=1e-13, atol=0)
    assert np.allclose(host(s2), s_o, rtol=1e-13, atol=0)
    tol = gram_abs_tol(d, "bf16x3")
    for Q, q in ((Q1, q1), (Q2, q2)):
        Qh = host(Q).astype(np.float64)
        assert np.abs(Qh - Q_o).max() <= tol
        assert np.array_equal(Qh, Qh.T)
        bn = np.linalg.norm(B.astype(np.float64), axis=0)
        assert (np.abs(host(q).astype(np.float64) - q_o) / bn[None, :]).max() <= tol


def test_prepare_fp64_parity():
    A, b, _ = W.make_small()
    say("prepare fp64 200x50")
    Q, q, s = N.prepare(dev(A), dev(b))
    s_o, Q_o, q_o = orc().prepare(A, b)
    assert np.allclose(host(s), s_o, rtol=1e-14)
    assert np.abs(host(Q) - Q_o).max() <= 1e-13
    assert np.allclose(host(q), q_o, rtol=1e-12, atol=1e-12 * np.abs(q_o).max())


def test_prepare_zero_column():
    say("prepare zero column")
    A, B = _uniform_case(5, 300, 140, 2)
    A[:, 17] = 0.0
    Q, q, s = N.prepare(dev(A), dev(B))
    Qh, qh, sh = host(Q), host(q), host(s)
    assert sh[17] == 1.0 and np.all(Qh[17, :] == 0) and np.all(Qh[:, 17] == 0)
    assert np.all(qh[17] == 0)


# ---------------------------------------------------------------------------- solve -----------
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_solve_steps_match_oracle(dtype):
    """One update of Algorithm 2 from the same state, element by element: starting from the
    oracle's iterate y_m (m = 0, 1, 2, 5, 20), one GPU update must land on the oracle's y_{m+1}.
    Starting every comparison from the oracle's state keeps rounding differences from
    compounding over iterations of an ill-conditioned problem."""
    say(f"solve single steps {np.dtype(dtype).name}")
    A, B = _uniform_case(11, 400, 300, 4, dtype)
    Q, q, s = N.prepare(dev(A), dev(B))
    Qh, qh = host(Q).astype(np.float64), host(q).astype(np.float64)
    n, k = qh.shape
    eps = 2.0 ** -52 if dtype == np.float64 else 2.0 ** -23
    for m in [0, 1, 2, 5, 20]:
        Ym = np.zeros((n, k))
        Yn = np.zeros((n, k))
        for c in range(k):
            Ym[:, c] = orc().nqp(Qh, qh[:, c], 0.0, m)[0] if m else 0.0
        Ym_dev = dev(Ym.astype(dtype)) if m else None
        # the state handed to the GPU is y_m rounded to the working type; the oracle continues
        # from that same rounded state
        Ystart = Ym.astype(dtype).astype(np.float64)
        for c in range(k):
            Yn[:, c] = orc().nqp(Qh, qh[:, c], 0.0, 1, y0=Ystart[:, c])[0]
        Y, iters, kkt, st = N.solve(Q, q, None, tol=0.0, max_iter=1, Y0=Ym_dev)
        Yh = host(Y).astype(np.float64)
        assert np.all(host(iters) == 1)
        for c in range(k):
            err = np.abs(Yh[:, c] - Yn[:, c]).max()
            scale = np.abs(Ystart[:, c]).max() + np.abs(Yn[:, c]).max()
            # one update: gradient over n terms, two reductions over n terms, one multiply-add;
            # allow 8 n eps relative to the size of the iterates
            assert err <= 8 * n * eps * scale, (m, c, err / scale)


def _check_solution(A, B, X, tol, ref, what):
    r, F = orc().kkt_x(A, B, X)
    gap = O.relative_gap(F, ref)
    say(f"{what}: max r={r.max():.3e} max gap={gap.max():.3e}")
    assert np.all(X >= 0)
    assert r.max() <= tol, r.max()
    assert gap.max() <= 1e-6, gap.max()
    return r, gap


def test_end_to_end_small_fp64():
    """The 200 x 50 FP64 instance, tolerance 1e-8 (the small plain-method workload)."""
    A, b, _ = W.make_small()
    say("e2e small fp64")
    res = N.nnls(dev(A), dev(b), tol=1e-8, max_iter=100000, inner_tol=5e-9)
    st = host(res["status"])
    assert st[0] == N.CONVERGED
    ref = O.reference_solution(A, b)
    X = host(res["X"])
    _check_solution(A, b, X, 1e-8, ref, "small fp64")
    r_o, _ = orc().kkt_x(A, b, X)
    assert abs(host(res["kkt64"])[0] - r_o[0]) <= 1e-6 * r_o[0] + 1e-15


@pytest.mark.parametrize("d,n,k,seed", [(2000, 500, 1, 1), (3000, 700, 2, 2), (1500, 257, 6, 3)])
def test_end_to_end_fp32(d, n, k, seed):
    say(f"e2e fp32 d={d} n={n} k={k}")
    A, B = _uniform_case(seed, d, n, k)
    res = N.nnls(dev(A), dev(B), tol=1e-5, max_iter=100000, inner_tol=3e-6)
    assert np.all(host(res["status"]) == N.CONVERGED)
    ref = O.reference_solution(A, B)
    X = host(res["X"])
    r, _ = _check_solution(A, B, X, 1e-5, ref, "fp32")
    assert np.allclose(host(res["kkt64"]), r, rtol=1e-6, atol=1e-14)


def test_many_rhs_small():
    """Scaled-down many-RHS workload (|N(0,1)| dictionary, Gamma(2,1) codes, 1 % noise)."""
    A, B, _ = W.make_manyrhs(seed=4, d=2000, n=96, k=37)
    say("many-rhs small")
    res = N.nnls(dev(A), dev(B), tol=1e-5, max_iter=100000, inner_tol=3e-6)
    assert np.all(host(res["status"]) == N.CONVERGED)
    ref = O.reference_solution(A, B)
    _check_solution(A, B, host(res["X"]), 1e-5, ref, "many-rhs")


# (700, 130, 70) and (2100, 64, 40) split the FP64 product over K (2 and 8 ways)
@pytest.mark.parametrize("dtype,d,n,k", [(np.float32, 700, 130, 70), (np.float64, 500, 67, 9),
                                         (np.float32, 300, 256, 5), (np.float32, 2100, 64, 40)])
@pytest.mark.parametrize("start", ["loose", "zero"])
def test_refine_many_rhs_matches_oracle(dtype, d, n, k, start):
    """FP64 check and refinement step for more than four right-hand sides (the FP64 Gram path):
    reported residual and objective are the oracle's for the returned X, and a column's step is
    kept exactly where the FP64 step lowers the residual without raising the objective."""
    say(f"refine many rhs {np.dtype(dtype).name} d={d} n={n} k={k} start={start}")
    _refine_case(dtype, d, n, k, start)


# one right-hand side with FP32 A, 16-byte rows and n <= 6144 takes the fused row/column pass
# (one, two or three 2048-column blocks; ragged and tiny d); n % 4 != 0, k > 1 and FP64 A take the
# two-pass form
@pytest.mark.parametrize("dtype,d,n,k", [(np.float32, 700, 132, 1), (np.float32, 1001, 2052, 1),
                                         (np.float32, 523, 4100, 1), (np.float32, 5, 5000, 1),
                                         (np.float32, 1500, 6144, 1), (np.float32, 600, 130, 1),
                                         (np.float32, 800, 300, 2), (np.float64, 400, 96, 1)])
@pytest.mark.parametrize("start", ["loose", "zero"])
def test_refine_few_rhs_matches_oracle(dtype, d, n, k, start):
    """FP64 check and refinement step for one to four right-hand sides (passes over A): the same
    bar as the many right-hand-side path."""
    say(f"refine few rhs {np.dtype(dtype).name} d={d} n={n} k={k} start={start}")
    _refine_case(dtype, d, n, k, start)


@pytest.mark.parametrize("d,n,k", [(2000, 300, 1), (3000, 700, 5), (500, 1100, 0)])
def test_prepare_split_then_product_equals_prepare(d, n, k):
    """nnls_prepare_split followed by nnls_prepare_product on one workspace gives nnls_prepare's
    Q, q and s bit for bit (they are its two launches)."""
    say(f"split + product d={d} n={n} k={k}")
    rng = np.random.default_rng(d + n)
    A = dev(rng.random((d, n)).astype(np.float32))
    B = dev(rng.random((d, max(k, 1))).astype(np.float32))[:, :k].contiguous() if k else \
        torch.zeros((d, 0), dtype=torch.float32, device=DEV)
    Q0, q0, s0 = N.prepare(A, B if k else None)
    wsb = N.workspace_bytes(N.OP_PREPARE, d, n, k, N.GRAM_BF16X3, N.F32)
    ws = torch.empty(wsb, dtype=torch.uint8, device=DEV)
    s = torch.empty(n, dtype=torch.float64, device=DEV)
    Q = torch.empty((n, n), dtype=torch.float32, device=DEV)
    q = torch.empty((n, k), dtype=torch.float32, device=DEV)
    N.prepare_split(A, B, s, ws)
    N.prepare_product(d, s, Q, q, ws)
    np.testing.assert_array_equal(host(s), host(s0))
    np.testing.assert_array_equal(host(Q), host(Q0))
    if k:
        np.testing.assert_array_equal(host(q), host(q0))


@pytest.mark.parametrize("d,n,k", [(600, 96, 3), (900, 160, 40), (1100, 256, 70)])
def test_refine_objective_noiseless(d, n, k):
    """Noiseless data b = A x*: F* = 0 and F at the returned x is tiny against 1/2 ||b||^2, so
    the reported objective must come from the residuals.  Checked relative to F itself (the
    Gram form 1/2 (x^T H x - 2 a^T x + ||b||^2) would be off by about eps ||b||^2 here, many
    times F), once after a solve and once at x* itself, where F is only the FP32 rounding of b;
    obj64 = NULL leaves the check and step unchanged."""
    say(f"refine noiseless objective d={d} n={n} k={k}")
    rng = np.random.default_rng(71 + k)
    A = rng.random((d, n)).astype(np.float32)
    Xt = np.where(rng.random((n, k)) < 0.5, 0.0, rng.random((n, k))).astype(np.float32)
    B = (A.astype(np.float64) @ Xt.astype(np.float64)).astype(np.float32)
    bb = 0.5 * (B.astype(np.float64) ** 2).sum(0)
    res = N.nnls(dev(A), dev(B), tol=1e-5, max_iter=100000, inner_tol=3e-6)
    X1 = host(res["X"])
    _, F1 = orc().kkt_x(A, B, X1)
    obj = host(res["obj64"])
    say(f"  after solve: F/(||b||^2/2) max {(F1 / bb).max():.2e}, "
        f"max |obj - F|/F {np.max(np.abs(obj - F1) / F1):.2e}")
    assert np.all(F1 < 1e-6 * bb)
    np.testing.assert_allclose(obj, F1, rtol=1e-6, atol=0)
    # at x* itself
    X = dev(Xt)
    kkt64, obj64 = N.refine(dev(A), dev(B), X)
    Xr = host(X)
    r2, F2 = orc().kkt_x(A, B, Xr)
    say(f"  at x*: F/(||b||^2/2) max {(F2 / bb).max():.2e}, "
        f"max |obj - F|/F {np.max(np.abs(host(obj64) - F2) / F2):.2e}")
    np.testing.assert_allclose(host(obj64), F2, rtol=1e-5, atol=0)
    np.testing.assert_allclose(host(kkt64), r2, rtol=1e-6, atol=1e-14)
    # without the objective: same X and residual
    X = dev(Xt)
    kkt_b, obj_b = N.refine(dev(A), dev(B), X, objective=False)
    assert obj_b is None
    np.testing.assert_array_equal(host(X), Xr)
    np.testing.assert_array_equal(host(kkt_b), host(kkt64))


def _refine_case(dtype, d, n, k, start):
    A, B = _uniform_case(31 + k, d, n, k, dtype)
    Q, q, s = N.prepare(dev(A), dev(B))
    if start == "loose":
        X, it, kkt, st = N.solve(Q, q, s, tol=1e-3, max_iter=0)
    else:
        X = torch.zeros_like(q)
    X0 = host(X).copy()
    kkt64, obj64 = N.refine(dev(A), dev(B), X)
    X1 = host(X)
    r0, F0 = orc().kkt_x(A, B, X0)
    r1, F1 = orc().kkt_x(A, B, X1)
    np.testing.assert_allclose(host(kkt64), r1, rtol=1e-6, atol=1e-14)
    bb = 0.5 * (B.astype(np.float64) ** 2).sum(0)
    assert np.all(np.abs(host(obj64) - F1) <= 1e-10 * bb)
    Xc = O.refine_candidate(A, B, X0, dtype)
    rc, Fc = orc().kkt_x(A, B, Xc)
    want = (rc < r0) & (Fc <= F0)
    clear = (np.abs(rc - r0) > 1e-6 * r0) & (np.abs(Fc - F0) > 1e-12 * bb)
    changed = np.any(X1 != X0, axis=0)
    say(f"  steps kept {int(changed.sum())} of {k}; expected {int(want.sum())}")
    assert np.array_equal(changed[clear], want[clear])
    if start == "zero":
        assert changed.any()
    np.testing.assert_allclose(X1[:, changed], Xc[:, changed], rtol=1e-6,
                               atol=1e-6 * max(np.abs(Xc).max(), 1e-30))
    assert np.all(r1 <= r0 * (1 + 1e-6))
    assert np.all(X1 >= 0)


# ---------------------------------------------------------------------------- edge cases ------
def test_n_equals_one():
    say("n = 1")
    rng = np.random.default_rng(8)
    A = (rng.random((50, 1)) + 0.1).astype(np.float64)
    b = rng.standard_normal((50, 3))
    b[:, 1] = -np.abs(b[:, 1]) - 1  # a^T b < 0: x = 0
    res = N.nnls(dev(A), dev(b), tol=1e-12, max_iter=10)
    X = host(res["X"])
    x_cf = np.maximum(0.0, A[:, 0] @ b) / (A[:, 0] @ A[:, 0])
    assert np.allclose(X[0], x_cf, rtol=1e-12, atol=1e-14)
    its = host(res["iters"])
    assert list(its) == [1 if v > 0 else 0 for v in x_cf]


def test_nonnegative_q_gives_zero():
    say("q >= 0")
    rng = np.random.default_rng(9)
    A = rng.random((100, 40)).astype(np.float32)
    b = -rng.random((100, 1)).astype(np.float32)
    res = N.nnls(dev(A), dev(b), tol=1e-6)
    assert np.all(host(res["X"]) == 0) and host(res["iters"])[0] == 0
    assert host(res["status"])[0] == N.CONVERGED


def test_status_maxiter_and_nonfinite():
    say("statuses")
    A, B = _uniform_case(12, 300, 200, 2)
    Q, q, s = N.prepare(dev(A), dev(B))
    X, it, kkt, st = N.solve(Q, q, s, tol=1e-12, max_iter=3)
    assert np.all(host(st) == N.MAXITER) and np.all(host(it) == 3)
    qb = q.clone()
    qb[5, 1] = float("nan")
    X, it, kkt, st = N.solve(Q, qb, s, tol=1e-6, max_iter=50)
    sth = host(st)
    assert sth[1] == N.NONFINITE and sth[0] != N.NONFINITE


def test_breakdown_on_indefinite_q():
    say("breakdown")
    Q = torch.tensor([[1.0, 0.0], [0.0, -1.0]], dtype=torch.float64, device=DEV)
    q = torch.tensor([[0.0], [-1.0]], dtype=torch.float64, device=DEV)
    X, it, kkt, st = N.solve(Q, q, None, tol=1e-10, max_iter=50)
    assert host(st)[0] == N.BREAKDOWN


def test_warm_start_at_solution():
    """Y0 = the converged y: the solve stops at once with the same point."""
    say("warm start at solution")
    A, B = _uniform_case(13, 800, 150, 3)
    Q, q, s = N.prepare(dev(A), dev(B))
    Y, it, kkt, st = N.solve(Q, q, None, tol=1e-6, max_iter=100000)
    Y2, it2, kkt2, st2 = N.solve(Q, q, None, tol=1e-6, max_iter=100000, Y0=Y)
    assert np.all(host(it2) == 0) and np.all(host(st2) == N.CONVERGED)
    assert np.array_equal(host(Y2), host(Y))


# ---------------------------------------------------------------------------- whole-GPU solvers
# "regq" keeps Q in the register file of the whole GPU (n <= 5120), "persistent" streams it.
@pytest.fixture(params=["regq", "persistent"])
def whole_gpu(request, monkeypatch):
    monkeypatch.setenv("NNLS_SOLVER", request.param)
    yield request.param
    monkeypatch.delenv("NNLS_SOLVER", raising=False)


@pytest.mark.parametrize("n", [512, 1024, 2000, 2500, 4000, 5000, 5120])
def test_persistent_steps_match_oracle(n, whole_gpu):
    """Whole-GPU solvers, one update from the oracle's state (as for the per-column solver).
    The sizes cover every register shape of the register-resident solver (n <= 2048, 3072,
    4096, 5120) and its largest n."""
    say(f"{whole_gpu} single steps n={n}")
    A, B = _uniform_case(21, 2 * n, n, 1)
    Q, q, s = N.prepare(dev(A), dev(B))
    Qh, qh = host(Q).astype(np.float64), host(q).astype(np.float64)[:, 0]
    eps = 2.0 ** -23
    for m in [0, 1, 2, 5, 20]:
        ym = orc().nqp(Qh, qh, 0.0, m)[0] if m else np.zeros(n)
        ystart = ym.astype(np.float32).astype(np.float64)
        yn = orc().nqp(Qh, qh, 0.0, 1, y0=ystart)[0]
        Y, iters, kkt, st = N.solve(Q, q, None, tol=0.0, max_iter=1,
                                    Y0=dev(ym.astype(np.float32).reshape(n, 1)) if m else None)
        Yh = host(Y)[:, 0].astype(np.float64)
        assert host(iters)[0] == 1
        err = np.abs(Yh - yn).max()
        scale = np.abs(ystart).max() + np.abs(yn).max()
        assert err <= 8 * n * eps * scale, (m, err / scale)


@pytest.mark.parametrize("d,n,seed", [(1500, 512, 4), (6000, 2000, 5), (9000, 3072, 6),
                                      (12000, 4100, 7)])
def test_persistent_end_to_end(d, n, seed, whole_gpu):
    """Large single right-hand sides (n >= 1536 takes a whole-GPU solver by default)."""
    say(f"{whole_gpu} e2e d={d} n={n}")
    A, b, _ = W.make_large(seed=seed, d=d, n=n)
    res = N.nnls(dev(A), dev(b), tol=1e-5, max_iter=100000, inner_tol=3e-6)
    assert host(res["status"])[0] == N.CONVERGED
    ref = O.reference_solution(A, b)
    _check_solution(A, b, host(res["X"]), 1e-5, ref, f"{whole_gpu} n={n}")


def test_persistent_statuses(whole_gpu):
    say(f"{whole_gpu} statuses")
    A, B = _uniform_case(22, 3000, 1024, 1)
    Q, q, s = N.prepare(dev(A), dev(B))
    X, it, kkt, st = N.solve(Q, q, s, tol=1e-12, max_iter=4)
    assert host(st)[0] == N.MAXITER and host(it)[0] == 4
    Y, it, kkt, st = N.solve(Q, q, None, tol=1e-6, max_iter=100000)
    assert host(st)[0] == N.CONVERGED
    Y2, it2, kkt2, st2 = N.solve(Q, q, None, tol=1e-6, max_iter=100000, Y0=Y)
    assert host(it2)[0] == 0 and host(st2)[0] == N.CONVERGED
    assert np.array_equal(host(Y2), host(Y))
    qb = q.clone()
    qb[7, 0] = float("nan")
    X, it, kkt, st = N.solve(Q, qb, s, tol=1e-6, max_iter=50)
    assert host(st)[0] == N.NONFINITE
    qp = q.abs()
    X, it, kkt, st = N.solve(Q, qp, s, tol=1e-6, max_iter=50)
    assert host(st)[0] == N.CONVERGED and host(it)[0] == 0 and np.all(host(X) == 0)


def test_whole_gpu_give_up_ends_every_wait(whole_gpu, monkeypatch):
    """A poll limit of 0, forced from the host: the first workgroup that does not find the
    others ready gives up and sets the abort word, every other workgroup leaves its wait at its
    next check, and the launch ends normally with BREAKDOWN, iters = -1 and a NaN residual.  A
    solve with the normal limit on the same workspace afterwards is unaffected."""
    say(f"{whole_gpu} forced give-up")
    A, b, _ = W.make_large(seed=9, d=3000, n=1600)
    n = A.shape[1]
    Q, q, s = N.prepare(dev(A), dev(b))
    ws = torch.empty(N.workspace_bytes(N.OP_SOLVE, 0, n, 1, 0, N.F32), dtype=torch.uint8,
                     device=DEV)
    X0, it0, kkt0, st0 = N.solve(Q, q, s, tol=1e-5, max_iter=100000, ws=ws)
    monkeypatch.setenv("NNLS_SPIN_LIMIT", "0")
    X, it, kkt, st = N.solve(Q, q, s, tol=1e-5, max_iter=100000, ws=ws)
    assert host(st)[0] == N.BREAKDOWN and host(it)[0] == -1 and np.isnan(host(kkt)[0])
    monkeypatch.delenv("NNLS_SPIN_LIMIT")
    X1, it1, kkt1, st1 = N.solve(Q, q, s, tol=1e-5, max_iter=100000, ws=ws)
    assert host(st1)[0] == N.CONVERGED and host(it1)[0] == host(it0)[0]
    np.testing.assert_array_equal(host(X1), host(X0))


def test_whole_gpu_solve_is_bitwise_reproducible(whole_gpu):
    """The exchanges between workgroups fix the order of every sum (partials added in workgroup
    order, whichever workgroup publishes first), so the full-size large single right-hand-side
    workload (20000 x 5000) prepared and solved twice gives bitwise the same Q, X, iteration
    count and residual."""
    say(f"{whole_gpu} reproducible 20000x5000")
    A, b, _ = W.make_large()
    Ad, bd = dev(A), dev(b)
    runs = []
    for _ in range(3):
        Q, q, s = N.prepare(Ad, bd)
        X, it, kkt, st = N.solve(Q, q, s, tol=8e-6, max_iter=25000)
        runs.append((host(Q), host(X), int(host(it)[0]), float(host(kkt)[0]), int(host(st)[0])))
    say(f"  iters {[r[2] for r in runs]} kkt {[r[3] for r in runs]}")
    assert runs[0][4] == N.CONVERGED
    for r in runs[1:]:
        np.testing.assert_array_equal(r[0], runs[0][0])
        np.testing.assert_array_equal(r[1], runs[0][1])
        assert r[2:] == runs[0][2:]


def test_regq_rows_read_counts_passive_and_clipped(monkeypatch):
    """The register solver reports the rows a streaming solver reads (|P| + |C| per update plus
    n per exact refresh): the same count as the streaming solver on the same problem."""
    A, b, _ = W.make_large(seed=8, d=3000, n=1600)
    Q, q, s = N.prepare(dev(A), dev(b))
    counts = {}
    for solver in ["regq", "persistent"]:
        monkeypatch.setenv("NNLS_SOLVER", solver)
        rows = torch.zeros(1, dtype=torch.int64, device=DEV)
        X, it, kkt, st = N.solve(Q, q, s, tol=1e-5, max_iter=5, rows_read=rows)
        counts[solver] = (int(host(rows)[0]), int(host(it)[0]))
    monkeypatch.delenv("NNLS_SOLVER", raising=False)
    say(f"rows read {counts}")
    assert counts["regq"][1] == counts["persistent"][1] == 5
    assert abs(counts["regq"][0] - counts["persistent"][0]) <= 0.02 * counts["persistent"][0]


# ---------------------------------------------------------------------------- many-RHS solver
@pytest.mark.parametrize("solver", ["mrhs", "wg"])
@pytest.mark.parametrize("n,k", [(96, 20), (100, 33)])
def test_multi_rhs_steps_match_oracle(solver, n, k, monkeypatch):
    """Matrix-core many-RHS solver (and the per-column solver) against the oracle, one update
    from the oracle's state per column, for several column slots and a padded n."""
    monkeypatch.setenv("NNLS_SOLVER", solver)
    say(f"{solver} single steps n={n} k={k}")
    A, B = _uniform_case(31 + n, 3 * n, n, k)
    Q, q, s = N.prepare(dev(A), dev(B))
    Qh, qh = host(Q).astype(np.float64), host(q).astype(np.float64)
    eps = 2.0 ** -23
    for m in [0, 1, 3, 10]:
        Ym = np.zeros((n, k))
        if m:
            for c in range(k):
                Ym[:, c] = orc().nqp(Qh, qh[:, c], 0.0, m)[0]
        Ystart = Ym.astype(np.float32).astype(np.float64)
        Y, iters, kkt, st = N.solve(Q, q, None, tol=0.0, max_iter=1,
                                    Y0=dev(Ym.astype(np.float32)) if m else None)
        Yh = host(Y).astype(np.float64)
        assert np.all(host(iters) == 1)
        for c in range(k):
            yn = orc().nqp(Qh, qh[:, c], 0.0, 1, y0=Ystart[:, c])[0]
            err = np.abs(Yh[:, c] - yn).max()
            scale = np.abs(Ystart[:, c]).max() + np.abs(yn).max()
            assert err <= 8 * n * eps * scale, (m, c, err / scale)


def test_multi_rhs_end_to_end():
    """Many-RHS workload recipe at reduced size; every column meets the tolerances."""
    A, B, _ = W.make_manyrhs(seed=6, d=3000, n=128, k=300)
    say("mrhs e2e 3000x128 k=300")
    res = N.nnls(dev(A), dev(B), tol=1e-5, max_iter=100000, inner_tol=3e-6)
    assert np.all(host(res["status"]) == N.CONVERGED)
    ref = O.reference_solution(A, B)
    _check_solution(A, B, host(res["X"]), 1e-5, ref, "mrhs")


def test_multi_rhs_queue_refill():
    """More columns than resident slots: finished slots take new columns from the queue."""
    rng = np.random.default_rng(41)
    d, n, k = 40, 8, 12000
    A = rng.random((d, n)).astype(np.float32)
    X = np.where(rng.random((n, k)) < 0.5, 0.0, rng.random((n, k)))
    B = (A.astype(np.float64) @ X + 0.01 * rng.standard_normal((d, k))).astype(np.float32)
    say("mrhs queue refill k=12000")
    res = N.nnls(dev(A), dev(B), tol=1e-5, max_iter=100000, inner_tol=3e-6)
    assert np.all(host(res["status"]) == N.CONVERGED)
    r, F = orc().kkt_x(A, B, host(res["X"]))
    assert r.max() <= 1e-5
    assert np.all(host(res["iters"]) >= 0)
