"""Checks that pin the FP64 oracle to facts fixed by the paper and by mathematics, independent of
the oracle's own code.  Each function takes an Oracle handle and raises AssertionError on a
mismatch, so the same checks can also be run against deliberately broken builds.

Sources of truth used here (never the oracle itself):
  - the worked example of equation (3) and Figures 1-2 (tests/golden/eq3_example.json);
  - closed forms: n = 1 (exact line search of Algorithm 2 in one variable), orthogonal columns
    (Q = I, one exact step), q >= 0 (empty passive set);
  - brute-force enumeration of all 2^n supports with numpy least squares, for tiny n;
  - scipy's Lawson-Hanson NNLS (the classical active-set method the paper cites);
  - numpy's matrix product for the Gram of Problem (2);
  - the Remark and Lemma of Sections 3-4 (unit diagonal, cosines, sqrt(n) <= ||Q||_F <= n);
  - invariances of the problem: column scaling, column permutation, positive homogeneity in b.
"""
from __future__ import annotations

import itertools
import json
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _rng(seed):
    return np.random.default_rng(seed)


def brute_force_nnls(A, b):
    """Exact NNLS by enumerating every support S: least squares on S, kept when feasible and the
    KKT conditions hold (gradient >= 0 off S).  Exponential; tiny n only."""
    d, n = A.shape
    best = None
    for mask in itertools.product([0, 1], repeat=n):
        S = [i for i in range(n) if mask[i]]
        x = np.zeros(n)
        if S:
            xs, *_ = np.linalg.lstsq(A[:, S], b, rcond=None)
            if np.any(xs < 0):
                continue
            x[S] = xs
        g = A.T @ (A @ x - b)
        scale = max(1.0, np.abs(A.T @ b).max())
        off = [i for i in range(n) if not mask[i]]
        if off and np.min(g[off]) < -1e-9 * scale:
            continue
        F = 0.5 * np.sum((A @ x - b) ** 2)
        if best is None or F < best[1]:
            best = (x, F)
    return best


def pin_eq3_example(orc):
    """Equation (3) from x0 = [30, 2]: the unscaled method creeps (Figure 1, 40 steps to the
    optimum); after the rescale the same method is there in about 3 steps (Figure 2)."""
    with open(os.path.join(GOLDEN, "eq3_example.json")) as f:
        ex = json.load(f)
    H = np.array(ex["H"])
    h = np.array(ex["h"])
    x0 = np.array(ex["x0"])
    xs = np.array(ex["x_star_numerators"]) / ex["x_star_denominator"]
    # closed form of the unconstrained (and feasible) minimiser, independent of the oracle
    assert np.allclose(H @ xs, -h, rtol=0, atol=1e-13)

    def err_unscaled(m):
        y, it, _, _ = orc.nqp(H, h, 0.0, m, y0=x0)
        return np.linalg.norm(y - xs) / np.linalg.norm(xs), it

    n_un = ex["steps_unscaled"]
    e40, it40 = err_unscaled(n_un)
    assert it40 == n_un
    assert e40 < 1e-15, e40                    # at the optimum to machine precision by step 40
    e20, _ = err_unscaled(n_un // 2)
    assert e20 > 1e-10, e20                    # ... and clearly not there at half the steps
    e3u, _ = err_unscaled(ex["steps_rescaled"])
    assert e3u > 0.1, e3u

    s, Q, q = orc.rescale(H, h.reshape(2, 1))
    assert np.allclose(s, np.sqrt(np.diag(H)), rtol=1e-15)
    y, it, _, _ = orc.nqp(Q, q[:, 0], 0.0, ex["steps_rescaled"], y0=x0 * s)
    e3 = np.linalg.norm(y / s - xs) / np.linalg.norm(xs)
    assert e3 < 1e-4, e3                       # 3 rescaled steps: at plot resolution, the optimum
    y, it, _, _ = orc.nqp(Q, q[:, 0], 0.0, 12, y0=x0 * s)
    assert np.linalg.norm(y / s - xs) / np.linalg.norm(xs) < 1e-14


def pin_n1_closed_form(orc):
    """n = 1: f(y) = y^2/2 + q y on y >= 0, minimised at max(0, -q); one exact step if q < 0."""
    rng = _rng(11)
    for trial in range(20):
        d = int(rng.integers(1, 9))
        a = rng.random((d, 1)) + 0.1
        b = rng.standard_normal((d, 1))
        out = orc.nnls(a, b, 1e-14, 100)
        x_cf = max(0.0, float(a[:, 0] @ b[:, 0])) / float(a[:, 0] @ a[:, 0])
        assert abs(out["X"][0, 0] - x_cf) <= 1e-13 * max(1.0, abs(x_cf))
        assert out["iters"][0] == (1 if x_cf > 0 else 0)


def pin_orthogonal_columns(orc):
    """Orthogonal columns give Q = I, so the first exact step lands on the clipped least-squares
    solution x_i = max(0, A_i^T b) / ||A_i||^2 and the solve ends after one update."""
    rng = _rng(12)
    for trial in range(5):
        d, n = 40, 12
        U, _ = np.linalg.qr(rng.standard_normal((d, n)))
        A = U * (rng.random(n) * 5 + 0.5)[None, :]
        b = rng.standard_normal((d, 1))
        out = orc.nnls(A, b, 1e-12, 100)
        x_ls = np.maximum(0.0, A.T @ b[:, 0]) / np.sum(A * A, axis=0)
        assert np.allclose(out["X"][:, 0], x_ls, rtol=1e-10, atol=1e-12)
        assert out["iters"][0] == 1


def pin_nonneg_q(orc):
    """A >= 0 and b <= 0 give q = -A^T b / s >= 0: the passive set is empty at x = 0."""
    rng = _rng(13)
    A = rng.random((30, 10))
    b = -rng.random((30, 1))
    out = orc.nnls(A, b, 1e-10, 100)
    assert np.all(out["X"] == 0.0)
    assert out["iters"][0] == 0 and out["status"][0] == 0


def pin_brute_force(orc, count=120):
    """Tiny instances (n <= 8) against exhaustive support enumeration."""
    rng = _rng(14)
    for trial in range(count):
        n = int(rng.integers(1, 9))
        d = int(rng.integers(n, 3 * n + 2))
        A = rng.standard_normal((d, n)) if trial % 2 else rng.random((d, n))
        b = rng.standard_normal(d) * 2
        x_bf, F_bf = brute_force_nnls(A, b)
        out = orc.nnls(A, b.reshape(d, 1), 1e-13, 200000)
        x = out["X"][:, 0]
        F = 0.5 * np.sum((A @ x - b) ** 2)
        assert F <= F_bf + 1e-9 * max(1.0, F_bf), (trial, F, F_bf)
        assert np.allclose(x, x_bf, rtol=1e-6, atol=1e-7 * max(1.0, np.abs(x_bf).max())), trial


def pin_scipy_nnls(orc):
    """Moderate n against scipy's Lawson-Hanson active-set solver: objectives agree."""
    from scipy.optimize import nnls
    rng = _rng(15)
    for (d, n) in [(60, 20), (300, 100), (500, 200)]:
        A = rng.random((d, n))
        xt = np.where(rng.random(n) < 0.5, 0.0, rng.random(n))
        b = A @ xt + 0.01 * rng.standard_normal(d)
        x_s, rn = nnls(A, b, maxiter=50 * n)
        out = orc.nnls(A, b.reshape(d, 1), 1e-12, 1000000)
        x = out["X"][:, 0]
        F = 0.5 * np.sum((A @ x - b) ** 2)
        F_s = 0.5 * rn ** 2
        assert abs(F - F_s) <= 1e-9 * max(F_s, 1e-30) + 1e-14, (d, n, F, F_s)
        assert np.all(x >= 0)


def pin_gram(orc):
    """H = A^T A and h = -A^T B against numpy's product (Problem (2))."""
    rng = _rng(16)
    A = rng.standard_normal((37, 13))
    B = rng.standard_normal((37, 3))
    H, h = orc.gram(A, B)
    assert np.allclose(H, A.T @ A, rtol=1e-13, atol=1e-12)
    assert np.allclose(h, -(A.T @ B), rtol=1e-13, atol=1e-12)


def pin_rescale_remark(orc):
    """Remark of Section 3 and Lemma of Section 4: Q_ii = 1, Q_ij = cos(A_i, A_j) in [-1, 1],
    Q symmetric positive semidefinite, sqrt(n) <= ||Q||_F <= n; q_i = -A_i^T b / ||A_i||."""
    rng = _rng(17)
    for (d, n) in [(50, 20), (30, 40)]:
        A = rng.standard_normal((d, n)) * rng.random(n)[None, :] * 10
        b = rng.standard_normal((d, 1))
        s, Q, q = orc.prepare(A, b)
        norms = np.linalg.norm(A, axis=0)
        cos = (A.T @ A) / np.outer(norms, norms)
        assert np.allclose(Q, cos, rtol=1e-12, atol=1e-13)
        assert np.all(np.diag(Q) == 1.0)
        assert np.all(np.abs(Q) <= 1.0 + 1e-14)
        assert np.array_equal(Q, Q.T)
        assert np.linalg.eigvalsh(Q).min() > -1e-10
        fro = np.linalg.norm(Q)
        assert np.sqrt(n) - 1e-12 <= fro <= n + 1e-12
        assert np.allclose(s, norms, rtol=1e-14)
        assert np.allclose(q[:, 0], -(A.T @ b[:, 0]) / norms, rtol=1e-12, atol=1e-13)


def pin_invariances(orc):
    """Column scaling leaves the rescaled problem and the iteration count unchanged and maps
    x to x / c (the anti-lopsided property); permuting columns permutes x; x*(c b) = c x*(b)."""
    rng = _rng(18)
    d, n = 80, 30
    A = rng.random((d, n))
    xt = np.where(rng.random(n) < 0.5, 0.0, rng.random(n))
    b = (A @ xt + 0.01 * rng.standard_normal(d)).reshape(d, 1)
    base = orc.nnls(A, b, 1e-11, 100000, want_problem=True)
    c = np.exp(rng.uniform(-4, 4, n))
    sc = orc.nnls(A * c[None, :], b, 1e-11, 100000, want_problem=True)
    assert np.allclose(sc["Q"], base["Q"], rtol=1e-12, atol=1e-13)
    assert np.allclose(sc["q"], base["q"], rtol=1e-12, atol=1e-13)
    # same iterates up to rounding: identical counts at a moderate tolerance (rounding-level
    # differences in Q only shift the count of a long, ill-conditioned tail)
    assert orc.nnls(A * c[None, :], b, 1e-5, 100000)["iters"][0] == \
        orc.nnls(A, b, 1e-5, 100000)["iters"][0]
    assert abs(int(sc["iters"][0]) - int(base["iters"][0])) <= 0.05 * base["iters"][0]
    assert np.allclose(sc["X"][:, 0] * c, base["X"][:, 0], rtol=1e-7, atol=1e-9)
    perm = rng.permutation(n)
    pm = orc.nnls(A[:, perm], b, 1e-11, 100000)
    assert np.allclose(pm["X"][:, 0], base["X"][perm, 0], rtol=1e-7, atol=1e-9)
    hm = orc.nnls(A, 3.5 * b, 1e-11, 100000)
    assert np.allclose(hm["X"][:, 0], 3.5 * base["X"][:, 0], rtol=1e-7, atol=1e-9)


def pin_noiseless_recovery(orc):
    """b = A x_true with A of full column rank: the unique solution is x_true and F* = 0
    (the noiseless non-negative cases of Section 5)."""
    rng = _rng(19)
    d, n = 120, 40
    A = rng.random((d, n))
    xt = np.where(rng.random(n) < 0.6, 0.0, rng.random(n) + 0.1)
    b = (A @ xt).reshape(d, 1)
    out = orc.nnls(A, b, 1e-13, 1000000)
    assert np.allclose(out["X"][:, 0], xt, atol=1e-8 * xt.max())


def pin_kkt_metric(orc):
    """The x-space residual: 0 at the exact NNLS solution; 1 at x = 0 when A, b >= 0 (every
    entry of the scaled gradient is negative there, so min(y, g) = g = q)."""
    from scipy.optimize import nnls
    rng = _rng(20)
    A = rng.random((50, 15))
    b = rng.random(50)
    x_s, rn = nnls(A, b)
    r, F = orc.kkt_x(A, b.reshape(-1, 1), x_s.reshape(-1, 1))
    assert r[0] < 1e-10 and abs(F[0] - 0.5 * rn ** 2) < 1e-10
    r0, F0 = orc.kkt_x(A, b.reshape(-1, 1), np.zeros((15, 1)))
    assert abs(r0[0] - 1.0) < 1e-14 and abs(F0[0] - 0.5 * b @ b) < 1e-10


def pin_statuses(orc):
    """MAXITER when the cap is hit; NONFINITE on a NaN input; BREAKDOWN on a line-search
    denominator <= 0 (Q not positive semidefinite); a zero column gets scale 1 and x_i = 0."""
    rng = _rng(21)
    A = rng.random((60, 20))
    b = rng.random((60, 1))
    out = orc.nnls(A, b, 1e-14, 3)
    assert out["status"][0] == 1 and out["iters"][0] == 3
    An = A.copy()
    An[5, 5] = np.nan
    assert orc.nnls(An, b, 1e-8, 100)["status"][0] == 3
    Qbad = np.array([[1.0, 0.0], [0.0, -1.0]])
    y, it, kkt, st = orc.nqp(Qbad, np.array([0.0, -1.0]), 1e-10, 50)
    assert st == 2
    Az = A.copy()
    Az[:, 7] = 0.0
    out = orc.nnls(Az, b, 1e-10, 100000, want_problem=True)
    assert out["s"][7] == 1.0 and out["X"][7, 0] == 0.0
    assert np.all(out["Q"][7, :] == 0.0) and out["q"][7, 0] == 0.0
    fro = np.linalg.norm(out["Q"])
    assert np.sqrt(19) - 1e-12 <= fro <= 19 + 1e-12


ALL_PINS = [pin_eq3_example, pin_n1_closed_form, pin_orthogonal_columns, pin_nonneg_q,
            pin_brute_force, pin_scipy_nnls, pin_gram, pin_rescale_remark, pin_invariances,
            pin_noiseless_recovery, pin_kkt_metric, pin_statuses]
