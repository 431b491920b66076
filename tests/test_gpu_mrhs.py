"""Matrix-core many-right-hand-side solver against the FP64 oracle at every kernel instance.

The solver has one instance per register shape of Q: n <= 64, 128, 192 (Q in registers, 256
threads), n in (192, 256] (Q in registers over 8 waves, 512 threads) and n > 256 (Q read from
L2).  With Q in registers the products run in FP32 by default and as split FP16 products under
NNLS_MRHS_PRODUCT=split16; both forms are checked.  Each instance is checked one
update at a time from the oracle's own iterates (the line-search product Q gbar), two updates at
a time (the gradient carried from one update to the next through the correction product
Q (y' - y), or -alpha Q gbar when no slot clipped), and end to end on the shapes of the many-RHS and warm-start workloads with more
columns than resident slots, so the column queue refills.
"""
import numpy as np
import pytest
import torch

from gpu_common import dev, host, orc, say
from oracle import oracle as O
from paper_1502_01645_amd import nnls as N
from paper_1502_01645_amd import workloads as W

pytestmark = pytest.mark.gpu


def _uniform_case(seed, d, n, k):
    rng = np.random.default_rng(seed)
    A = rng.random((d, n)).astype(np.float32)
    X = np.where(rng.random((n, k)) < 0.6, 0.0, rng.random((n, k)))
    B = (A.astype(np.float64) @ X + 0.01 * rng.standard_normal((d, k))).astype(np.float32)
    return A, B


def _passive_and_clipped(Q, q, y):
    """|P| and |C| of one FP64 update of Algorithm 2 from y: the passive set of the masked
    gradient and the entries the projection clips."""
    g = Q @ y + q
    p = np.where((y > 0) | (g < 0), g, 0.0)
    P = int(np.count_nonzero((y > 0) | (g < 0)))
    den = p @ Q @ p
    if P == 0 or not den > 0:
        return P, 0
    alpha = (p @ p) / den
    return P, int(np.count_nonzero(y - alpha * p < 0))


# (n, k): 160 and 192 take the 3-tile instance, 200 and 256 the 512-thread 4-tile instance,
# 300 and 512 the instance that reads Q from L2; k leaves a ragged last group of 16 slots
# (k = 2, 3, 4: one nearly empty group, n = 64, 128, 256: one to four register tiles).
@pytest.mark.parametrize("product", ["split16", "fp32"])
@pytest.mark.parametrize("n,k", [(160, 37), (192, 21), (200, 37), (256, 37), (300, 21),
                                 (512, 19), (256, 19), (64, 2), (128, 4), (256, 3)])
def test_mrhs_steps_match_oracle(n, k, product, monkeypatch):
    monkeypatch.setenv("NNLS_SOLVER", "mrhs")
    if product == "split16":
        if n > 256:
            pytest.skip("Q read from L2 has only the FP32 product")
        monkeypatch.setenv("NNLS_MRHS_PRODUCT", "split16")
    assert N.solver_name(n, k) == "mrhs"
    say(f"mrhs single steps n={n} k={k} product={product}")
    A, B = _uniform_case(500 + n, 3 * n, n, k)
    Q, q, s = N.prepare(dev(A), dev(B))
    Qh, qh = host(Q).astype(np.float64), host(q).astype(np.float64)
    eps = 2.0 ** -23
    clipped_total = 0
    for m in [0, 1, 3, 10, 30]:
        Ym = np.zeros((n, k))
        if m:
            for c in range(k):
                Ym[:, c] = orc().nqp(Qh, qh[:, c], 0.0, m)[0]
        Ystart = Ym.astype(np.float32).astype(np.float64)
        rows = torch.zeros(k, dtype=torch.int64, device="cuda")
        Y, iters, kkt, st = N.solve(Q, q, None, tol=0.0, max_iter=1,
                                    Y0=dev(Ym.astype(np.float32)) if m else None,
                                    rows_read=rows)
        Yh = host(Y).astype(np.float64)
        rows_h = host(rows)
        assert np.all(host(iters) == 1)
        assert np.all(host(st) == N.MAXITER)
        worst = 0.0
        for c in range(k):
            yn = orc().nqp(Qh, qh[:, c], 0.0, 1, y0=Ystart[:, c])[0]
            err = np.abs(Yh[:, c] - yn).max()
            scale = np.abs(Ystart[:, c]).max() + np.abs(yn).max()
            worst = max(worst, err / scale)
            assert err <= 8 * n * eps * scale, (m, c, err / scale)
            # rows of Q the solve read: an exact refresh (n rows) when a start is given, the
            # passive rows of the line-search product, the clipped rows of the correction and
            # the exact refresh that confirms the MAXITER stop
            P, C = _passive_and_clipped(Qh, qh[:, c], Ystart[:, c])
            clipped_total += C
            want = (n if m else 0) + P + C + n
            assert abs(int(rows_h[c]) - want) <= 2, (m, c, int(rows_h[c]), want)
        say(f"  m={m}: worst rel err {worst:.2e}")
    # the gradient correction with clipped entries (the second product) was exercised
    assert clipped_total > 0


# Two updates from the oracle's iterates: the second update's line search runs on the gradient
# the first one carried forward (g + Q (y' - y), or g - alpha Q gbar when no slot clipped), so
# it checks the gradient correction product, in both product forms.
@pytest.mark.parametrize("product", ["split16", "fp32"])
@pytest.mark.parametrize("n,k", [(64, 2), (128, 19), (192, 21), (200, 37), (256, 37), (300, 21)])
def test_mrhs_two_updates_match_oracle(n, k, product, monkeypatch):
    monkeypatch.setenv("NNLS_SOLVER", "mrhs")
    if product == "split16":
        if n > 256:
            pytest.skip("Q read from L2 has only the FP32 product")
        monkeypatch.setenv("NNLS_MRHS_PRODUCT", "split16")
    say(f"mrhs two updates n={n} k={k} product={product}")
    A, B = _uniform_case(900 + n, 3 * n, n, k)
    Q, q, _ = N.prepare(dev(A), dev(B))
    Qh, qh = host(Q).astype(np.float64), host(q).astype(np.float64)
    eps = 2.0 ** -23
    clipped_total = 0
    for m in [0, 3, 12]:
        Ym = np.zeros((n, k))
        if m:
            for c in range(k):
                Ym[:, c] = orc().nqp(Qh, qh[:, c], 0.0, m)[0]
        Ystart = Ym.astype(np.float32).astype(np.float64)
        Y, iters, _, st = N.solve(Q, q, None, tol=0.0, max_iter=2,
                                  Y0=dev(Ym.astype(np.float32)) if m else None)
        Yh = host(Y).astype(np.float64)
        assert np.all(host(iters) == 2)
        assert np.all(host(st) == N.MAXITER)
        worst = 0.0
        for c in range(k):
            clipped_total += _passive_and_clipped(Qh, qh[:, c], Ystart[:, c])[1]
            yn = orc().nqp(Qh, qh[:, c], 0.0, 2, y0=Ystart[:, c])[0]
            err = np.abs(Yh[:, c] - yn).max()
            scale = np.abs(Ystart[:, c]).max() + np.abs(yn).max()
            worst = max(worst, err / scale)
            assert err <= 16 * n * eps * scale, (m, c, err / scale)
        say(f"  m={m}: worst rel err {worst:.2e}")
    assert clipped_total > 0


def _one_update(Q, q, Y0):
    Y, iters, _, st = N.solve(Q, q, None, tol=0.0, max_iter=1, Y0=Y0)
    assert np.all(host(iters) == 1) and np.all(host(st) == N.MAXITER)
    return host(Y).astype(np.float64)


def test_mrhs_split_products_on_unscaled_lopsided_gram(monkeypatch):
    """Algorithm 2 on the unscaled problem (H, h) = (A^T A, -A^T B) with column lengths spread
    over four decades: rows of H differ by up to 10^8 and its largest entries exceed FP16's
    range, so only the per-row scales of the split products keep them representable.  One
    update from the oracle's iterates agrees with the FP64 step as closely as the FP32
    products' update does."""
    monkeypatch.setenv("NNLS_SOLVER", "mrhs")
    n, k, d = 256, 37, 768
    rng = np.random.default_rng(77)
    A = (rng.random((d, n)) * 10.0 ** rng.uniform(-2, 2, n)).astype(np.float32)
    X = np.where(rng.random((n, k)) < 0.6, 0.0, rng.random((n, k)))
    B = (A.astype(np.float64) @ X).astype(np.float32)
    H, h = N.gram(dev(A), dev(B))
    Hh, hh = host(H).astype(np.float64), host(h).astype(np.float64)
    assert np.abs(Hh).max() > 65504.0
    say(f"mrhs split products on the unscaled Gram: max |H| {np.abs(Hh).max():.3e}")
    for m in [0, 5, 40]:
        Ym = np.zeros((n, k))
        if m:
            for c in range(k):
                Ym[:, c] = orc().nqp(Hh, hh[:, c], 0.0, m)[0]
        Ystart = Ym.astype(np.float32)
        Y0 = dev(Ystart) if m else None
        monkeypatch.setenv("NNLS_MRHS_PRODUCT", "split16")
        Ys = _one_update(H, h, Y0)
        monkeypatch.setenv("NNLS_MRHS_PRODUCT", "fp32")
        Yf = _one_update(H, h, Y0)
        monkeypatch.delenv("NNLS_MRHS_PRODUCT")
        for c in range(k):
            yn = orc().nqp(Hh, hh[:, c], 0.0, 1, y0=Ystart[:, c].astype(np.float64))[0]
            scale = np.abs(Ystart[:, c]).max() + np.abs(yn).max()
            err_s = np.abs(Ys[:, c] - yn).max()
            err_f = np.abs(Yf[:, c] - yn).max()
            assert np.isfinite(err_s), (m, c)
            assert err_s <= max(8 * n * 2.0 ** -23 * scale, 4 * err_f), (m, c, err_s, err_f)


def _check(A, B, res, sample, what):
    """FP64 KKT of every column against (A, B); relative objective gap against the oracle's
    tight solution on a sample of columns."""
    X = host(res["X"])
    assert np.all(X >= 0)
    r, F = orc().kkt_x(A, B, X)
    ref = O.reference_solution(A, B[:, sample])
    gap = O.relative_gap(F[sample], ref)
    say(f"{what}: max r={r.max():.3e} p99 r={np.percentile(r, 99):.3e} "
        f"max gap={gap.max():.3e} (sample {len(sample)})")
    assert r.max() <= 1e-5, r.max()
    assert gap.max() <= 1e-6, gap.max()
    np.testing.assert_allclose(host(res["kkt64"]), r, rtol=1e-6, atol=1e-14)


@pytest.mark.parametrize("product", ["fp32", "split16"])
def test_mrhs_end_to_end_manyrhs_shape(product, monkeypatch):
    """The many-RHS recipe (|N(0,1)| dictionary, Gamma(2,1) codes, 1 % noise) at n = 256 with
    8192 columns: twice the 4096 slots resident on 256 compute units, so every group refills
    from the queue."""
    monkeypatch.setenv("NNLS_MRHS_PRODUCT", product)
    A, B, _ = W.make_manyrhs(seed=7, d=3000, n=256, k=8192)
    say(f"mrhs e2e 3000x256 k=8192 product={product}")
    assert N.solver_name(256, 8192) == "mrhs"
    res = N.nnls(dev(A), dev(B), tol=1e-5, max_iter=100000, inner_tol=3e-6)
    assert np.all(host(res["status"]) == N.CONVERGED)
    it = host(res["iters"])
    say(f"  updates mean {it.mean():.1f} max {it.max()}")
    _check(A, B, res, np.arange(0, 8192, 128), "mrhs n=256")


@pytest.mark.parametrize("n,k", [(192, 9000), (320, 2500)])
def test_mrhs_end_to_end_other_instances(n, k):
    """The 3-tile register instance and the L2 instance end to end, more columns than slots."""
    A, B, _ = W.make_manyrhs(seed=8, d=3 * n, n=n, k=k)
    say(f"mrhs e2e {3 * n}x{n} k={k}")
    assert N.solver_name(n, k) == "mrhs"
    res = N.nnls(dev(A), dev(B), tol=1e-5, max_iter=100000, inner_tol=3e-6)
    assert np.all(host(res["status"]) == N.CONVERGED)
    _check(A, B, res, np.arange(0, k, max(1, k // 48)), f"mrhs n={n}")


@pytest.mark.parametrize("product", ["fp32", "split16"])
def test_mrhs_end_to_end_warm_shape(product, monkeypatch):
    """The warm-start recipe (A 4096 x 256 |N(0,1)|, noiseless b = A x, 85 % zeros) from the
    cold start, 6000 held-out columns."""
    monkeypatch.setenv("NNLS_MRHS_PRODUCT", product)
    A = W.make_warm_matrix()
    B, _ = W.make_warm_rhs(A, 6000, split=1, start=0)
    say("mrhs e2e warm shape 4096x256 k=6000")
    res = N.nnls(dev(A), dev(B), tol=1e-5, max_iter=100000, inner_tol=3e-6)
    assert np.all(host(res["status"]) == N.CONVERGED)
    _check(A, B, res, np.arange(0, 6000, 125), "mrhs warm shape")


@pytest.mark.parametrize("n,k", [(96, 3), (256, 4), (256, 20)])
def test_mrhs_nearly_empty_groups_end_to_end(n, k, monkeypatch):
    """Groups with few live columns (k <= 4, and the last group of k = 20) reach the
    tolerances against the oracle."""
    monkeypatch.setenv("NNLS_SOLVER", "mrhs")
    A, B, _ = W.make_manyrhs(seed=9, d=3 * n, n=n, k=k)
    say(f"mrhs few-column e2e {3 * n}x{n} k={k}")
    assert N.solver_name(n, k) == "mrhs"
    res = N.nnls(dev(A), dev(B), tol=1e-5, max_iter=100000, inner_tol=3e-6)
    assert np.all(host(res["status"]) == N.CONVERGED)
    _check(A, B, res, np.arange(k), f"mrhs few columns n={n}")
