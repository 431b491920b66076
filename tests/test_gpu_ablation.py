"""The unscaled ablation on the GPU: Algorithm 2 on (H, h) = (A^T A, -A^T b) without the
anti-lopsided rescale, against the FP64 oracle on the same data.

Section 3 contrasts the two on the two-variable example of equation (3) (Figure 1: 40 unscaled
steps, Figure 2: 3 after the rescale); the oracle pins that example.  Here the same contrast is
checked at the size of a real problem with lopsided columns (column scales over two decades),
measured with the scale-invariant FP64 KKT residual of x against (A, b).
"""
import numpy as np
import pytest
import torch

from gpu_common import DEV, dev, gram_abs_tol, host, orc, say
from paper_1502_01645_amd import nnls as N
from paper_1502_01645_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("d,n,k,mode", [(700, 300, 2, "bf16x3"), (513, 384, 130, "bf16x3"),
                                        (300, 130, 1, "fp32")])
def test_gram_unscaled_matches_oracle(d, n, k, mode):
    """H = A^T A and h = -A^T b, no rescale: entries within the product's bound relative to
    ||A_i|| ||A_j|| (and ||A_i|| ||b||), exactly symmetric, the diagonal as computed."""
    say(f"unscaled gram {mode} d={d} n={n} k={k}")
    A, B, _, _ = W.make_lopsided(seed=d + n, d=d, n=n, decades=2.0)
    if k > 1:
        B = np.random.default_rng(d).random((d, k)).astype(np.float32)
    m = N.GRAM_BF16X3 if mode == "bf16x3" else N.GRAM_FP32
    H, h = N.gram(dev(A), dev(B), mode=m)
    Ho, ho = orc().gram(A, B)
    sn = np.sqrt(np.diag(Ho))
    bn = np.linalg.norm(B.astype(np.float64), axis=0)
    tol = gram_abs_tol(d, mode)
    Hh = host(H).astype(np.float64)
    assert np.array_equal(Hh, Hh.T)
    assert np.all(np.abs(Hh - Ho) <= tol * np.outer(sn, sn))
    assert np.all(np.abs(host(h).astype(np.float64) - ho) <= tol * np.outer(sn, bn))
    # the diagonal is H_ii itself, not the unit diagonal of the rescaled Q
    assert np.abs(np.diag(Hh) / np.diag(Ho) - 1.0).max() <= tol


@pytest.mark.parametrize("solver,k", [("wg", 1), ("regq", 1), ("mrhs", 3)])
def test_unscaled_steps_match_oracle(solver, k, monkeypatch):
    """One update of Algorithm 2 on the unscaled (H, h) from the oracle's iterate, element by
    element, for each solver kind."""
    monkeypatch.setenv("NNLS_SOLVER", solver)
    A, B, _, _ = W.make_lopsided(seed=5, d=400, n=96, decades=2.0)
    B = np.repeat(B, k, axis=1) * np.linspace(1.0, 2.0, k)[None, :].astype(np.float32)
    say(f"unscaled single steps {solver} k={k}")
    H, h = N.gram(dev(A), dev(B))
    Hh, hh = host(H).astype(np.float64), host(h).astype(np.float64)
    n = Hh.shape[0]
    eps = 2.0 ** -23
    for m in [0, 1, 3, 10]:
        Ym = np.zeros((n, k))
        for c in range(k):
            Ym[:, c] = orc().nqp(Hh, hh[:, c], 0.0, m)[0] if m else 0.0
        Ystart = Ym.astype(np.float32).astype(np.float64)
        Y, iters, _, _ = N.solve(H, h, None, tol=0.0, max_iter=1,
                                 Y0=dev(Ym.astype(np.float32)) if m else None)
        Yh = host(Y).astype(np.float64)
        assert np.all(host(iters) == 1)
        for c in range(k):
            yn = orc().nqp(Hh, hh[:, c], 0.0, 1, y0=Ystart[:, c])[0]
            err = np.abs(Yh[:, c] - yn).max()
            scale = np.abs(Ystart[:, c]).max() + np.abs(yn).max()
            assert err <= 8 * n * eps * scale, (m, c, err / scale)
    monkeypatch.delenv("NNLS_SOLVER", raising=False)


def test_unscaled_needs_far_more_updates():
    """Lopsided columns (scales over two decades), 2000 x 500: the anti-lopsided solve reaches
    the scale-invariant FP64 KKT residual 1e-5; the unscaled method, given the same number of
    updates and then ten times as many, is still orders of magnitude away, as the oracle's own
    unscaled run from the same start is."""
    A, b, _, _ = W.make_lopsided(seed=0, d=2000, n=500, decades=2.0)
    say("ablation 2000 x 500")
    Q, q, s = N.prepare(dev(A), dev(b))
    X, it, _, st = N.solve(Q, q, s, tol=1e-5, max_iter=100000, out=None)
    m = int(host(it)[0])
    assert int(host(st)[0]) == N.CONVERGED
    r_s, _ = orc().kkt_x(A, b, host(X))
    H, h = N.gram(dev(A), dev(b))
    Hh, hh = host(H).astype(np.float64), host(h).astype(np.float64)[:, 0]
    for mult in [1, 10]:
        Xu, itu, _, _ = N.solve(H, h, None, tol=0.0, max_iter=mult * m)
        assert int(host(itu)[0]) == mult * m
        r_u, _ = orc().kkt_x(A, b, host(Xu))
        ro_u, _ = orc().kkt_x(A, b, orc().nqp(Hh, hh, 0.0, mult * m)[0].reshape(-1, 1))
        say(f"  {m} anti-lopsided updates r={r_s[0]:.2e}; {mult * m} unscaled r={r_u[0]:.2e} "
            f"(oracle {ro_u[0]:.2e})")
        assert r_s[0] <= 1e-5
        assert r_u[0] >= 30 * r_s[0] and ro_u[0] >= 30 * r_s[0]
        # the GPU's FP32 unscaled run follows the oracle's FP64 one to within a factor of 3
        assert ro_u[0] / 3 <= r_u[0] <= 3 * ro_u[0]
