"""The alternating NNLS outer loop of a nonnegative matrix factorisation on the GPU (each half a
many-right-hand-side NNLS problem through the library's calls), against the FP64 oracle."""
import numpy as np
import pytest
import torch

from gpu_common import dev, host, orc, say
from oracle import oracle as O
from paper_1502_01645_amd import nmf as F
from paper_1502_01645_amd import nnls as N
from paper_1502_01645_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("rows,cols,pad", [(130, 77, 0), (64, 64, 5), (1, 300, 0), (1000, 3, 2)])
def test_transpose_exact(rows, cols, pad):
    rng = np.random.default_rng(rows + cols)
    big = rng.standard_normal((rows, cols + pad)).astype(np.float32)
    src = dev(big)[:, :cols]
    out = host(N.transpose(src))
    assert np.array_equal(out, big[:, :cols].T)


def _check(A, B, X, what):
    r, Fv = orc().kkt_x(A, B, X)
    ref = O.reference_solution(A, B)
    gap = O.relative_gap(Fv, ref)
    say(f"  {what}: max r={r.max():.2e} max gap={gap.max():.2e}")
    assert np.all(X >= 0)
    assert r.max() <= 1e-5
    assert gap.max() <= 1e-6
    return float(Fv.sum())


def test_nmf_step_matches_oracle():
    """One outer step from W0: H1 solves min ||V - W0 H|| and W1 solves min ||V - W H1|| column
    by column to the method's tolerances against the oracle's tight solutions, the reported FP64
    objectives are those of the returned factors, and the W half does not raise the objective."""
    m, p, r = 240, 150, 12
    V, W0, _, _ = W.make_nmf(seed=3, m=m, p=p, r=r)
    say(f"nmf step {m} x {p} rank {r}")
    alt = F.AlternatingNNLS(dev(V), dev(W0), inner_tol=3e-6)
    alt.step()
    H1, W1 = host(alt.H).astype(np.float64), host(alt.W).astype(np.float64)
    fH = _check(W0, V, H1, "H half")
    fW = _check(H1.astype(np.float32).T.copy(), V.T.copy(), W1.T.copy(), "W half")
    oH, oW = alt.objective()
    assert abs(oH - fH) <= 1e-9 * fH and abs(oW - fW) <= 1e-9 * fW
    assert oW <= oH * (1 + 1e-6)
    assert np.array_equal(host(alt.Wt), host(alt.W).T)


def test_nmf_objective_decreases():
    """Four outer steps at a larger size: the objective never rises (beyond the solves'
    tolerance) and the fit improves on the start."""
    m, p, r = 2000, 1000, 32
    V, W0, _, _ = W.make_nmf(seed=4, m=m, p=p, r=r)
    say(f"nmf 4 steps {m} x {p} rank {r}")
    alt = F.AlternatingNNLS(dev(V), dev(W0))
    objs = []
    for _ in range(4):
        alt.step()
        objs.extend(alt.objective())
        st = alt.stats()
        assert st["H"]["not_converged"] == 0 and st["W"]["not_converged"] == 0
    say(f"  objectives {['%.6e' % o for o in objs]}")
    for a, b in zip(objs, objs[1:]):
        assert b <= a * (1 + 1e-6)
    assert objs[-1] < 0.9 * objs[0]


def test_rescale_start():
    rng = np.random.default_rng(9)
    s = rng.random(37) * 10 + 0.1
    X = rng.random((37, 5)).astype(np.float32)
    Y = host(N.rescale_start(dev(s), dev(X)))
    assert np.array_equal(Y, (s[:, None] * X.astype(np.float64)).astype(np.float32))


def test_nmf_warm_steps_match_oracle():
    """From the second step on each half starts from its previous factor: the halves still land
    on the oracle's solutions of their own problems, with fewer updates than cold starts."""
    m, p, r = 240, 150, 12
    V, W0, _, _ = W.make_nmf(seed=5, m=m, p=p, r=r)
    say(f"nmf warm steps {m} x {p} rank {r}")
    warm = F.AlternatingNNLS(dev(V), dev(W0), inner_tol=3e-6)
    cold = F.AlternatingNNLS(dev(V), dev(W0), inner_tol=3e-6, warm=False)
    for _ in range(3):
        W_prev = host(warm.W).astype(np.float32)
        warm.step()
        cold.step()
    H3, W3 = host(warm.H).astype(np.float64), host(warm.W).astype(np.float64)
    _check(W_prev, V, H3, "H half, warm")
    _check(H3.astype(np.float32).T.copy(), V.T.copy(), W3.T.copy(), "W half, warm")
    uw, uc = warm.stats(), cold.stats()
    say(f"  mean updates warm H {uw['H']['updates_mean']:.1f} W {uw['W']['updates_mean']:.1f}; "
        f"cold H {uc['H']['updates_mean']:.1f} W {uc['W']['updates_mean']:.1f}")
    assert uw["H"]["updates_mean"] < uc["H"]["updates_mean"]
    assert uw["W"]["updates_mean"] < uc["W"]["updates_mean"]
