"""Stand-ins for the test cases T1-T6 of Section 5 at reduced size (d = 600, n = 400, 20 %
sparsity): the GPU path end to end against the FP64 oracle's tight solution."""
import numpy as np
import pytest

from gpu_common import dev, host, orc, say
from oracle import oracle as O
from paper_1502_01645_amd import nnls as N
from paper_1502_01645_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("kind", range(1, 7))
def test_paper_case_end_to_end(kind):
    A, b, _ = W.make_paper_case(kind, 0.2, seed=2, d=600, n=400)
    say(f"T{kind} {W.PAPER_KINDS[kind]} 600 x 400")
    res = N.nnls(dev(A), dev(b), tol=1e-5, max_iter=100000, inner_tol=3e-6)
    X = host(res["X"])
    assert int(host(res["status"])[0]) == N.CONVERGED
    ref = O.reference_solution(A, b)
    r, F = orc().kkt_x(A, b, X)
    gap = O.relative_gap(F, ref)
    say(f"  r={r.max():.2e} gap={gap.max():.2e} updates={int(host(res['iters'])[0])}")
    assert np.all(X >= 0)
    assert r.max() <= 1e-5
    assert gap.max() <= 1e-6
