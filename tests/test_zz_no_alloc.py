"""nnls_solve_noalloc (the solve that allocates nothing) against nnls_solve on the same inputs.

Two calls in a row through the C ABI, the second with a smaller input, so the second call finds
the first call's state in the library's fixed scratch array: a whole-GPU single right-hand-side
solve (n = 3000), then a many right-hand-side solve (n = 256, k = 300, fewer columns than
resident slots, so the column-to-slot order is fixed), then a small FP64 per-column solve.  The
solvers are deterministic for these shapes, so results must match bit for bit."""
import numpy as np
import pytest
import torch

from gpu_common import dev, host, say
from paper_1502_01645_amd import nnls as N
from paper_1502_01645_amd import workloads as W

pytestmark = pytest.mark.gpu


def _outputs(n, k, dtype, device):
    return (torch.empty((n, k), dtype=dtype, device=device),
            torch.empty(k, dtype=torch.int32, device=device),
            torch.empty(k, dtype=torch.float64, device=device),
            torch.empty(k, dtype=torch.int32, device=device))


def _compare(Q, q, s, tol, max_iter, Y0=None):
    n, k = q.shape
    rows_ref = torch.zeros(k, dtype=torch.int64, device=Q.device)
    ref = N.solve(Q, q, s, tol=tol, max_iter=max_iter, Y0=Y0, rows_read=rows_ref)
    out = _outputs(n, k, Q.dtype, Q.device)
    rows = torch.zeros(k, dtype=torch.int64, device=Q.device)
    got = N.solve_noalloc(Q, q, s, tol, max_iter, Y0, out, rows_read=rows)
    torch.cuda.synchronize()
    for a, b in zip(ref, got):
        np.testing.assert_array_equal(host(a), host(b))
    np.testing.assert_array_equal(host(rows), host(rows_ref))
    return host(got[3]), host(got[1])


def test_noalloc_solve_matches_solve_twice_smaller_second():
    # 1. one right-hand side, n = 3000: the whole-GPU solver (exchange words, barrier and abort
    #    word in the scratch array)
    A, b, _ = W.make_large(seed=21, d=6000, n=3000)
    say(f"noalloc 1: n=3000 k=1 solver={N.solver_name(3000, 1)}")
    Q, q, s = N.prepare(dev(A), dev(b))
    st, it = _compare(Q, q, s, 1e-5, 100000)
    assert st[0] == N.CONVERGED and it[0] > 0
    # 2. smaller: n = 256, k = 300, the matrix-core many right-hand-side solver (queue counter)
    A, B, _ = W.make_manyrhs(seed=22, d=1500, n=256, k=300)
    say(f"noalloc 2: n=256 k=300 solver={N.solver_name(256, 300)}")
    Q, q, s = N.prepare(dev(A), dev(B))
    st, it = _compare(Q, q, s, 1e-5, 100000)
    assert np.all(st == N.CONVERGED)
    # 3. smaller still: FP64 per-column solver, n = 40, k = 7, from a warm start
    rng = np.random.default_rng(23)
    A = rng.random((120, 40))
    B = A @ np.where(rng.random((40, 7)) < 0.5, 0.0, rng.random((40, 7))) \
        + 0.01 * rng.standard_normal((120, 7))
    say(f"noalloc 3: n=40 k=7 FP64 solver={N.solver_name(40, 7, N.F64)}")
    Q, q, s = N.prepare(dev(A), dev(B))
    Y0 = dev(rng.random((40, 7)))
    st, it = _compare(Q, q, s, 1e-10, 100000, Y0=Y0)
    assert np.all(st == N.CONVERGED)


def test_noalloc_rejects_oversized_scratch_on_device():
    """A per-column solve whose state exceeds the fixed array is refused, nothing launched."""
    Q = torch.eye(500, dtype=torch.float64, device="cuda")
    q = -torch.ones((500, 1000), dtype=torch.float64, device="cuda")
    out = _outputs(500, 1000, torch.float64, "cuda")
    with pytest.raises(N.NNLSError, match="workspace"):
        N.solve_noalloc(Q, q, None, 1e-6, 0, None, out)
