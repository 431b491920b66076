"""The stand-ins for the test cases T1-T6 of Section 5 (Table 1): signs, sparsity, column lengths
and the noiseless right-hand side, checked on the generator itself (CPU only)."""
import numpy as np
import pytest

from paper_1502_01645_amd import workloads as W


@pytest.mark.parametrize("kind", range(1, 7))
@pytest.mark.parametrize("sparsity", [0.0, 0.3])
def test_paper_case_structure(kind, sparsity):
    d, n = 300, 200
    A, b, x = W.make_paper_case(kind, sparsity, seed=1, d=d, n=n)
    signs, lengths = W.PAPER_KINDS[kind]
    assert A.shape == (d, n) and A.dtype == np.float32 and b.shape == (d, 1) and x.shape == (n,)
    if signs == "+":
        assert np.all(A >= 0) and np.all(x >= 0)
    else:
        assert (A < 0).any() and (x < 0).any()
    assert np.all(np.sum(A == 0, axis=0) == int(round(sparsity * d)))
    assert np.sum(x == 0) == int(round(sparsity * n))
    norms = np.linalg.norm(A.astype(np.float64), axis=0)
    if lengths == "SAM":
        assert np.allclose(norms, 1.0, rtol=1e-6)
    elif lengths == "RAN":
        assert norms.max() <= 1.0 + 1e-6 and norms.min() < 0.1
    else:
        assert norms.max() / norms.min() >= 1e3
    bx = A.astype(np.float64) @ x
    assert np.allclose(b[:, 0], bx, rtol=1e-6, atol=1e-6 * np.abs(bx).max())


def test_paper_case_seeding():
    """Each (kind, sparsity, seed) is its own stream: repeatable, and distinct across kinds."""
    a1 = W.make_paper_case(2, 0.1, seed=3, d=50, n=40)[0]
    a2 = W.make_paper_case(2, 0.1, seed=3, d=50, n=40)[0]
    a3 = W.make_paper_case(4, 0.1, seed=3, d=50, n=40)[0]
    assert np.array_equal(a1, a2) and not np.array_equal(a1, a3)
