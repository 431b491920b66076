"""The FP64 oracle against what the paper and mathematics fix (CPU only)."""
import os
import subprocess

import numpy as np
import pytest

import oracle_pins as P
from oracle import oracle as O


@pytest.fixture(scope="module")
def orc():
    return O.load()


@pytest.mark.parametrize("pin", P.ALL_PINS, ids=lambda f: f.__name__)
def test_pin(orc, pin):
    pin(orc)


# Each planted slip (see PLANT in oracle.c) must be caught by at least one pin.
PLANTS = {
    1: "off-diagonal Gram entries perturbed",
    2: "minus sign of h dropped",
    3: "scale by H_ii instead of sqrt(H_ii)",
    4: "wrong sign in the passive-set test",
    5: "half the exact line-search step",
    6: "plus sign in the projected update",
}


@pytest.mark.parametrize("plant", sorted(PLANTS), ids=lambda p: PLANTS[p].replace(" ", "_"))
def test_pins_catch_planted_mistake(plant, tmp_path):
    path = O.build(plant=plant, out=str(tmp_path / f"liboracle_plant{plant}.so"))
    bad = O.Oracle(path)
    failed = []
    for pin in P.ALL_PINS:
        try:
            pin(bad)
        except (AssertionError, FloatingPointError, ValueError, TypeError,
                __import__("numpy").linalg.LinAlgError):
            failed.append(pin.__name__)
    assert failed, f"planted mistake '{PLANTS[plant]}' passed every pin"


# ---- the FP64 refinement step (one step of Algorithm 2 from a given x) ----------------------
def test_refine_candidate_n1_closed_form():
    """n = 1 from x = 0: the exact step lands on max(0, a^T b) / ||a||^2."""
    rng = P._rng(31)
    for _ in range(10):
        a = rng.random((7, 1)) + 0.1
        b = rng.standard_normal((7, 3))
        xc = O.refine_candidate(a, b, np.zeros((1, 3)))
        x_cf = np.maximum(0.0, a[:, 0] @ b) / (a[:, 0] @ a[:, 0])
        assert np.allclose(xc[0], x_cf, rtol=1e-13, atol=1e-15)


def test_refine_candidate_orthogonal_columns():
    """Q = I: one step from x = 0 is the clipped least-squares solution."""
    rng = P._rng(32)
    U, _ = np.linalg.qr(rng.standard_normal((30, 8)))
    A = U * (rng.random(8) * 4 + 0.5)[None, :]
    B = rng.standard_normal((30, 4))
    xc = O.refine_candidate(A, B, np.zeros((8, 4)))
    x_ls = np.maximum(0.0, A.T @ B) / np.sum(A * A, axis=0)[:, None]
    assert np.allclose(xc, x_ls, rtol=1e-10, atol=1e-12)


def test_refine_candidate_fixed_point_and_rounding():
    """At the solution the masked gradient vanishes and x stays; FP32 output is rounded."""
    rng = P._rng(33)
    A = rng.random((50, 6))
    x = np.array([0.5, 0.0, 1.5, 0.0, 0.25, 2.0])
    b = A @ x                                   # noiseless, full rank: x is the solution
    xc = O.refine_candidate(A, b, x)
    assert np.allclose(xc[:, 0], x, rtol=0, atol=1e-12)
    x32 = O.refine_candidate(A, b + 0.1, x, np.float32)
    assert np.array_equal(x32, x32.astype(np.float32).astype(np.float64))


def test_unscaled_ablation_on_lopsided_columns(orc):
    """Section 3's contrast at the size of a real problem: with column scales over two decades
    the anti-lopsided method reaches the scale-invariant KKT residual 1e-5, while Algorithm 2 on
    the unscaled (H, h), given the same number of updates and then ten times as many, stays
    orders of magnitude away; its own x-space stop test is no guide (it is not scale
    invariant)."""
    from paper_1502_01645_amd import workloads as W
    A, b, _, _ = W.make_lopsided(seed=0, d=2000, n=500, decades=2.0)
    H, h = orc.gram(A, b)
    s, Q, q = orc.rescale(H, h)
    y, m, _, st = orc.nqp(Q, q[:, 0], 1e-5, 100000)
    assert st == 0
    r_s, _ = orc.kkt_x(A, b, (y / s).reshape(-1, 1))
    assert r_s[0] <= 1e-5
    for mult in [1, 10]:
        x_u, it, _, _ = orc.nqp(H, h[:, 0], 0.0, mult * m)
        assert it == mult * m
        r_u, _ = orc.kkt_x(A, b, x_u.reshape(-1, 1))
        assert r_u[0] >= 30 * r_s[0], (mult, r_u, r_s)
    # stopping on the unscaled problem's own relative residual accepts a poor point
    x_u, it, r_own, st = orc.nqp(H, h[:, 0], 1e-5, 100000)
    r_u, _ = orc.kkt_x(A, b, x_u.reshape(-1, 1))
    assert st == 0 and r_own <= 1e-5 and r_u[0] >= 100 * r_s[0]
