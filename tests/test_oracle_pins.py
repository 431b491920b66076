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


# ---- the relative objective gap behind every parity check ---------------------------------------
def _gap_flipped(F, ref):
    """Planted slip: the difference taken the wrong way round."""
    F = np.asarray(F, dtype=np.float64)
    fstar = ref.F - ref.half_bb
    return (ref.F - F) / np.where(np.abs(fstar) > 0, np.abs(fstar), 1.0)


def _gap_over_Fstar(F, ref):
    """Planted slip: (F - F*) / F*, the residual-relative reading, undefined at F* = 0."""
    F = np.asarray(F, dtype=np.float64)
    return (F - ref.F) / np.where(ref.F > 0, ref.F, 1.0)


def _gap_whole_bb(F, ref):
    """Planted slip: f = F - ||b||^2 (the 1/2 dropped) in the denominator."""
    F = np.asarray(F, dtype=np.float64)
    fstar = ref.F - 2.0 * ref.half_bb
    return (F - ref.F) / np.where(np.abs(fstar) > 0, np.abs(fstar), 1.0)


def _gap_pins(gap, orc):
    """What the definition of the gap fixes without the oracle's help.
    For n = 1, f(x) = 1/2 ||a||^2 x^2 - (a^T b) x is a parabola with minimum x* = a^T b / ||a||^2
    and f* = -(a^T b)^2 / (2 ||a||^2), so gap(x) = (f(x) - f*) / |f*| = ((x - x*) / x*)^2 exactly;
    where a^T b <= 0, x* = 0, f* = 0 and the gap is the absolute f(x).  For any instance with
    f* < 0, x = 0 gives f = 0 and so gap = 1; the solution gives 0 and any other feasible point
    a positive gap."""
    rng = np.random.default_rng(41)
    for _ in range(4):
        a = rng.random((9, 1)) + 0.1
        b = (2.0 * a[:, 0] + 0.3 * rng.standard_normal(9)).reshape(9, 1)
        ab, aa = float(a[:, 0] @ b[:, 0]), float(a[:, 0] @ a[:, 0])
        assert ab > 0
        xs = ab / aa
        ref = O.reference_solution(a, b, orc=orc)
        for t in (0.0, 0.5, 1.0, 1.3, 2.0):
            x = np.array([[t * xs]])
            _, F = orc.kkt_x(a, b, x)
            g = float(gap(F, ref)[0])
            assert abs(g - (t - 1.0) ** 2) <= 1e-9, (t, g)
    # x* = 0: f* = 0, the gap is f(x) itself
    a = rng.random((9, 1)) + 0.1
    b = -(a + 0.1 * rng.random((9, 1)))
    ab, aa = float(a[:, 0] @ b[:, 0]), float(a[:, 0] @ a[:, 0])
    ref = O.reference_solution(a, b, orc=orc)
    for x in (0.0, 0.7):
        _, F = orc.kkt_x(a, b, np.array([[x]]))
        g = float(gap(F, ref)[0])
        assert abs(g - (0.5 * aa * x * x - ab * x)) <= 1e-12 * (1 + abs(ab)), (x, g)
    # a generic instance: 1 at the origin, 0 at the solution, positive elsewhere
    A = rng.random((40, 12))
    x_true = np.where(rng.random(12) < 0.5, 0.0, rng.random(12))
    B = (A @ x_true + 0.05 * rng.standard_normal(40)).reshape(40, 1)
    ref = O.reference_solution(A, B, orc=orc)
    _, F0 = orc.kkt_x(A, B, np.zeros((12, 1)))
    assert abs(float(gap(F0, ref)[0]) - 1.0) <= 1e-12
    assert abs(float(gap(ref.F, ref)[0])) <= 1e-15
    xp = ref.X + 0.01 * rng.random((12, 1))
    _, Fp = orc.kkt_x(A, B, xp)
    assert float(gap(Fp, ref)[0]) > 0


def test_relative_gap_pins(orc):
    _gap_pins(O.relative_gap, orc)


@pytest.mark.parametrize("planted", [_gap_flipped, _gap_over_Fstar, _gap_whole_bb],
                         ids=lambda f: f.__name__)
def test_gap_pins_catch_planted_mistake(orc, planted):
    with pytest.raises(AssertionError):
        _gap_pins(planted, orc)
