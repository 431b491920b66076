"""Warm-start network on the GPU against the FP64 reference of the network, plus the objective
check that guards the warm start (a fallback to the cold start y = 0 of Algorithm 2)."""
import numpy as np
import pytest
import torch

from gpu_common import DEV, dev, host, orc, say
from oracle import mlp_ref as M
from paper_1502_01645_amd import nnls as N
from paper_1502_01645_amd import workloads as W

pytestmark = pytest.mark.gpu

LAM = 0.01


def _offsets():
    out, off = {}, 0
    for name, shape in M.SIZES:
        size = int(np.prod(shape))
        out[name] = (off, off + size)
        off += size
    return out


OFF = _offsets()


@pytest.fixture(scope="module")
def params():
    p = W.make_mlp_params(11).astype(np.float64)
    rng = np.random.default_rng(12)
    for name in ("b1", "b2", "b3"):  # nonzero biases so every bias path carries signal
        a, b = OFF[name]
        p[a:b] = 0.05 * rng.standard_normal(b - a)
    return p.astype(np.float32)


def _batch(b, seed):
    rng = np.random.default_rng(seed)
    u = rng.standard_normal((b, 256))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    t = np.where(rng.random((b, 256)) < 0.85, 0.0, 0.05 * rng.gamma(1.5, 1.0, (b, 256)))
    return u.astype(np.float32), t.astype(np.float32)


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("batch", [64, 192])
def test_forward_matches_reference(params, batch):
    say(f"mlp forward batch={batch}")
    u, _ = _batch(batch, batch)
    net = N.WarmStartNet(params, DEV)
    z = host(net.forward(dev(u)))
    z_em, _ = M.forward(params, u, emulate=True)
    assert _rel(z, z_em) <= 1e-3, _rel(z, z_em)
    # against exact FP64 arithmetic on the FP32 parameters: BF16 operands cost ~2^-8 relative
    z_ex, _ = M.forward(params, u)
    assert _rel(z, z_ex) <= 3e-2, _rel(z, z_ex)


def test_gradients_match_reference(params):
    say("mlp gradients batch=128")
    u, t = _batch(128, 3)
    net = N.WarmStartNet(params, DEV)
    loss, g = net.gradients(dev(u), dev(t), LAM)
    loss, g = float(host(loss)[0]), host(g).astype(np.float64)
    loss_ref, g_ref = M.gradients(params, u, t, LAM, emulate=True)
    assert abs(loss - loss_ref) <= 1e-4 * abs(loss_ref), (loss, loss_ref)
    for name, (a, b) in OFF.items():
        r = _rel(g[a:b], g_ref[a:b])
        say(f"  grad {name}: rel {r:.2e}")
        assert r <= 1e-3, (name, r)


def test_adam_first_step_and_bf16_copy(params):
    """Adam's bias-corrected first step is lr * g / (|g| + eps) exactly; the BF16 copy follows
    the master weights with round-to-nearest-even."""
    say("mlp adam step")
    u, t = _batch(64, 5)
    net = N.WarmStartNet(params, DEV)
    _, g = net.gradients(dev(u), dev(t), LAM)
    g = host(g).astype(np.float64)
    lr = 1e-3
    net.train_step(dev(u), dev(t), lr, LAM)
    w1 = host(net.master).astype(np.float64)
    w0 = params.astype(np.float64)
    expect = w0 - lr * g / (np.abs(g) + 1e-8)
    err = np.abs(w1 - expect)
    assert np.all(err <= 1e-6 * lr + 2 * 2.0 ** -24 * np.abs(w0) + 1e-12), err.max()
    P = net.P
    copy = host(net.blob[12 * P:14 * P].view(torch.int16)).astype(np.uint16)
    want = M.bf16(host(net.master)).astype(np.float32).view(np.uint32) >> 16
    assert np.array_equal(copy, want.astype(np.uint16))


def test_reset_state_clears_moments(params):
    net = N.WarmStartNet(params, DEV)
    u, t = _batch(64, 6)
    net.train_step(dev(u), dev(t), 1e-3, LAM)
    assert N.lib().nnls_mlp_reset_state(N._ptr(net.blob), N._stream(DEV)) == 0
    P = net.P
    mv = host(net.blob[4 * P:12 * P].view(torch.float32))
    assert np.all(mv == 0)


def _warm_problem(k, seed):
    A = W.make_warm_matrix()
    B, _ = W.make_warm_rhs(A, k, split=1, start=seed)
    return A, B


def _net_with_head(params, z_head):
    """A network whose output is z_head for every input: W3 = 0, b3 = z_head."""
    p = params.copy()
    a, b = OFF["W3"]
    p[a:b] = 0.0
    a, b = OFF["b3"]
    p[a:b] = z_head
    return N.WarmStartNet(p, DEV)


@pytest.mark.parametrize("factor,expect_fallback", [(3.0, 1), (1.0, 0)])
def test_warm_start_objective_check(params, factor, expect_fallback):
    """y0 = c u with u = max(-q, 0): f(c u) = c^2 u'Qu / 2 - c ||u||^2 is positive for
    c > 2 ||u||^2 / u'Qu (forced fallback) and negative at c = ||u||^2 / u'Qu."""
    say(f"warm start objective check factor={factor}")
    A, B = _warm_problem(1, 0)
    Q, q, s = N.prepare(dev(A), dev(B))
    Qh, qh = host(Q).astype(np.float64), host(q)[:, 0].astype(np.float64)
    uu = np.maximum(-qh, 0.0)
    c = factor * (uu @ uu) / (uu @ Qh @ uu)
    qn = np.linalg.norm(qh)
    net = _net_with_head(params, (c * uu / qn).astype(np.float32))
    Y0, fb = net.warm_start(Q, q)
    Y0, fb = host(Y0)[:, 0], host(fb)
    assert fb[0] == expect_fallback
    if expect_fallback:
        assert np.all(Y0 == 0)
        X_w, it_w, _, st_w = N.solve(Q, q, s, 1e-5, 0, Y0=torch.zeros_like(q))
        X_c, it_c, _, st_c = N.solve(Q, q, s, 1e-5, 0)
        assert np.array_equal(host(X_w), host(X_c))
        assert np.array_equal(host(it_w), host(it_c))
    else:
        np.testing.assert_allclose(Y0, c * uu, rtol=1e-5, atol=1e-6 * np.abs(c * uu).max())


def test_fallback_flags_follow_objective_sign(params):
    """Across many right-hand sides, the flag is set exactly where the FP64 objective of the
    predicted point is positive (columns with |f| within rounding of 0 may go either way)."""
    k = 320
    say(f"warm start flags k={k}")
    A, B = _warm_problem(k, 100)
    Q, q, s = N.prepare(dev(A), dev(B))
    # scale the head (W3, b3) by gamma: z, and so y0, scale by gamma, and f(gamma y) =
    # gamma^2 y'Qy / 2 + gamma q'y changes sign at gamma = -2 q'y / y'Qy.  The median of that
    # threshold over the columns (from the FP64 reference network) splits them about evenly.
    Qh, qh = host(Q).astype(np.float64), host(q).astype(np.float64)
    qn = np.linalg.norm(qh, axis=0)
    z0, _ = M.forward(params, (qh / qn).T, emulate=True)
    y0 = (qn[:, None] * np.maximum(z0, 0.0)).T
    thr = -2 * np.einsum("ik,ik->k", qh, y0) / np.einsum("ik,ij,jk->k", y0, Qh, y0)
    gamma = float(np.nanmedian(thr))
    p = params.astype(np.float64)
    for name in ("W3", "b3"):
        a, b = OFF[name]
        p[a:b] *= gamma
    net = N.WarmStartNet(p.astype(np.float32), DEV)
    Y0, fb = net.warm_start(Q, q)
    U, _ = N.mlp_inputs(q)
    z = host(net.forward(U)).astype(np.float64)
    y = (qn[:, None] * np.maximum(z, 0.0)).T
    f = 0.5 * np.einsum("ik,ij,jk->k", y, Qh, y) + np.einsum("ik,ik->k", qh, y)
    scale = np.einsum("ik,ij,jk->k", np.abs(y), np.abs(Qh), np.abs(y)) + np.abs(qh * y).sum(0)
    fb = host(fb)
    sure = np.abs(f) > 1e-4 * scale
    say(f"  fallbacks {int(fb.sum())} of {k}; undecided {int((~sure).sum())}")
    assert 0 < fb.sum() < k
    assert np.array_equal(fb[sure], (f[sure] > 0).astype(np.int32))
    Y0 = host(Y0)
    assert np.all(Y0[:, fb == 1] == 0)
    keep = fb == 0
    np.testing.assert_allclose(Y0[:, keep], y[:, keep], rtol=1e-4, atol=1e-6 * np.abs(y).max())


def test_mlp_inputs(params):
    A, B = _warm_problem(70, 7)
    Q, q, s = N.prepare(dev(A), dev(B))
    X, _, _, _ = N.solve(Q, q, None, 1e-5, 0)
    U, T = N.mlp_inputs(q, X)
    qh, Yh = host(q).astype(np.float64), host(X).astype(np.float64)
    qn = np.linalg.norm(qh, axis=0)
    np.testing.assert_allclose(host(U), (qh / qn).T, rtol=1e-6, atol=1e-7)
    np.testing.assert_allclose(host(T), (Yh / qn).T, rtol=1e-6, atol=1e-7)
