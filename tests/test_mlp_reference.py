"""The FP64 network reference against finite differences and closed-form values (CPU only)."""
import math

import numpy as np

from oracle import mlp_ref as M
from paper_1502_01645_amd import workloads as W


def test_layout_size():
    assert M.P == 256 * 1024 + 1024 + 1024 * 1024 + 1024 + 1024 * 256 + 256


def test_bf16_rounding():
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, 3.14159265, -2.5e-3, 0.0])
    y = M.bf16(x)
    assert y[0] == 1.0 and y[1] == 1.0           # tie to even
    assert y[2] == 1.0 + 2 ** -7                   # above the midpoint rounds up
    assert abs(y[3] - 3.140625) < 1e-12
    assert np.all(np.abs(y - x) <= np.abs(x) * 2 ** -8)


def test_gelu_closed_forms():
    assert M.gelu(np.array([0.0]))[0] == 0.0
    x = np.array([1.0])
    assert abs(M.gelu(x)[0] - 0.5 * (1 + math.erf(1 / math.sqrt(2)))) < 1e-15
    xs = np.linspace(-4, 4, 41)
    fd = (M.gelu(xs + 1e-6) - M.gelu(xs - 1e-6)) / 2e-6
    assert np.allclose(M.gelu_grad(xs), fd, atol=1e-8)


def test_loss_at_zero_logits():
    """z = 0: ReLU part = 1/2 ||t||^2, BCE = log 2 per entry."""
    z = np.zeros((3, 256))
    t = np.abs(np.random.default_rng(0).standard_normal((3, 256)))
    loss, dz = M.loss_and_grad_z(z, t, 0.1)
    expect = (0.5 * np.sum(t * t) + 0.1 * 3 * 256 * math.log(2)) / 3
    assert abs(loss - expect) < 1e-10


def test_gradients_match_finite_differences():
    rng = np.random.default_rng(1)
    flat = W.make_mlp_params(3).astype(np.float64)
    flat[M.P - 256:] = 0.05 * rng.standard_normal(256)  # nonzero b3 so ReLU is not flat
    u = rng.standard_normal((4, 256))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    t = np.maximum(rng.standard_normal((4, 256)), 0) * 0.1
    loss, g = M.gradients(flat, u, t, 0.05)
    idx = np.concatenate([rng.choice(M.P, 40, replace=False),
                          np.arange(M.P - 256, M.P - 250)])
    h = 1e-6
    for i in idx:
        e = np.zeros(M.P)
        e[i] = h
        lp, _ = M.gradients(flat + e, u, t, 0.05)
        lm, _ = M.gradients(flat - e, u, t, 0.05)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 + 1e-4 * abs(g[i]), (i, fd, g[i])
