"""Plain FP64 numpy reference of the warm-start network (test infrastructure only).

The network maps u = q / ||q|| (256) through 1024 -> 1024 GELU hidden layers to a 256-wide head z
whose ReLU is the direction of the start point.  Loss per sample:
1/2 ||ReLU(z) - t||^2 + lambda * BCE(z, 1[t > 0]) with t = y* / ||y*||, averaged over the batch.  Everything here is written from those definitions:
exact GELU x * Phi(x) via erf, hand-derived backward pass.  `emulate` rounds the same tensors to
bfloat16 that the GPU kernels store in bfloat16 (weights, inputs, hidden activations and the
backward signals), so kernel logic can be compared tightly; without it the reference is exact
FP64 math on the given parameters.
"""
from __future__ import annotations

import math

import numpy as np

IN, H, OUT = 256, 1024, 256
SIZES = [("W1", (IN, H)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("W3", (H, OUT)),
         ("b3", (OUT,))]
P = sum(int(np.prod(s)) for _, s in SIZES)

_erf = np.vectorize(math.erf)


def unpack(flat):
    """Split a flat parameter vector (the library's layout) into named arrays."""
    out, off = {}, 0
    for name, shape in SIZES:
        size = int(np.prod(shape))
        out[name] = np.asarray(flat[off:off + size], dtype=np.float64).reshape(shape)
        off += size
    return out


def pack(params):
    return np.concatenate([np.asarray(params[name], dtype=np.float64).reshape(-1)
                           for name, _ in SIZES])


def bf16(x):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    x32 = np.asarray(x, dtype=np.float32)
    u = x32.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def gelu(x):
    return 0.5 * x * (1.0 + _erf(x / math.sqrt(2.0)))


def gelu_grad(x):
    cdf = 0.5 * (1.0 + _erf(x / math.sqrt(2.0)))
    pdf = np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)
    return cdf + x * pdf


def standardise(u, shift=None, scale=None):
    """x = (u - shift) * scale per feature (identity when not given), in FP32 as the kernels
    compute it before rounding x to bfloat16."""
    u = np.asarray(u, dtype=np.float32)
    if shift is None:
        return u.astype(np.float64)
    x = (u - np.asarray(shift, np.float32)) * np.asarray(scale, np.float32)
    return x.astype(np.float32).astype(np.float64)


def forward(flat, u, emulate=False, shift=None, scale=None):
    """z and the intermediates of the forward pass for inputs u [batch, 256]."""
    p = unpack(flat)
    r = bf16 if emulate else (lambda a: np.asarray(a, dtype=np.float64))
    W1, W2, W3 = r(p["W1"]), r(p["W2"]), r(p["W3"])
    x = r(standardise(u, shift, scale))
    h1 = x @ W1 + p["b1"]
    a1 = r(gelu(h1))
    h2 = a1 @ W2 + p["b2"]
    a2 = r(gelu(h2))
    z = a2 @ W3 + p["b3"]
    return z, dict(x=x, h1=h1, a1=a1, h2=h2, a2=a2, W1=W1, W2=W2, W3=W3)


def loss_and_grad_z(z, t, lam):
    """Mean loss over the batch and its gradient with respect to z."""
    m = z.shape[0]
    relu = np.maximum(z, 0.0)
    lab = (t > 0).astype(np.float64)
    diff = relu - t
    bce = relu - z * lab + np.log1p(np.exp(-np.abs(z)))
    loss = np.sum(0.5 * diff * diff + lam * bce) / m
    sig = 1.0 / (1.0 + np.exp(-z))
    dz = (diff * (z > 0) + lam * (sig - lab)) / m
    return loss, dz


def gradients(flat, u, t, lam, emulate=False, shift=None, scale=None):
    """(loss, flat gradient) for a batch."""
    z, c = forward(flat, u, emulate, shift, scale)
    loss, dz = loss_and_grad_z(z, t, lam)
    r = bf16 if emulate else (lambda a: a)
    dz = r(dz)
    g = {}
    g["W3"] = c["a2"].T @ dz
    g["b3"] = dz.sum(axis=0)
    dh2 = r((dz @ c["W3"].T) * gelu_grad(c["h2"]))
    g["W2"] = c["a1"].T @ dh2
    g["b2"] = dh2.sum(axis=0)
    dh1 = r((dh2 @ c["W2"].T) * gelu_grad(c["h1"]))
    g["W1"] = c["x"].T @ dh1
    g["b1"] = dh1.sum(axis=0)
    return loss, pack(g)
