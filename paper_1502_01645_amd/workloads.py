"""Seeded synthetic NNLS instances shared by the oracle checks, the GPU tests and the benchmark.

This module only draws random inputs (A, b / B and the planted solution x_true).  It holds none
of the method's arithmetic: no Gram product, rescale or iteration lives here, so it can feed both
the plain CPU oracle and the HIP path without coupling them.

The paper (Section 5, Table 1) builds its test cases as b = A x* from random A and x* with a share
of zero entries; its own files were never published, so the five workloads below are stand-ins of
the same kind, each generated from a fixed seed:

  small    200 x 50, FP64, A ~ U[0,1], 25 zeros in x, the rest U[0,1], noise N(0, 0.01^2)
  large    20000 x 5000, FP32, A ~ U[0,1], 3500 zeros in x, nonzeros Exp(1),
           noise sigma = 0.01 * mean(b0)
  manyrhs  10000 x 256, A ~ |N(0,1)|, X 256 x 4096 with 205 zeros per column and Gamma(2,1)
           nonzeros, per-column noise sigma = 0.01 * RMS(b0)
  batched  8192 problems, problem i seeded by SeedSequence([0, i]): n ~ U{16..512}, d = 3n,
           A ~ U[0,1], x with round(0.6 n) zeros and U[0,1] nonzeros, 1 % relative noise
  warm     A 4096 x 256 ~ |N(0,1)| (seed 0); right-hand sides b = A x with 218 zeros per x and
           Gamma(1.5,1) nonzeros, noiseless; training set SeedSequence([5,0]), eval SeedSequence([5,1])

Draw order per instance: A, zero-index permutation, nonzero values, noise.  "1 % relative noise"
means sigma = 0.01 * RMS of the noise-free column.  Every size can be scaled down for tests.
"""
from __future__ import annotations

import numpy as np


def _zero_pattern(rng: np.random.Generator, n: int, n_zero: int, nonzero_draw) -> np.ndarray:
    x = np.zeros(n, dtype=np.float64)
    perm = rng.permutation(n)
    nz_idx = perm[n_zero:]
    x[nz_idx] = nonzero_draw(len(nz_idx))
    return x


def make_small(seed: int = 0, d: int = 200, n: int = 50):
    """Small FP64 instance: A ~ U[0,1], half of x zero, the rest U[0,1], noise N(0, 0.01^2)."""
    rng = np.random.default_rng(seed)
    A = rng.random((d, n))
    x = _zero_pattern(rng, n, int(round(0.5 * n)), lambda m: rng.random(m))
    b0 = A @ x
    b = b0 + rng.normal(0.0, 0.01, size=d)
    return A.astype(np.float64), b.reshape(d, 1).astype(np.float64), x


def make_large(seed: int = 0, d: int = 20000, n: int = 5000, dtype=np.float32):
    """Large single right-hand side: A ~ U[0,1] dense, 70 % of x zero, nonzeros Exp(1),
    noise sigma = 0.01 * mean(b0)."""
    rng = np.random.default_rng(seed)
    A = rng.random((d, n), dtype=np.float64).astype(dtype)
    x = _zero_pattern(rng, n, int(round(0.7 * n)), lambda m: rng.exponential(1.0, m))
    b0 = A.astype(np.float64) @ x
    sigma = 0.01 * float(np.mean(b0))
    b = b0 + rng.normal(0.0, sigma, size=d)
    return A, b.reshape(d, 1).astype(dtype), x


def make_lopsided(seed: int = 0, d: int = 20000, n: int = 5000, decades: float = 2.0,
                  dtype=np.float32):
    """The large single right-hand side recipe with lopsided columns: column j of A is multiplied
    by c_j = 10^u, u ~ U(-decades / 2, decades / 2) (drawn from SeedSequence([9, seed]) after the
    base instance), b unchanged, so the solution is x / c.  Returns (A c, b, x / c, c)."""
    A, b, x = make_large(seed, d, n, dtype=np.float64)
    rng = np.random.default_rng(np.random.SeedSequence([9, seed]))
    c = 10.0 ** rng.uniform(-decades / 2.0, decades / 2.0, n)
    return (A * c[None, :]).astype(dtype), b.astype(dtype), x / c, c


PAPER_KINDS = {  # kind: (signs of A and x*, column lengths), Section 5, Table 1
    1: ("+", "SAM"), 2: ("+-", "RAN"), 3: ("+", "VAR"),
    4: ("+-", "SAM"), 5: ("+", "RAN"), 6: ("+-", "VAR"),
}
PAPER_SPARSITY = (0.0, 0.1, 0.2, 0.3, 0.4)


def make_paper_case(kind: int, sparsity: float, seed: int = 0, d: int = 6000, n: int = 4000,
                    dtype=np.float32):
    """Stand-in for test case T<kind> of Section 5 (the paper's 30 cases were never published):
    A [d, n] and x* [n] nonnegative (entries U[0, 1]) or mixed-sign (U[-1, 1]); round(sparsity d)
    zeros in every column of A and round(sparsity n) zeros in x*; the columns of A then scaled to
    the same length 1 (SAM), to random lengths U(0, 1] (RAN) or to lengths 10^U(-2, 2) spanning
    four decades (VAR); b = A x* without noise.  Returns (A, b [d, 1], x*)."""
    signs, lengths = PAPER_KINDS[kind]
    rng = np.random.default_rng(np.random.SeedSequence([11, kind, int(round(100 * sparsity)),
                                                        seed]))
    lo = 0.0 if signs == "+" else -1.0
    A = rng.uniform(lo, 1.0, (d, n))
    nz = int(round(sparsity * d))
    if nz:
        for j in range(n):
            A[rng.permutation(d)[:nz], j] = 0.0
    norms = np.linalg.norm(A, axis=0)
    norms[norms == 0] = 1.0
    if lengths == "SAM":
        target = np.ones(n)
    elif lengths == "RAN":
        target = 1.0 - rng.random(n)            # U(0, 1]
    else:
        target = 10.0 ** rng.uniform(-2.0, 2.0, n)
    A *= (target / norms)[None, :]
    x = rng.uniform(lo, 1.0, n)
    x[rng.permutation(n)[: int(round(sparsity * n))]] = 0.0
    A = A.astype(dtype)
    b = A.astype(np.float64) @ x
    return A, b.reshape(d, 1).astype(dtype), x


def make_nmf(seed: int = 0, m: int = 10000, p: int = 4096, r: int = 256, dtype=np.float32):
    """Data for a nonnegative factorisation: V = max(W* H* + noise, 0) with W* [m, r] U[0,1] with
    30 % zeros per column, H* [r, p] with 70 % zeros per column and Exp(1) nonzeros, noise
    0.01 * RMS(W* H*); the start W0 [m, r] is U[0,1] from its own stream SeedSequence([13, seed]).
    Returns (V, W0, W*, H*)."""
    rng = np.random.default_rng(np.random.SeedSequence([12, seed]))
    Ws = rng.random((m, r))
    for j in range(r):
        Ws[rng.permutation(m)[: int(round(0.3 * m))], j] = 0.0
    Hs = np.zeros((r, p))
    for c in range(p):
        Hs[:, c] = _zero_pattern(rng, r, int(round(0.7 * r)), lambda k: rng.exponential(1.0, k))
    V0 = Ws @ Hs
    rms = float(np.sqrt(np.mean(V0 * V0)))
    V = np.maximum(V0 + rng.normal(0.0, 0.01 * rms, V0.shape), 0.0)
    W0 = np.random.default_rng(np.random.SeedSequence([13, seed])).random((m, r))
    return V.astype(dtype), W0.astype(dtype), Ws, Hs


def make_manyrhs(seed: int = 0, d: int = 10000, n: int = 256, k: int = 4096, dtype=np.float32):
    """Many right-hand sides sharing A (an NMF-style update): A ~ |N(0,1)|, each column of X has
    round(0.8 n) zeros and Gamma(2,1) nonzeros, per-column noise 0.01 * RMS(b0)."""
    rng = np.random.default_rng(seed)
    A = np.abs(rng.standard_normal((d, n))).astype(dtype)
    X = np.zeros((n, k), dtype=np.float64)
    n_zero = int(round(0.8 * n))
    for c in range(k):
        X[:, c] = _zero_pattern(rng, n, n_zero, lambda m: rng.gamma(2.0, 1.0, m))
    B0 = A.astype(np.float64) @ X
    rms = np.sqrt(np.mean(B0 * B0, axis=0))
    B = B0 + rng.standard_normal((d, k)) * (0.01 * rms)[None, :]
    return A, B.astype(dtype), X


def make_batched_problem(i: int, n_lo: int = 16, n_hi: int = 512, dtype=np.float32):
    """Problem i of the uneven batch: n ~ U{n_lo..n_hi}, d = 3n, A ~ U[0,1], round(0.6 n) zeros
    in x with U[0,1] nonzeros, 1 % relative noise."""
    rng = np.random.default_rng(np.random.SeedSequence([0, i]))
    n = int(rng.integers(n_lo, n_hi + 1))
    d = 3 * n
    A = rng.random((d, n)).astype(dtype)
    x = _zero_pattern(rng, n, int(round(0.6 * n)), lambda m: rng.random(m))
    b0 = A.astype(np.float64) @ x
    rms = float(np.sqrt(np.mean(b0 * b0)))
    b = b0 + rng.normal(0.0, 0.01 * rms, size=d)
    return A, b.reshape(d, 1).astype(dtype), x


def batched_sizes(count: int, n_lo: int = 16, n_hi: int = 512):
    """The n of each problem of the uneven batch, without drawing the matrices."""
    out = np.empty(count, dtype=np.int64)
    for i in range(count):
        rng = np.random.default_rng(np.random.SeedSequence([0, i]))
        out[i] = int(rng.integers(n_lo, n_hi + 1))
    return out


def make_warm_matrix(d: int = 4096, n: int = 256, dtype=np.float32):
    """Fixed dictionary of the warm-start workload: A ~ |N(0,1)|, seed 0."""
    rng = np.random.default_rng(0)
    return np.abs(rng.standard_normal((d, n))).astype(dtype)


def make_warm_codes(n: int, count: int, split: int, start: int = 0) -> np.ndarray:
    """Codes x [n, count] of the warm-start workload (85 % zeros, Gamma(1.5, 1) nonzeros).
    split 0 = training set, split 1 = held-out evaluation set.  Column j is sample start + j of
    its split (each sample has its own counter-derived stream, so any slice can be drawn
    alone)."""
    n_zero = int(round(0.85 * n))
    X = np.zeros((n, count), dtype=np.float64)
    for j in range(count):
        rng = np.random.default_rng(np.random.SeedSequence([5, split, start + j]))
        X[:, j] = _zero_pattern(rng, n, n_zero, lambda m: rng.gamma(1.5, 1.0, m))
    return X


def make_warm_rhs(A: np.ndarray, count: int, split: int, start: int = 0, dtype=np.float32):
    """Noiseless right-hand sides b = A x for the warm-start workload (codes from
    make_warm_codes), b formed in FP64 and rounded to dtype."""
    X = make_warm_codes(A.shape[1], count, split, start)
    B = A.astype(np.float64) @ X
    return B.astype(dtype), X


MLP_SHAPES = [((256, 1024), True), ((1024,), False), ((1024, 1024), True), ((1024,), False),
              ((1024, 256), True), ((256,), False)]


def make_mlp_params(seed: int = 0) -> np.ndarray:
    """Initial FP32 parameters of the warm-start network in the library's flat layout
    (W1, b1, W2, b2, W3, b3): weights U(-1/sqrt(fan_in), 1/sqrt(fan_in)), biases zero."""
    rng = np.random.default_rng(np.random.SeedSequence([7, seed]))
    parts = []
    for shape, is_weight in MLP_SHAPES:
        if is_weight:
            lim = 1.0 / np.sqrt(shape[0])
            parts.append(rng.uniform(-lim, lim, size=shape).reshape(-1))
        else:
            parts.append(np.zeros(shape))
    return np.concatenate(parts).astype(np.float32)
