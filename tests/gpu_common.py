"""Helpers of the GPU parity tests: device transfer, the oracle handle and tolerance formulas."""
from __future__ import annotations

import sys

import numpy as np
import torch

from oracle import oracle as O

DEV = "cuda"
U_BF16X3 = 2.0 ** -15   # per-product error of hi*hi + hi*lo + lo*hi (dropped lo*lo and the
                        # bf16 rounding of lo), relative to |a_r b_r|
U_F32 = 2.0 ** -24


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def orc():
    return O.load()


def gram_abs_tol(d: int, mode: str) -> float:
    """Bound on |Q_gpu - Q_exact| for entries of a cosine matrix (|Q_ij| <= 1): per-product
    splitting error plus FP32 accumulation over d terms, both relative to sum |a_ri a_rj|, which
    Cauchy-Schwarz bounds by ||A_i|| ||A_j||."""
    per = {"bf16x3": U_BF16X3, "fp32": U_F32, "fp64": 2.0 ** -53}[mode]
    acc = (U_F32 if mode != "fp64" else 2.0 ** -53) * d
    return 2.0 * (per + acc)
