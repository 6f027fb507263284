"""Helpers for GPU parity tests: run a plan on host arrays, compare to the oracle."""
from __future__ import annotations

import sys

import numpy as np

import oracle

FP16_TOL = 5e-3     # relative L2 per transform, FP16 storage
SPLIT_TOL = 2e-5    # relative L2 per transform, split hi+lo FP16
FP32_TOL = 1e-5     # FP32 radix-2 comparator


def log(msg: str) -> None:
    print(msg, flush=True)
    sys.stdout.flush()


def run_plan(plan, x, inplace: bool = False):
    """x: float16 (B, *dims, 2) | split pair (hi, lo) | float32 (B, n, 2).
    Returns the output as complex128 scaled back by 2^S."""
    import torch

    if isinstance(x, tuple):
        host = np.stack([x[0], x[1]])
    else:
        host = x
    t = torch.from_numpy(np.ascontiguousarray(host)).cuda()
    out = t if inplace else torch.empty_like(t)
    plan(t, out)
    torch.cuda.synchronize()
    y = out.cpu().numpy().astype(np.float64)
    scale = 2.0 ** plan.scale_log2
    if isinstance(x, tuple):
        z = (y[0, ..., 0] + 2.0 ** -11 * y[1, ..., 0]) + 1j * (y[0, ..., 1] + 2.0 ** -11 * y[1, ..., 1])
    else:
        z = y[..., 0] + 1j * y[..., 1]
    return z * scale


def to_complex(x):
    if isinstance(x, tuple):
        return oracle.from_split(x[0], x[1])
    if x.dtype == np.float16:
        return oracle.from_half(x)
    return x[..., 0].astype(np.float64) + 1j * x[..., 1].astype(np.float64)


def reference(x, rank: int, sign: int):
    z = to_complex(x)
    return oracle.fft(z, sign) if rank == 1 else oracle.fft2(z, sign)


def rel_err(y, ref, rank: int):
    axes = -1 if rank == 1 else (-2, -1)
    return oracle.rel_l2(y, ref, axis=axes)
