"""Data movement of a distributed four-step transform around the shard steps
(tcfft_plan_create_shard): which part of x a device holds, the all-to-all,
and where each device's step-2 output sits in X.  Pure index bookkeeping (no
transform arithmetic), shared by the CPU check of the layout algebra and the
GPU parity tests.  Arrays carry a leading plane axis P (1 for FP16, 2 for
split hi/lo) and the batch axis: shape (P, B, points, ...)."""
from __future__ import annotations

import numpy as np


def geometry(n: int, n1: int, g: int):
    m = n // n1
    return m, n1 // g, m // g  # M, n1l, ml


def slab(x, n1: int, nshards: int, shard: int):
    """x: (P, B, N, ...) -> device `shard`'s step-1 input (P, B, N1 * ml, ...):
    x[n1 M + shard ml + m_l] at n1 ml + m_l."""
    p, b, n = x.shape[:3]
    m, _, ml = geometry(n, n1, nshards)
    v = x.reshape(p, b, n1, m, *x.shape[3:])[:, :, :, shard * ml:(shard + 1) * ml]
    return v.reshape(p, b, n1 * ml, *x.shape[3:])


def exchange(step1_out, n: int, n1: int, nshards: int, cat):
    """step1_out[g]: (P, B, N/G, ...) laid out [G][ml][n1l] -> the step-2 input
    of every device h: block h of each device g, concatenated in g order
    ([M][n1l]).  `cat` concatenates along axis 2 (numpy or torch)."""
    m, n1l, ml = geometry(n, n1, nshards)
    recv = []
    for h in range(nshards):
        parts = [s[:, :, h * ml * n1l:(h + 1) * ml * n1l] for s in step1_out]
        recv.append(cat(parts))
    return recv


def assemble(step2_out, n: int, n1: int, nshards: int):
    """step2_out[h]: (P, B, N/G, ...) numpy arrays laid out [M][n1l] ->
    X (P, B, N, ...) with X[k' N1 + h n1l + k1_l] = out_h[k' n1l + k1_l]."""
    m, n1l, ml = geometry(n, n1, nshards)
    p, b = step2_out[0].shape[:2]
    rest = step2_out[0].shape[3:]
    full = np.empty((p, b, m, nshards, n1l) + rest, dtype=step2_out[0].dtype)
    for h, o in enumerate(step2_out):
        full[:, :, :, h] = o.reshape((p, b, m, n1l) + rest)
    return full.reshape((p, b, n) + rest)
