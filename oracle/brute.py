"""Independent brute-force DFTs in numpy -- TEST INFRASTRUCTURE ONLY.

These exist only to pin the C oracle (``oracle/tcfft_oracle.c``) on tiny
inputs; they share nothing with it.  Eq. (1) of the tcFFT paper is a
matrix-vector product with the DFT matrix W[k, n] = exp(sign*2*pi*i*n*k/N);
here that matrix is built with the exponent reduced modulo N in integers and
multiplied with numpy, and a second form sums the terms in pure-Python loops.
``dft_longdouble`` evaluates the same sum in extended precision
(``np.longdouble``), to measure the FP64 oracle's own rounding error.
"""
from __future__ import annotations

import math

import numpy as np


def dft_matrix(n: int, sign: int = -1) -> np.ndarray:
    k = np.arange(n).reshape(-1, 1)
    j = np.arange(n).reshape(1, -1)
    e = (k * j) % n
    return np.exp(sign * 2j * np.pi * e / n)


def dft(x, sign: int = -1) -> np.ndarray:
    """Eq. (1) over the last axis as a product with the DFT matrix."""
    x = np.asarray(x, dtype=np.complex128)
    n = x.shape[-1]
    return x @ dft_matrix(n, sign).T


def dft_loops(x, sign: int = -1) -> list:
    """Eq. (1) summed term by term with Python complex numbers (tiny N only)."""
    n = len(x)
    out = []
    for k in range(n):
        s = 0j
        for j in range(n):
            ang = sign * 2.0 * math.pi * ((j * k) % n) / n
            s += complex(x[j]) * complex(math.cos(ang), math.sin(ang))
        out.append(s)
    return out


def dft2(x, sign: int = -1) -> np.ndarray:
    """2D DFT over the last two axes as the double sum of its definition:
    X[k1, k2] = sum_{n1, n2} x[n1, n2] W_nx^{n1 k1} W_ny^{n2 k2}."""
    x = np.asarray(x, dtype=np.complex128)
    nx, ny = x.shape[-2], x.shape[-1]
    wx = dft_matrix(nx, sign)
    wy = dft_matrix(ny, sign)
    return np.einsum("ab,...bc,dc->...ad", wx, x, wy)


def dft_longdouble(x, sign: int = -1):
    """Eq. (1) in extended precision; returns (re, im) as np.longdouble arrays."""
    x = np.asarray(x, dtype=np.complex128)
    n = x.shape[-1]
    xr = x.real.astype(np.longdouble)
    xi = x.imag.astype(np.longdouble)
    two_pi = np.longdouble(2) * np.arccos(np.longdouble(-1))
    j = np.arange(n)
    re = np.empty(n, dtype=np.longdouble)
    im = np.empty(n, dtype=np.longdouble)
    for k in range(n):
        e = ((j * k) % n).astype(np.longdouble)
        ang = np.longdouble(sign) * two_pi * e / np.longdouble(n)
        c = np.cos(ang)
        s = np.sin(ang)
        re[k] = np.sum(xr * c - xi * s)
        im[k] = np.sum(xr * s + xi * c)
    return re, im
