"""FP64 CPU oracle for the batched complex FFT -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s ``cpu_baseline``
leg may import this package.  The product path never imports it; it shares no
code with ``paper_2104_11471_amd``.

Functions (tcFFT paper, Sec. 2.1 and Sec. 3.1):

* :func:`dft_direct` -- Eq. (1) evaluated as written, O(N^2) (C, FP64).
* :func:`fft` -- Eq. (2) applied recursively with N1 = 2 (iterative radix-2
  decimation in time, FP64, libm twiddles per index), batched.
* :func:`fft2` -- rows then columns of a row-major array (Sec. 3.1).
* :func:`merge` -- one merging process in the matrix form of Eq. (3).
* :func:`fft3` -- Eq. (1) over three indices of a row-major array, evaluated
  as 1D transforms of :func:`fft` along each axis (the sum is separable).
* :func:`rfft`, :func:`irfft` -- Eq. (1) for a real sequence (the spectrum's
  first N/2 + 1 bins) and its inverse from those bins (Hermitian extension,
  then the unnormalised inverse sum, real part); both by definition on top of
  :func:`fft`.
* :mod:`oracle.brute` -- an independent pure-numpy DFT (explicit sums / the DFT
  matrix), used only to pin the C routines on tiny inputs.

Conventions: ``sign=-1`` is the forward transform of Eq. (1); ``sign=+1`` is the
inverse, read as the same unnormalised sum with the opposite sign (the paper
does not state it), so ``fft(fft(x, -1), +1) == N * x``.

Split hi+lo inputs are read as ``hi + 2**-11 * lo`` exactly in FP64
(:func:`from_split`); FP16 inputs are upcast exactly (:func:`from_half`).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tcfft_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

SPLIT_LO_SCALE = 2.0 ** -11


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (plain -O2, OpenMP, no intrinsics)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class Oracle:
    """ctypes view of one build of the C oracle (the default build, or a
    mutant compiled by the pin-strength tests)."""

    def __init__(self, libpath: str):
        lib = ctypes.CDLL(libpath)
        dp = ctypes.POINTER(ctypes.c_double)
        i64 = ctypes.c_int64
        lib.oracle_dft_direct.argtypes = [dp, dp, i64, ctypes.c_int]
        lib.oracle_fft.argtypes = [dp, dp, i64, i64, ctypes.c_int, ctypes.c_int]
        lib.oracle_fft2.argtypes = [dp, dp, i64, i64, i64, ctypes.c_int, ctypes.c_int]
        lib.oracle_merge.argtypes = [dp, dp, i64, i64, ctypes.c_int]
        lib.oracle_max_threads.argtypes = []
        for f in (lib.oracle_dft_direct, lib.oracle_fft, lib.oracle_fft2, lib.oracle_merge,
                  lib.oracle_max_threads):
            f.restype = ctypes.c_int
        self.lib = lib

    def max_threads(self) -> int:
        return int(self.lib.oracle_max_threads())

    def dft_direct(self, x, sign: int = -1) -> np.ndarray:
        """Eq. (1) as an O(N^2) sum over the last axis."""
        x = _as_c128(x)
        out = np.empty_like(x)
        flat_in = x.reshape(-1, x.shape[-1])
        flat_out = out.reshape(-1, x.shape[-1])
        for i in range(flat_in.shape[0]):
            row = np.ascontiguousarray(flat_in[i])
            res = np.empty_like(row)
            if self.lib.oracle_dft_direct(_ptr(row), _ptr(res), row.shape[0], sign) != 0:
                raise ValueError("oracle_dft_direct: bad argument")
            flat_out[i] = res
        return out

    def fft(self, x, sign: int = -1, threads: int = 0) -> np.ndarray:
        """Batched radix-2 FFT over the last axis (power-of-two length)."""
        x = _as_c128(x)
        n = x.shape[-1]
        batch = x.size // n if n else 0
        out = np.empty_like(x)
        if self.lib.oracle_fft(_ptr(x), _ptr(out), n, batch, sign, threads) != 0:
            raise ValueError(f"oracle_fft: bad argument (n={n}, batch={batch}, sign={sign})")
        return out

    def fft2(self, x, sign: int = -1, threads: int = 0) -> np.ndarray:
        """Batched 2D FFT over the last two axes (rows, then columns)."""
        x = _as_c128(x)
        nx, ny = x.shape[-2], x.shape[-1]
        batch = x.size // (nx * ny)
        out = np.empty_like(x)
        if self.lib.oracle_fft2(_ptr(x), _ptr(out), nx, ny, batch, sign, threads) != 0:
            raise ValueError("oracle_fft2: bad argument")
        return out

    def merge(self, xin, sign: int = -1) -> np.ndarray:
        """Eq. (3): X_out = F_{N1} . (T (.) X_in) for an N1-by-N2 matrix X_in."""
        xin = _as_c128(xin)
        n1, n2 = xin.shape
        out = np.empty_like(xin)
        if self.lib.oracle_merge(_ptr(xin), _ptr(out), n1, n2, sign) != 0:
            raise ValueError("oracle_merge: bad argument")
        return out


def _as_c128(x) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(x, dtype=np.complex128))


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def default() -> Oracle:
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        _lib = Oracle(_LIB)
    return _lib


def max_threads() -> int:
    return default().max_threads()


def dft_direct(x, sign: int = -1) -> np.ndarray:
    return default().dft_direct(x, sign)


def fft(x, sign: int = -1, threads: int = 0) -> np.ndarray:
    return default().fft(x, sign, threads)


def fft2(x, sign: int = -1, threads: int = 0) -> np.ndarray:
    return default().fft2(x, sign, threads)


def merge(xin, sign: int = -1) -> np.ndarray:
    return default().merge(xin, sign)


def fft3(x, sign: int = -1, threads: int = 0) -> np.ndarray:
    """Batched 3D DFT over the last three axes: the triple sum factors into
    1D transforms along z (last axis), then y, then x."""
    z = np.asarray(x, dtype=np.complex128)
    assert z.ndim >= 3
    for ax in (-1, -2, -3):
        t = np.ascontiguousarray(np.moveaxis(z, ax, -1))
        t = fft(t.reshape(-1, t.shape[-1]), sign, threads).reshape(t.shape)
        z = np.moveaxis(t, -1, ax)
    return np.ascontiguousarray(z)


def rfft(x, threads: int = 0) -> np.ndarray:
    """Eq. (1) for real x (..., N): bins 0..N/2 of the complex DFT of x + 0i."""
    x = np.asarray(x, dtype=np.float64)
    n = x.shape[-1]
    return fft(x.astype(np.complex128), -1, threads)[..., : n // 2 + 1]


def irfft(X, n: int, threads: int = 0) -> np.ndarray:
    """Unnormalised inverse of :func:`rfft`: the spectrum of a real sequence
    is Hermitian, Y[N - k] = conj(Y[k]), so bins 0..N/2 fix all N; X[0] and
    X[N/2] of a real sequence are real, their imaginary parts are dropped.
    Returns sum_k Y[k] W_N^{-nk} (= N x for X = rfft(x))."""
    X = np.asarray(X, dtype=np.complex128)
    m = n // 2
    assert X.shape[-1] == m + 1
    Y = np.zeros(X.shape[:-1] + (n,), dtype=np.complex128)
    Y[..., : m + 1] = X
    Y[..., 0] = X[..., 0].real
    Y[..., m] = X[..., m].real
    Y[..., m + 1:] = np.conj(X[..., 1:m][..., ::-1])
    return fft(Y, +1, threads).real


def from_half(a: np.ndarray) -> np.ndarray:
    """FP16 interleaved (..., 2) -> exact complex128."""
    a = np.asarray(a)
    assert a.dtype == np.float16 and a.shape[-1] == 2
    f = a.astype(np.float64)
    return f[..., 0] + 1j * f[..., 1]


def from_split(hi: np.ndarray, lo: np.ndarray) -> np.ndarray:
    """Split hi+lo FP16 pair -> exact complex128 value hi + 2^-11 * lo."""
    return from_half(hi) + SPLIT_LO_SCALE * from_half(lo)


def rel_l2(y: np.ndarray, ref: np.ndarray, axis=-1) -> np.ndarray:
    """Per-transform relative L2 error ||y - ref|| / ||ref|| along ``axis``
    (an all-zero reference row counts as error 0 only if y is zero too)."""
    num = np.sqrt(np.sum(np.abs(y - ref) ** 2, axis=axis))
    den = np.sqrt(np.sum(np.abs(ref) ** 2, axis=axis))
    with np.errstate(divide="ignore", invalid="ignore"):
        e = np.where(den > 0, num / np.where(den > 0, den, 1.0), np.where(num > 0, np.inf, 0.0))
    return e


def eq5_error(y: np.ndarray, ref: np.ndarray) -> float:
    """Secondary accuracy reading of Eq. (5): the mean over bins with a non-zero
    reference of |ref - y| / |ref|.  Reported only, never a gate."""
    y = np.asarray(y).ravel()
    ref = np.asarray(ref).ravel()
    m = np.abs(ref) > 0
    return float(np.mean(np.abs(ref[m] - y[m]) / np.abs(ref[m]))) if m.any() else 0.0
