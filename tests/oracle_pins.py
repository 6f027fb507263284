"""Pins of the FP64 oracle against what the mathematics fixes.

Each ``pin_*`` function takes an :class:`oracle.Oracle` (the real build, or a
deliberately broken copy compiled by ``test_oracle_mutants.py``) and raises
``AssertionError`` when the oracle disagrees with a closed form, an invariant,
brute force or a published error bound.  None of them retypes the oracle's own
formula: each compares against something computed another way.
"""
from __future__ import annotations

import json
import math
import os

import numpy as np

from oracle import brute

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "dft_pairs.json")


def _rng(seed):
    return np.random.default_rng(seed)


def _crandn(g, *shape):
    return g.standard_normal(shape) + 1j * g.standard_normal(shape)


def _rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / max(np.linalg.norm(np.ravel(b)), 1e-300))


def pin_golden_pairs(o):
    """Textbook DFT pairs written out by hand from Eq. (1)."""
    data = json.load(open(GOLDEN))
    for p in data["pairs"]:
        x = np.array([complex(a, b) for a, b in p["x"]])
        X = np.array([complex(a, b) for a, b in p["X"]])
        for name, got in (("fft", o.fft(x)), ("dft_direct", o.dft_direct(x))):
            assert np.allclose(got, X, atol=1e-12), f"{p['name']} via {name}: {got} != {X}"


def pin_delta_and_constant(o):
    """delta[n] -> 1 for every k; 1 -> N delta[k]; both directions."""
    for n in (1, 2, 4, 8, 64, 1024):
        d = np.zeros(n, complex)
        d[0] = 1
        c = np.ones(n, complex)
        nd = np.zeros(n, complex)
        nd[0] = n
        for sign in (-1, 1):
            assert np.allclose(o.fft(d, sign), np.ones(n), atol=1e-13), (n, sign)
            assert np.allclose(o.fft(c, sign), nd, atol=1e-10 * n), (n, sign)
        assert np.allclose(o.dft_direct(d), np.ones(n), atol=1e-12)


def pin_tones(o):
    """x[n] = exp(+2 pi i f n/N) -> N delta[k-f] forward; the conjugate tone
    -> N delta[k-f] inverse.  Pins the sign of the exponent and the index map."""
    for n in (4, 16, 256, 4096):
        idx = np.arange(n)
        for f in sorted({0, 1, 3 % n, n // 2, n - 1, (7 * n) // 13}):
            tone = np.exp(2j * np.pi * ((f * idx) % n) / n)
            ref = np.zeros(n, complex)
            ref[f] = n
            got = o.fft(tone, -1)
            assert np.abs(got - ref).max() < 1e-9 * n, (n, f, "forward")
            got = o.fft(np.conj(tone), +1)
            assert np.abs(got - ref).max() < 1e-9 * n, (n, f, "inverse")
            if n <= 256:
                got = o.dft_direct(tone, -1)
                assert np.abs(got - ref).max() < 1e-9 * n, (n, f, "direct")


def pin_shift_theorem(o):
    """A circular shift by s multiplies bin k by W_N^{k s} (catches index and
    twiddle-exponent mistakes that a tone alone may miss)."""
    g = _rng(11)
    for n in (8, 32, 512):
        x = _crandn(g, n)
        for s in (1, 3, n // 2 + 1):
            k = np.arange(n)
            lhs = o.fft(np.roll(x, s))
            rhs = o.fft(x) * np.exp(-2j * np.pi * ((k * s) % n) / n)
            assert _rel(lhs, rhs) < 1e-13, (n, s)


def pin_parseval_linearity_roundtrip(o):
    g = _rng(5)
    for n in (2, 16, 128, 2048, 1 << 14):
        x = _crandn(g, 3, n)
        y = _crandn(g, 3, n)
        X = o.fft(x)
        # Parseval: N * sum |x|^2 = sum |X|^2
        lhs = n * np.sum(np.abs(x) ** 2, axis=-1)
        rhs = np.sum(np.abs(X) ** 2, axis=-1)
        assert np.allclose(lhs, rhs, rtol=1e-12), n
        # linearity
        a, b = 0.75 - 0.5j, -1.25 + 2j
        assert _rel(o.fft(a * x + b * y), a * X + b * o.fft(y)) < 1e-13, n
        # inverse(forward(x)) = N x
        assert _rel(o.fft(X, +1), n * x) < 1e-13, n


def pin_brute_force_small(o):
    """fft == dft_direct == numpy DFT matrix == Python loops for every N <= 64."""
    g = _rng(3)
    for lg in range(0, 7):
        n = 1 << lg
        x = _crandn(g, n)
        ref = brute.dft(x)
        loops = np.array(brute.dft_loops(x))
        assert _rel(ref, loops) < 1e-13
        for sign in (-1, 1):
            r = brute.dft(x, sign)
            assert _rel(o.fft(x, sign), r) <= 1e-13, (n, sign)
            assert _rel(o.dft_direct(x, sign), r) <= 1e-13, (n, sign)


def pin_batch_independence(o):
    """Row b of a batched call equals the single transform of row b."""
    g = _rng(9)
    for n, batch in ((16, 5), (256, 17), (4096, 3)):
        x = _crandn(g, batch, n)
        X = o.fft(x)
        for b in (0, batch // 2, batch - 1):
            assert _rel(X[b], brute.dft(x[b])) < 1e-12, (n, b)


def pin_error_bound(o):
    """FP64 radix-2 error against an extended-precision DFT of the same input,
    within the published bound for radix-2 Cooley-Tukey (Higham, Accuracy and
    Stability of Numerical Algorithms, 2nd ed., Thm 24.2):
    ||y - X|| / ||X|| <= log2(N) eta / (1 - log2(N) eta),
    eta = mu + gamma_4 (sqrt 2 + mu), mu = twiddle error (<= u for libm), u = 2^-53."""
    u = 2.0 ** -53
    mu = u
    gamma4 = 4 * u / (1 - 4 * u)
    eta = mu + gamma4 * (math.sqrt(2) + mu)
    g = _rng(21)
    for n in (64, 512, 2048):
        x = _crandn(g, n)
        re, im = brute.dft_longdouble(x)
        y = o.fft(x)
        dr = y.real.astype(np.longdouble) - re
        di = y.imag.astype(np.longdouble) - im
        err = float(np.sqrt(np.sum(dr * dr + di * di)) / np.sqrt(np.sum(re * re + im * im)))
        lg = math.log2(n)
        bound = lg * eta / (1 - lg * eta)
        assert err <= bound, (n, err, bound)


def pin_fft2(o):
    """2D: against the double-sum definition (tiny sizes) and separability."""
    g = _rng(13)
    for nx, ny in ((1, 4), (4, 1), (2, 8), (8, 4), (16, 16), (4, 32)):
        x = _crandn(g, 2, nx, ny)
        for sign in (-1, 1):
            assert _rel(o.fft2(x, sign), brute.dft2(x, sign)) < 1e-12, (nx, ny, sign)
    # separability: the transform of an outer product is the outer product of
    # the 1D transforms
    a = _crandn(g, 32)
    b = _crandn(g, 64)
    lhs = o.fft2(np.outer(a, b)[None])[0]
    rhs = np.outer(brute.dft(a), brute.dft(b))
    assert _rel(lhs, rhs) < 1e-12


def pin_merge_eq3(o):
    """Eq. (3) against Eq. (2): feeding the N1 sub-DFTs X_m of x_m[n] = x[n N1 + m]
    into the matrix form reproduces the full N-point DFT, X_out[l][k] = X[l N2 + k]."""
    g = _rng(17)
    for n1, n2 in ((2, 4), (16, 16), (4, 32), (16, 2)):
        n = n1 * n2
        x = _crandn(g, n)
        xin = np.stack([brute.dft(x[m::n1]) for m in range(n1)])
        xout = o.merge(xin)
        assert _rel(xout.reshape(-1), brute.dft(x)) < 1e-12, (n1, n2)


def pin_numpy_library(o):
    """Independent library routine (pocketfft in numpy, FP64)."""
    g = _rng(23)
    for n in (2, 64, 1024, 1 << 16):
        x = _crandn(g, 2, n)
        assert _rel(o.fft(x), np.fft.fft(x)) < 1e-12, n
        assert _rel(o.fft(x, +1), n * np.fft.ifft(x)) < 1e-12, n
    x = _crandn(g, 2, 64, 128)
    assert _rel(o.fft2(x), np.fft.fft2(x)) < 1e-12


def pin_bad_arguments(o):
    """Non-power-of-two sizes and bad signs are refused, not computed."""
    import pytest

    with pytest.raises(ValueError):
        o.fft(np.zeros(12, complex))
    with pytest.raises(ValueError):
        o.fft(np.zeros(16, complex), sign=2)
    with pytest.raises(ValueError):
        o.fft2(np.zeros((1, 6, 8), complex))


ALL_PINS = [pin_golden_pairs, pin_delta_and_constant, pin_tones, pin_shift_theorem,
            pin_parseval_linearity_roundtrip, pin_brute_force_small, pin_batch_independence,
            pin_error_bound, pin_fft2, pin_merge_eq3, pin_numpy_library]
