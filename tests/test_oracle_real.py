"""The oracle's real-input transforms against their pins: closed-form spectra of
tones and impulses, numpy's rfft/irfft (an independent library routine for
this special case of Eq. 1), brute-force sums on tiny sizes, and the round
trip."""
import numpy as np
import pytest

import oracle
from oracle import brute


@pytest.mark.parametrize("n", [32, 64, 256, 4096])
def test_rfft_matches_library(n):
    x = np.random.default_rng(n).standard_normal((3, n))
    X = oracle.rfft(x)
    assert X.shape == (3, n // 2 + 1)
    ref = np.fft.rfft(x)
    assert np.max(np.abs(X - ref)) <= 1e-12 * n


@pytest.mark.parametrize("n", [32, 128])
def test_rfft_brute_force(n):
    x = np.random.default_rng(7).standard_normal(n)
    full = brute.dft(x.astype(np.complex128))
    assert np.max(np.abs(oracle.rfft(x) - full[: n // 2 + 1])) <= 1e-12 * n


@pytest.mark.parametrize("n,f", [(64, 1), (64, 5), (1024, 100), (1024, 511)])
def test_rfft_tones(n, f):
    """cos(2 pi f m / N) -> N/2 at bin f; sin -> -i N/2 at bin f."""
    m = np.arange(n)
    Xc = oracle.rfft(np.cos(2 * np.pi * f * m / n))
    Xs = oracle.rfft(np.sin(2 * np.pi * f * m / n))
    ec = np.zeros(n // 2 + 1, complex)
    ec[f] = n / 2
    es = np.zeros(n // 2 + 1, complex)
    es[f] = -0.5j * n
    assert np.max(np.abs(Xc - ec)) < 1e-9 and np.max(np.abs(Xs - es)) < 1e-9


def test_rfft_nyquist_and_impulse():
    n = 256
    m = np.arange(n)
    X = oracle.rfft((-1.0) ** m)
    e = np.zeros(n // 2 + 1, complex)
    e[n // 2] = n
    assert np.max(np.abs(X - e)) < 1e-9
    x = np.zeros(n)
    x[3] = 1.0
    k = np.arange(n // 2 + 1)
    assert np.max(np.abs(oracle.rfft(x) - np.exp(-2j * np.pi * 3 * k / n))) < 1e-12


@pytest.mark.parametrize("n", [32, 512, 8192])
def test_irfft_matches_library(n):
    rng = np.random.default_rng(n + 1)
    X = rng.standard_normal((2, n // 2 + 1)) + 1j * rng.standard_normal((2, n // 2 + 1))
    y = oracle.irfft(X, n)
    ref = n * np.fft.irfft(X, n)  # numpy drops Im X[0], Im X[N/2] as well
    assert np.max(np.abs(y - ref)) <= 1e-11 * n


def test_irfft_tone_and_round_trip():
    n = 128
    X = np.zeros(n // 2 + 1, complex)
    X[9] = 1.0  # one bin and its mirror: 2 cos(2 pi 9 m / N)
    m = np.arange(n)
    assert np.max(np.abs(oracle.irfft(X, n) - 2 * np.cos(2 * np.pi * 9 * m / n))) < 1e-12
    x = np.random.default_rng(3).standard_normal((4, n))
    assert np.max(np.abs(oracle.irfft(oracle.rfft(x), n) - n * x)) < 1e-10
