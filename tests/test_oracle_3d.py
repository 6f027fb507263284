"""The oracle's 3D transform against its pins: the triple sum of Eq. (1)
evaluated by brute force on tiny shapes, numpy's fftn (an independent
library routine), a plane wave (closed form) and the inverse round trip."""
import numpy as np
import pytest

import oracle
from oracle import brute


def test_fft3_brute_force():
    rng = np.random.default_rng(5)
    x = rng.standard_normal((2, 4, 8, 16)) + 1j * rng.standard_normal((2, 4, 8, 16))
    fx, fy, fz = (brute.dft_matrix(n) for n in (4, 8, 16))
    ref = np.einsum("ka,lb,mc,nabc->nklm", fx, fy, fz, x)
    assert np.max(np.abs(oracle.fft3(x) - ref)) < 1e-10


@pytest.mark.parametrize("shape", [(16, 16, 16), (32, 16, 64), (16, 64, 32)])
def test_fft3_matches_library(shape):
    rng = np.random.default_rng(sum(shape))
    x = rng.standard_normal((2,) + shape) + 1j * rng.standard_normal((2,) + shape)
    for sign, ref in ((-1, np.fft.fftn(x, axes=(-3, -2, -1))),
                      (1, np.fft.ifftn(x, axes=(-3, -2, -1)) * np.prod(shape))):
        y = oracle.fft3(x, sign)
        assert np.max(np.abs(y - ref)) <= 1e-12 * np.prod(shape)


def test_fft3_plane_wave():
    nx, ny, nz = 16, 32, 64
    f = (3, 17, 40)
    gx, gy, gz = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    x = np.exp(2j * np.pi * (f[0] * gx / nx + f[1] * gy / ny + f[2] * gz / nz))[None]
    y = oracle.fft3(x)
    n = nx * ny * nz
    assert abs(y[0][f] - n) < 1e-8 * n
    y[0][f] = 0
    assert np.max(np.abs(y)) < 1e-8 * n


def test_fft3_round_trip():
    x = np.random.default_rng(2).standard_normal((1, 16, 16, 32)) + 0j
    assert np.max(np.abs(oracle.fft3(oracle.fft3(x), +1) - x * 16 * 16 * 32)) < 1e-9
