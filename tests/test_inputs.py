"""Seeded generators: deterministic, right shapes/distributions, tones exact."""
import hashlib

import numpy as np

from paper_2104_11471_amd import inputs


def _h(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def test_uniform_deterministic_and_moments():
    a = inputs.uniform((64, 256), seed=0)
    b = inputs.uniform((64, 256), seed=0)
    c = inputs.uniform((64, 256), seed=1)
    assert a.dtype == np.float16 and a.shape == (64, 256, 2)
    assert _h(a) == _h(b) and _h(a) != _h(c)
    f = a.astype(np.float64)
    assert f.min() >= -1 and f.max() <= 1
    assert abs(f.mean()) < 0.02 and abs(f.var() - 1 / 3) < 0.02


def test_batched_1d_tones():
    x, tones = inputs.batched_1d(4096, 200, seed=0)
    assert x.shape == (200, 4096, 2) and len(tones.rows) == 2
    n = np.arange(4096)
    for r, f in zip(tones.rows, tones.freqs):
        z = x[r, :, 0].astype(np.float64) + 1j * x[r, :, 1].astype(np.float64)
        ref = np.exp(2j * np.pi * ((f * n) % 4096) / 4096)
        assert np.abs(z - ref).max() < 1e-3


def test_long_1d_and_split():
    (hi, lo), bins, amps = inputs.long_1d(1024, 2, seed=0, as_split=True)
    assert hi.shape == lo.shape == (2, 1024, 2) and bins.shape == (2, 8)
    assert np.all((amps >= 0.01) & (amps <= 1.0))
    assert all(len(set(b)) == 8 for b in bins)
    z = inputs.uniform_f64((3, 64))
    h, l = inputs.to_split(z)
    back = (h.astype(np.float64) + 2.0 ** -11 * l.astype(np.float64))
    back = back[..., 0] + 1j * back[..., 1]
    assert np.abs(back - z).max() < 2.0 ** -22


def test_smooth_2d_range_and_salt():
    x = inputs.smooth_2d(64, 64, 2, seed=0)
    f = x.astype(np.float64)
    assert f.min() >= -1 and f.max() <= 1
    frac = np.mean(f[..., 0] == 1.0)
    assert 0.03 < frac < 0.08


def test_serving_mix():
    reqs = inputs.serving_stream(rate_hz=20000, duration_s=0.5, seed=0)
    assert 9000 < len(reqs) < 11000
    t = np.array([r.t_arrival for r in reqs])
    assert np.all(np.diff(t) > 0)
    kinds = np.array([0 if (r.rank == 1 and r.dims[0] < (1 << 20)) else (1 if r.rank == 2 else 2)
                      for r in reqs])
    frac = np.bincount(kinds, minlength=3) / len(reqs)
    assert abs(frac[0] - 0.6) < 0.03 and abs(frac[1] - 0.3) < 0.03 and abs(frac[2] - 0.1) < 0.02
    assert abs(np.mean([r.split for r in reqs]) - 0.2) < 0.03
