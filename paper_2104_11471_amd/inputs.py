"""Seeded synthetic inputs shaped like the paper's workloads.

This module holds no transform arithmetic: it only draws numbers.  Both the
GPU path's tests/bench and the CPU oracle take their inputs from here.

Every generator is deterministic in (workload, sizes, seed): the stream is
``numpy.random.default_rng(SeedSequence([tag, *sizes, seed]))``.

Layouts returned
  * FP16 mode: ``float16`` array ``(..., 2)`` -- interleaved (re, im).
  * split mode: a pair ``(hi, lo)`` of such arrays with value ``hi + 2**-11 * lo``
    (``lo`` is the residual scaled by 2**11 so it stays clear of FP16 subnormals).

Workloads (tcFFT paper, Sec. 5.1 draws every input uniformly in [-1, 1]):
  * :func:`uniform` -- re and im i.i.d. U[-1, 1] (the paper's test case).
  * :func:`batched_1d` -- uniform rows plus a 1 % subset of unit pure tones
    x[n] = exp(+2 pi i f n / N), whose forward DFT is N * delta[k - f].
  * :func:`long_1d` -- N(0, 1) noise plus K = 8 on-grid sinusoids with
    amplitude U[0.01, 1] and random phase at distinct bins.
  * :func:`smooth_2d` -- independent re/im Gaussian-filtered noise (sigma = 4 px,
    periodic, truncated at 4 sigma) scaled to [-1, 1], then 5 % salt (+1).
  * :func:`serving_stream` -- Poisson arrivals of a mixed request population.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

SPLIT_LO_SCALE = 2.0 ** -11
_TAGS = {"uniform": 1, "batched_1d": 2, "long_1d": 3, "smooth_2d": 4, "serving": 5, "split": 6}


def rng_for(tag: str, *ints: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([_TAGS[tag], *[int(i) for i in ints]]))


def _interleave_f16(re: np.ndarray, im: np.ndarray) -> np.ndarray:
    out = np.empty(re.shape + (2,), dtype=np.float16)
    out[..., 0] = re
    out[..., 1] = im
    return out


def uniform(shape, seed: int = 0) -> np.ndarray:
    """re, im i.i.d. U[-1, 1], rounded to FP16 (round to nearest even)."""
    shape = tuple(int(s) for s in shape)
    g = rng_for("uniform", *shape, seed)
    v = g.random(shape + (2,), dtype=np.float32)
    v *= 2.0
    v -= 1.0
    return v.astype(np.float16)


def uniform_f64(shape, seed: int = 0) -> np.ndarray:
    """re, im i.i.d. U[-1, 1] in FP64 (source values for split-mode inputs)."""
    shape = tuple(int(s) for s in shape)
    g = rng_for("split", *shape, seed)
    v = g.random(shape + (2,)) * 2.0 - 1.0
    return v[..., 0] + 1j * v[..., 1]


def to_split(z: np.ndarray):
    """complex128 -> (hi, lo) FP16 interleaved pair with z ~= hi + 2^-11 lo."""
    z = np.asarray(z, dtype=np.complex128)
    hr = z.real.astype(np.float16)
    hi_ = z.imag.astype(np.float16)
    lr = ((z.real - hr.astype(np.float64)) * 2048.0).astype(np.float16)
    li = ((z.imag - hi_.astype(np.float64)) * 2048.0).astype(np.float16)
    return _interleave_f16(hr, hi_), _interleave_f16(lr, li)


@dataclass
class Tones:
    rows: np.ndarray   # indices of the tone rows
    freqs: np.ndarray  # on-grid frequency of each tone row
    amp: float = 1.0


def batched_1d(n: int, batch: int, seed: int = 0, tone_frac: float = 0.01):
    """Uniform complex rows plus ``tone_frac`` of rows replaced by unit tones.

    Returns ``(x_f16 (batch, n, 2), Tones)``."""
    x = uniform((batch, n), seed)
    g = rng_for("batched_1d", n, batch, seed)
    ntone = int(round(tone_frac * batch))
    rows = np.sort(g.choice(batch, size=ntone, replace=False)) if ntone else np.zeros(0, np.int64)
    freqs = g.integers(0, n, size=ntone)
    if ntone:
        idx = np.arange(n, dtype=np.int64)
        for r, f in zip(rows, freqs):
            ang = 2.0 * np.pi * ((f * idx) % n) / n
            x[r, :, 0] = np.cos(ang).astype(np.float16)
            x[r, :, 1] = np.sin(ang).astype(np.float16)
    return x, Tones(rows=rows, freqs=freqs)


def long_1d(n: int, batch: int, seed: int = 0, k: int = 8, as_split: bool = False):
    """N(0,1) complex noise plus ``k`` on-grid sinusoids per sequence.

    Returns ``(x, bins (batch, k), amps (batch, k))`` where ``x`` is FP16 (or a
    split pair when ``as_split``)."""
    g = rng_for("long_1d", n, batch, seed)
    z = g.standard_normal((batch, n)) + 1j * g.standard_normal((batch, n))
    bins = np.stack([g.choice(n, size=k, replace=False) for _ in range(batch)])
    amps = g.uniform(0.01, 1.0, size=(batch, k))
    phases = g.uniform(0.0, 2.0 * np.pi, size=(batch, k))
    idx = np.arange(n, dtype=np.int64)
    for b in range(batch):
        for f, a, p in zip(bins[b], amps[b], phases[b]):
            z[b] += a * np.exp(1j * (2.0 * np.pi * ((f * idx) % n) / n + p))
    if as_split:
        return to_split(z), bins, amps
    return _interleave_f16(z.real.astype(np.float16), z.imag.astype(np.float16)), bins, amps


def smooth_2d(nx: int, ny: int, batch: int, seed: int = 0, sigma: float = 4.0,
              salt: float = 0.05, as_split: bool = False):
    """Smooth random fields in [-1, 1] with 5 % salt, (batch, nx, ny)."""
    from scipy.ndimage import gaussian_filter

    g = rng_for("smooth_2d", nx, ny, batch, seed)
    comps = []
    for _ in range(2):
        f = g.standard_normal((batch, nx, ny)).astype(np.float64)
        for b in range(batch):
            f[b] = gaussian_filter(f[b], sigma=sigma, mode="wrap", truncate=4.0)
        lo = f.min(axis=(1, 2), keepdims=True)
        hi = f.max(axis=(1, 2), keepdims=True)
        f = 2.0 * (f - lo) / np.where(hi > lo, hi - lo, 1.0) - 1.0
        m = g.random((batch, nx, ny)) < salt
        f[m] = 1.0
        comps.append(f)
    z = comps[0] + 1j * comps[1]
    if as_split:
        return to_split(z)
    return _interleave_f16(z.real.astype(np.float16), z.imag.astype(np.float16))


@dataclass
class Request:
    rid: int
    t_arrival: float     # seconds from the start of the stream
    rank: int            # 1 or 2
    dims: tuple          # (n,) or (nx, ny)
    batch: int
    split: bool          # split hi+lo FP16 precision when True


def serving_stream(rate_hz: float = 20000.0, duration_s: float = 5.0, seed: int = 0,
                   max_requests: int | None = None):
    """Poisson arrivals of mixed requests:
    60 % 1D with log2 N uniform in {8..16} and batch uniform in [1, 64];
    30 % 2D square in {128, 256, 512} with batch uniform in [1, 32];
    10 % 1D N = 2^20, batch 1; precision 80 % FP16 / 20 % split."""
    g = rng_for("serving", int(rate_hz), int(duration_s * 1000), seed)
    reqs = []
    t = 0.0
    rid = 0
    while True:
        t += g.exponential(1.0 / rate_hz)
        if t >= duration_s or (max_requests is not None and rid >= max_requests):
            break
        u = g.random()
        split = bool(g.random() < 0.2)
        if u < 0.6:
            n = 1 << int(g.integers(8, 17))
            reqs.append(Request(rid, t, 1, (n,), int(g.integers(1, 65)), split))
        elif u < 0.9:
            s = int(g.choice([128, 256, 512]))
            reqs.append(Request(rid, t, 2, (s, s), int(g.integers(1, 33)), split))
        else:
            reqs.append(Request(rid, t, 1, (1 << 20,), 1, split))
        rid += 1
    return reqs
