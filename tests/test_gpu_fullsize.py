"""Parity at the full workload sizes, in the launch configuration the bench
times, on sampled outputs the oracle computes one by one.

* batched 1D: N in {4096, 16384, 65536}, batch = 2^27/N, uniform + 1 % tones
* long 1D: N in {2^20, 2^22, 2^24}, batch {16, 4, 1}, FP16 and split
* batched 2D: 256^2 x 1024, 512^2 x 256, 1024^2 x 64, FP16 and split
* real input: R2C / C2R of 8192 x 16384 and 32768 x 4096 (fused), FP16
* batched 3D: 128^3 x 64 (plane pass + column pass), FP16 and split
Tolerance: relative L2 per transform 5e-3 (FP16), 2e-5 (split)."""
import numpy as np
import pytest

import oracle
from paper_2104_11471_amd import inputs
from tests.gpu_util import FP16_TOL, SPLIT_TOL, log

pytestmark = pytest.mark.gpu


def _run(plan, x):
    import torch
    host = np.stack(x) if isinstance(x, tuple) else x
    t = torch.from_numpy(np.ascontiguousarray(host)).cuda()
    y = plan(t)
    torch.cuda.synchronize()
    return t, y


def _fetch(y, rows, split):
    z = (y[:, rows] if split else y[rows]).cpu().numpy().astype(np.float64)
    if split:
        return (z[0, ..., 0] + 2.0 ** -11 * z[1, ..., 0]) + 1j * (z[0, ..., 1] + 2.0 ** -11 * z[1, ..., 1])
    return z[..., 0] + 1j * z[..., 1]


@pytest.mark.parametrize("n", [4096, 16384, 65536])
def test_batched_1d_full(n):
    from paper_2104_11471_amd import tcfft
    batch = (1 << 27) // n
    log(f"case batched_1d N={n} batch={batch}")
    x, tones = inputs.batched_1d(n, batch, seed=0)
    plan = tcfft.Plan((n,), batch)
    _, y = _run(plan, x)
    rng = np.random.default_rng(n)
    rows = np.unique(np.concatenate([rng.choice(batch, 24, replace=False), tones.rows[:8],
                                     [0, batch - 1]]))
    z = _fetch(y, rows, False) * 2.0 ** plan.scale_log2
    ref = oracle.fft(oracle.from_half(x[rows]), -1)
    e = oracle.rel_l2(z, ref)
    log(f"  max rel L2 {e.max():.3e} over {len(rows)} rows")
    assert e.max() <= FP16_TOL
    for r, f in zip(tones.rows[:8], tones.freqs[:8]):
        i = int(np.where(rows == r)[0][0])
        assert int(np.argmax(np.abs(z[i]))) == int(f)


@pytest.mark.parametrize("prec", ["fp16", "split"])
@pytest.mark.parametrize("n,batch", [(1 << 20, 16), (1 << 22, 4), (1 << 24, 1)])
def test_long_1d_full(n, batch, prec):
    from paper_2104_11471_amd import tcfft
    split = prec == "split"
    log(f"case long_1d N={n} batch={batch} prec={prec}")
    x, bins, amps = inputs.long_1d(n, batch, seed=0, as_split=split)
    plan = tcfft.Plan((n,), batch, precision=prec)
    _, y = _run(plan, x)
    rows = np.array(sorted({0, batch - 1, batch // 2}))
    z = _fetch(y, rows, split) * 2.0 ** plan.scale_log2
    xin = oracle.from_split(x[0][rows], x[1][rows]) if split else oracle.from_half(x[rows])
    ref = oracle.fft(xin, -1)
    e = oracle.rel_l2(z, ref)
    log(f"  max rel L2 {e.max():.3e}  S={plan.scale_log2}")
    assert e.max() <= (SPLIT_TOL if split else FP16_TOL)
    # the injected on-grid sinusoids stand out at their bins
    for i, r in enumerate(rows):
        top = np.argsort(np.abs(z[i]))[-8:]
        strong = bins[r][amps[r] > 0.2]
        assert set(strong.tolist()) <= set(top.tolist())


@pytest.mark.parametrize("prec", ["fp16", "split"])
@pytest.mark.parametrize("s,batch", [(256, 1024), (512, 256), (1024, 64)])
def test_batched_2d_full(s, batch, prec):
    from paper_2104_11471_amd import tcfft
    split = prec == "split"
    log(f"case smooth_2d {s}x{s} batch={batch} prec={prec}")
    x = inputs.smooth_2d(s, s, batch, seed=0, as_split=split)
    plan = tcfft.Plan((s, s), batch, precision=prec)
    _, y = _run(plan, x)
    rows = np.array([0, 1, batch // 2, batch - 1])
    z = _fetch(y, rows, split) * 2.0 ** plan.scale_log2
    xin = oracle.from_split(x[0][rows], x[1][rows]) if split else oracle.from_half(x[rows])
    ref = oracle.fft2(xin, -1)
    e = oracle.rel_l2(z, ref, axis=(-2, -1))
    log(f"  max rel L2 {e.max():.3e}")
    assert e.max() <= (SPLIT_TOL if split else FP16_TOL)


@pytest.mark.parametrize("n,batch", [(8192, 16384), (32768, 4096)])
def test_real_full(n, batch):
    """R2C then C2R at the bench's real workload sizes; sampled rows against
    the oracle's rfft, and the round trip against N x."""
    import torch
    from paper_2104_11471_amd import tcfft
    log(f"case real N={n} batch={batch}")
    m = n // 2
    x = inputs.uniform((batch, m), 5).reshape(batch, n)
    f = tcfft.Plan((n,), batch, tcfft.FORWARD, flags=tcfft.FLAG_REAL)
    i = tcfft.Plan((n,), batch, tcfft.INVERSE, flags=tcfft.FLAG_REAL)
    xd = torch.from_numpy(x).cuda()
    spec = f(xd)
    back = i(spec)
    torch.cuda.synchronize()
    rows = np.unique(np.concatenate([np.random.default_rng(n).choice(batch, 16, replace=False),
                                     [0, batch - 1]]))
    z = _fetch(spec, rows, False) * 2.0 ** f.scale_log2
    e = oracle.rel_l2(z, oracle.rfft(x[rows].astype(np.float64)))
    y = back[rows].cpu().numpy().astype(np.float64) * 2.0 ** (f.scale_log2 + i.scale_log2)
    e2 = oracle.rel_l2(y, n * x[rows].astype(np.float64))
    log(f"  max rel L2 {e.max():.3e} (R2C), {e2.max():.3e} (round trip) over {len(rows)} rows")
    assert e.max() <= FP16_TOL and e2.max() <= 2 * FP16_TOL


@pytest.mark.parametrize("prec", ["fp16", "split"])
def test_3d_full(prec):
    from paper_2104_11471_amd import tcfft
    dims, batch = (128, 128, 128), 64
    split = prec == "split"
    log(f"case 3d {dims} x {batch} prec={prec}")
    if split:
        x = inputs.to_split(inputs.uniform_f64((batch,) + dims, 0))
    else:
        x = inputs.uniform((batch,) + dims, 0)
    plan = tcfft.Plan(dims, batch, precision=prec)
    assert [p["kernel"] for p in plan.describe()["passes"]] == ["plane", "col"]
    _, y = _run(plan, x)
    rows = np.array([0, 17, batch - 1])
    z = _fetch(y, rows, split) * 2.0 ** plan.scale_log2
    xin = oracle.from_split(x[0][rows], x[1][rows]) if split else oracle.from_half(x[rows])
    e = oracle.rel_l2(z, oracle.fft3(xin), axis=(-3, -2, -1))
    log(f"  max rel L2 {e.max():.3e} over {len(rows)} arrays")
    assert e.max() <= (SPLIT_TOL if split else FP16_TOL)
