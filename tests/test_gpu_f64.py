"""FP64 matrix-core path (v_mfma_f64_16x16x4f64) against the FP64 oracle.

Tolerance: every stage rounds once per product and sum in FP64 (unit
roundoff u = 2^-53) and the twiddles carry about one ulp; the relative L2
error of a log16-depth decomposition grows like u * O(log2 N), about 1e-15 at
N = 4096.  The bound used is 1e-13, a hundred times that, still ten orders of
magnitude below the FP16 path's and seven below the split path's."""
import numpy as np
import pytest

import oracle
from paper_2104_11471_amd import inputs
from tests.gpu_util import log

pytestmark = pytest.mark.gpu

F64_TOL = 1e-13
SIZES = [16, 32, 64, 128, 256, 512, 1024, 2048, 4096]


def _run(n, batch, direction, seed, inplace=False):
    import torch
    from paper_2104_11471_amd import tcfft
    z = inputs.uniform_f64((batch, n), seed)
    x = np.stack([z.real, z.imag], -1)
    p = tcfft.Plan((n,), batch, direction, "fp64")
    assert p.scale_log2 == 0
    xd = torch.from_numpy(x).cuda()
    yd = xd if inplace else torch.empty_like(xd)
    p(xd, yd)
    torch.cuda.synchronize()
    y = yd.cpu().numpy()
    return z, y[..., 0] + 1j * y[..., 1]


@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("direction", [-1, 1])
def test_fp64_matches_oracle(n, direction):
    # batches: one transform, and one that ends inside a workgroup's tile
    for batch in (1, 4096 // n + 3):
        log(f"fp64 n={n} batch={batch} dir={direction}")
        z, y = _run(n, batch, direction, seed=n + batch)
        ref = oracle.fft(z, direction)
        e = oracle.rel_l2(y, ref)
        assert e.max() < F64_TOL, (n, batch, float(e.max()))


def test_fp64_in_place_and_full_tiles():
    for n in (256, 4096):
        batch = 2 * 4096 // n * 8
        z, y = _run(n, batch, -1, seed=7, inplace=True)
        e = oracle.rel_l2(y, oracle.fft(z, -1))
        log(f"fp64 in place n={n} batch={batch}: max rel L2 {e.max():.2e}")
        assert e.max() < F64_TOL


def test_fp64_closed_forms():
    """A unit impulse at n0 transforms to W_N^{k n0} exactly up to twiddle
    rounding; a constant to N at bin 0."""
    import torch
    from paper_2104_11471_amd import tcfft
    n = 1024
    x = np.zeros((2, n, 2))
    x[0, 5, 0] = 1.0
    x[1, :, 0] = 1.0
    p = tcfft.Plan((n,), 2, -1, "fp64")
    xd = torch.from_numpy(x).cuda()
    y = torch.empty_like(xd)
    p(xd, y)
    y = y.cpu().numpy()
    k = np.arange(n)
    w = np.exp(-2j * np.pi * k * 5 / n)
    assert np.abs((y[0, :, 0] + 1j * y[0, :, 1]) - w).max() < 1e-14
    c = y[1, :, 0] + 1j * y[1, :, 1]
    assert abs(c[0] - n) < 1e-11 and np.abs(c[1:]).max() < 1e-11


def test_fp64_in_exec_many():
    import torch
    from paper_2104_11471_amd import tcfft
    jobs = [((4096,), 3, "fp64"), ((512,), 9, "fp16"), ((64,), 100, "fp64")]
    plans, xs, ys = [], [], []
    for i, (dims, b, prec) in enumerate(jobs):
        plans.append(tcfft.Plan(dims, b, precision=prec))
        if prec == "fp64":
            z = inputs.uniform_f64((b,) + dims, 60 + i)
            xs.append(torch.from_numpy(np.stack([z.real, z.imag], -1)).cuda())
        else:
            xs.append(torch.from_numpy(inputs.uniform((b,) + dims, 60 + i)).cuda())
        ys.append(torch.empty_like(xs[-1]))
    tcfft.exec_many(plans, xs, ys)
    alone = [torch.empty_like(x) for x in xs]
    for p, x, o in zip(plans, xs, alone):
        p(x, o)
    torch.cuda.synchronize()
    for a, b in zip(ys, alone):
        assert torch.equal(a, b)
