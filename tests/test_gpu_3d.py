"""Batched 3D transforms (a row pass over nz, column passes over ny and nx)
against the oracle's fft3: FP16 and split, both directions, the tuned plan,
and grouped execution mixed with other ranks."""
import numpy as np
import pytest

import oracle
from paper_2104_11471_amd import inputs
from tests.gpu_util import FP16_TOL, SPLIT_TOL, log, run_plan

pytestmark = pytest.mark.gpu

# from (64, 128, 128) on: [ny][nz] planes of 16384 points (plane pass); the
# 4096- and 8192-point planes take the plane pass in FP16 only
SHAPES = [((16, 16, 16), 3), ((64, 64, 64), 2), ((128, 32, 256), 1), ((32, 256, 16), 5),
          ((16, 2048, 32), 1), ((2048, 16, 16), 2), ((64, 128, 128), 1), ((16, 256, 64), 3),
          ((32, 64, 256), 2), ((16, 32, 512), 2), ((16, 16, 1024), 3),
          # FP16: 4 planes of 4096 or 2 of 8192 points per workgroup
          ((16, 64, 64), 3), ((16, 32, 128), 2), ((32, 128, 64), 1), ((16, 64, 128), 2),
          ((16, 32, 256), 1)]


@pytest.fixture(scope="module")
def tc():
    from paper_2104_11471_amd import tcfft
    return tcfft


def rel3(y, ref):
    return oracle.rel_l2(y, ref, axis=(-3, -2, -1))


@pytest.mark.parametrize("prec", ["fp16", "split"])
@pytest.mark.parametrize("dims,batch", SHAPES)
def test_3d_parity(tc, dims, batch, prec):
    log(f"case 3d dims={dims} batch={batch} prec={prec}")
    if prec == "split":
        x = inputs.to_split(inputs.uniform_f64((batch,) + dims, 31))
        xc = oracle.from_split(*x)
        tol = SPLIT_TOL
    else:
        x = inputs.uniform((batch,) + dims, 31)
        xc = oracle.from_half(x)
        tol = FP16_TOL
    for sign in (-1, 1):
        p = tc.Plan(dims, batch, sign, prec)
        y = run_plan(p, x)
        e = rel3(y, oracle.fft3(xc, sign))
        log(f"  sign={sign} max rel L2 = {e.max():.3e}")
        assert e.max() <= tol


@pytest.mark.parametrize("dims", [(64, 32, 128), (32, 128, 128)])
def test_3d_tuned_and_inplace(tc, dims):
    batch = 4
    x = inputs.uniform((batch,) + dims, 32)
    p = tc.Plan(dims, batch, flags=tc.FLAG_TUNE)
    assert p.describe()["tuned"]
    y = run_plan(p, x, inplace=True)
    assert rel3(y, oracle.fft3(oracle.from_half(x))).max() <= FP16_TOL


@pytest.mark.parametrize("shape", [(32, 16, 64), (16, 128, 128)])
def test_3d_plane_wave(tc, shape):
    """A unit plane wave goes to one bin of height nx*ny*nz (closed form)."""
    nx, ny, nz = shape
    f = (5, 9, 50) if nz == 64 else (7, 100, 3)
    gx, gy, gz = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    w = np.exp(2j * np.pi * (f[0] * gx / nx + f[1] * gy / ny + f[2] * gz / nz))
    x = np.stack([w.real, w.imag], -1).astype(np.float16)[None]
    y = run_plan(tc.Plan((nx, ny, nz), 1), x)[0]
    n = nx * ny * nz
    assert abs(y[f] - n) < 1e-2 * n
    y[f] = 0
    assert np.max(np.abs(y)) < 3e-3 * n


def test_3d_grouped_matches_single(tc):
    import torch
    plans = [tc.Plan((64, 64, 64), 2), tc.Plan((16, 128, 32), 3), tc.Plan((256, 256), 4),
             tc.Plan((32, 32, 32), 1, precision="split"), tc.Plan((16, 128, 128), 2),
             tc.Plan((16, 64, 256), 1, precision="split"), tc.Plan((64, 64), 7),
             tc.Plan((16, 32, 128), 3)]
    xs = []
    for k, p in enumerate(plans):
        t = torch.from_numpy(inputs.uniform(p.in_shape()[:-1] if p.precision == 0 else
                                            p.in_shape()[1:-1], 40 + k)).cuda()
        xs.append(t if p.precision == 0 else torch.stack([t, t * 0]).contiguous())
    singles = [p(x) for p, x in zip(plans, xs)]
    outs = [p.empty_out() for p in plans]
    tc.exec_many(plans, xs, outs)
    torch.cuda.synchronize()
    for a, o in zip(singles, outs):
        assert torch.equal(a.view(torch.int16), o.view(torch.int16))


@pytest.mark.parametrize("dims", [(128, 128), (16, 128, 128), (32, 64, 256), (16, 16, 16)])
def test_no_scale_plane_and_3d(tc, dims):
    """TCFFT_FLAG_NO_SCALE (S = 0) through the plane pass, whose row and column
    halves each carry their own radix-R0 scale, and through 3D plans; inputs
    are scaled down so the unnormalised FP16 output stays in range."""
    batch = 2
    x = (inputs.uniform((batch,) + dims, 33).astype(np.float32) / 64).astype(np.float16)
    p = tc.Plan(dims, batch, flags=tc.FLAG_NO_SCALE)
    assert p.scale_log2 == 0
    y = run_plan(p, x)
    ref = oracle.fft2(oracle.from_half(x)) if len(dims) == 2 else oracle.fft3(oracle.from_half(x))
    axes = (-2, -1) if len(dims) == 2 else (-3, -2, -1)
    assert oracle.rel_l2(y, ref, axis=axes).max() <= FP16_TOL
