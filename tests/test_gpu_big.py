"""The single-pass 65536-point kernel (one workgroup per transform) against the
oracle, and its grouped-launch variant against the single launch."""
import os
import tempfile

import numpy as np
import pytest

from paper_2104_11471_amd import inputs
from tests.gpu_util import FP16_TOL, log, reference, rel_err, run_plan

pytestmark = pytest.mark.gpu

N = 65536


@pytest.fixture(scope="module")
def tc():
    from paper_2104_11471_amd import tcfft
    return tcfft


def big_plan(tc, batch, sign=-1):
    """A plan forced onto the single-pass kernel through a wisdom entry."""
    lg = (batch - 1).bit_length()  # the tuner's batch bucket: ceil(log2(batch))
    fd, path = tempfile.mkstemp(suffix=".txt")
    with os.fdopen(fd, "w") as fh:
        fh.write(f"tcfft-tune 3\nr1_{N}x1_b{lg}_p0 256 64 1 {N} 0 0 0 0 1.0\n")
    tc.tune_cache_clear()
    tc.tune_cache_load(path)
    os.unlink(path)
    p = tc.Plan((N,), batch, direction=sign, flags=tc.FLAG_TUNE)
    tc.tune_cache_clear()
    d = p.describe()
    assert [q["kernel"] for q in d["passes"]] == ["big"], d
    assert d["scale_log2"] == 8 and p.num_launches == 1
    return p


@pytest.mark.parametrize("sign", [-1, 1])
@pytest.mark.parametrize("batch,seed", [(1, 0), (3, 1), (8, 2)])
def test_big_parity(tc, batch, seed, sign):
    log(f"case big N={N} batch={batch} sign={sign} seed={seed}")
    x = inputs.uniform((batch, N), seed)
    p = big_plan(tc, batch, sign)
    y = run_plan(p, x)
    e = rel_err(y, reference(x, 1, sign), 1)
    log(f"  max rel L2 = {e.max():.3e}")
    assert e.max() <= FP16_TOL


def test_big_tones(tc):
    """Unit tones: the peak lands on the tone's bin at amplitude N."""
    batch = 64
    x, tones = inputs.batched_1d(N, batch, seed=4)
    p = big_plan(tc, batch)
    y = run_plan(p, x)
    for r, f in zip(tones.rows, tones.freqs):
        assert int(np.argmax(np.abs(y[r]))) == int(f)
        assert abs(abs(y[r, f]) - N) / N < 5e-3


def test_big_matches_two_pass_and_grouped(tc):
    """The grouped (exec_many) launch gives the single launch's bits; the
    two-pass plan agrees within the FP16 tolerance."""
    import torch
    batch = 4
    x = torch.from_numpy(inputs.uniform((batch, N), 7)).cuda()
    p = big_plan(tc, batch)
    a = p(x)
    b = torch.empty_like(x)
    tc.exec_many([p], [x], [b])
    torch.cuda.synchronize()
    assert torch.equal(a.view(torch.int16), b.view(torch.int16))
    q = tc.Plan((N,), batch)
    assert q.describe()["passes"][0]["kernel"] == "col"
    c = q(x)
    torch.cuda.synchronize()
    za = a.cpu().numpy().astype(np.float64)
    zc = c.cpu().numpy().astype(np.float64)
    za = (za[..., 0] + 1j * za[..., 1]) * 2.0 ** p.scale_log2
    zc = (zc[..., 0] + 1j * zc[..., 1]) * 2.0 ** q.scale_log2
    e = np.linalg.norm(za - zc, axis=1) / np.linalg.norm(zc, axis=1)
    assert e.max() <= 2 * FP16_TOL


def test_big_full_size_sampled(tc):
    """Bench shape (2048 transforms): sampled transforms against the oracle."""
    import oracle
    import torch
    batch = 2048
    x, tones = inputs.batched_1d(N, batch, seed=0)
    p = big_plan(tc, batch)
    xd = torch.from_numpy(x).cuda()
    yd = p(xd)
    torch.cuda.synchronize()
    rows = np.unique(np.concatenate([[0, 1, 1023, 2047], tones.rows[:8]]))
    y = yd[rows].cpu().numpy().astype(np.float64)
    z = (y[..., 0] + 1j * y[..., 1]) * 2.0 ** p.scale_log2
    ref = oracle.fft(oracle.from_half(x[rows]), -1)
    e = oracle.rel_l2(z, ref)
    log(f"  full size: max rel L2 = {e.max():.3e} over {len(rows)} rows")
    assert e.max() <= FP16_TOL
