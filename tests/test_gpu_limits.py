"""Parity at the edges of the supported range and at the largest magnitudes.

* 1D N = 2^25, 2^26, 2^27 (the longest lengths the library accepts; the paper
  evaluates up to 2^27, Sec. 5.1), batch 1, FP16 and split: uniform inputs
  against the full FP64 oracle transform.
* Worst-case output magnitude of the static scale policy: a constant (1 + i)
  input puts sqrt(2) N 2^-S into bin 0 and a unit tone puts N 2^-S into one
  bin.  Checked at N = 2^24 and 2^27 (1D) and at 1024 x 1024 and
  2048 x 16384 (2D) against the closed forms (constant -> N delta[k], tone at f
  -> N delta[k - f], both pinned for the oracle by the CPU tests): no inf or
  NaN anywhere, the peak in its bin, relative L2 within the tolerance.
Tolerance: relative L2 per transform 5e-3 (FP16), 2e-5 (split)."""
import numpy as np
import pytest

import oracle
from paper_2104_11471_amd import inputs
from tests.gpu_util import FP16_TOL, SPLIT_TOL, log

pytestmark = pytest.mark.gpu


def _fetch_all(y, split):
    z = y.cpu().numpy().astype(np.float64)
    if split:
        return (z[0, ..., 0] + 2.0 ** -11 * z[1, ..., 0]) + 1j * (z[0, ..., 1] + 2.0 ** -11 * z[1, ..., 1])
    return z[..., 0] + 1j * z[..., 1]


def _run(plan, host):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(host)).cuda()
    y = plan(t)
    torch.cuda.synchronize()
    del t
    return y


@pytest.mark.parametrize("prec", ["fp16", "split"])
@pytest.mark.parametrize("lg", [25, 26, 27])
def test_longest_1d(lg, prec):
    from paper_2104_11471_amd import tcfft
    import torch
    n = 1 << lg
    split = prec == "split"
    log(f"case longest_1d N=2^{lg} batch=1 prec={prec}")
    if split:
        x = inputs.to_split(inputs.uniform_f64((1, n), lg))
        host = np.stack(x)
        xin = oracle.from_split(x[0], x[1])
    else:
        x = inputs.uniform((1, n), lg)
        host = x
        xin = oracle.from_half(x)
    plan = tcfft.Plan((n,), 1, precision=prec)
    log(f"  passes {[(p['kernel'], p['L']) for p in plan.describe()['passes']]}")
    y = _run(plan, host)
    z = _fetch_all(y, split) * 2.0 ** plan.scale_log2
    del y
    torch.cuda.empty_cache()
    ref = oracle.fft(xin, -1)
    e = oracle.rel_l2(z, ref)
    log(f"  rel L2 {e.max():.3e}  S={plan.scale_log2}")
    assert np.isfinite(z).all()
    assert e.max() <= (SPLIT_TOL if split else FP16_TOL)


def _closed_form_check(z, peak_index, peak_value, split):
    """z: output scaled back by 2^S (one transform, any rank)."""
    assert np.isfinite(z).all(), "inf or NaN in the output"
    ref = np.zeros_like(z)
    ref[peak_index] = peak_value
    assert np.unravel_index(int(np.argmax(np.abs(z))), z.shape) == peak_index
    e = float(np.linalg.norm(z - ref) / np.linalg.norm(ref))
    log(f"  peak {abs(z[peak_index]):.6g} (exact {abs(peak_value):.6g}), rel L2 {e:.3e}")
    assert e <= (SPLIT_TOL if split else FP16_TOL)


def _const_and_tone(dims, f):
    """(constant 1+i, unit tone at multi-index f) as complex128 arrays."""
    const = np.full(dims, 1.0 + 1.0j)
    ph = np.zeros(dims)
    for ax, (n, fa) in enumerate(zip(dims, f)):
        shape = [1] * len(dims)
        shape[ax] = n
        idx = np.arange(n, dtype=np.int64)
        ph = ph + (((fa * idx) % n) / n).reshape(shape)
    tone = np.exp(2j * np.pi * ph)
    return const, tone


@pytest.mark.parametrize("prec", ["fp16", "split"])
@pytest.mark.parametrize("dims", [(1 << 24,), (1 << 27,), (1024, 1024), (2048, 16384)],
                         ids=["1d_2^24", "1d_2^27", "2d_1024x1024", "2d_2048x16384"])
def test_largest_magnitudes(dims, prec):
    from paper_2104_11471_amd import tcfft
    import torch
    split = prec == "split"
    npts = int(np.prod(dims))
    f = tuple(int(d) * 3 // 7 + 1 for d in dims)
    const, tone = _const_and_tone(dims, f)
    plan = tcfft.Plan(dims, 1, precision=prec)
    for name, xin, k, v in (("constant", const, (0,) * len(dims), npts * (1.0 + 1.0j)),
                            ("tone", tone, f, float(npts))):
        log(f"case magnitude {name} dims={dims} prec={prec} S={plan.scale_log2}")
        if split:
            hi, lo = inputs.to_split(xin[None])
            host = np.stack([hi, lo])
        else:
            h = np.empty((1,) + dims + (2,), np.float16)
            h[..., 0] = xin.real
            h[..., 1] = xin.imag
            host = h
            # the reference transforms the FP16-rounded input: the constant is
            # exact, the tone's rounding is a perturbation the tolerance covers
        y = _run(plan, host)
        z = _fetch_all(y, split)[0] * 2.0 ** plan.scale_log2
        del y
        torch.cuda.empty_cache()
        _closed_form_check(z, k, v, split)
