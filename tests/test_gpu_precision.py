"""Precision of the split hi+lo FP16 mode against plain FP32 arithmetic: on
the same uniform inputs (the split pairs, and their FP32 roundings), the split
matrix-core path is within a small factor of an FP32 radix-2 FFT, each
measured against the FP64 oracle of its own input."""
import numpy as np
import pytest

import oracle
from paper_2104_11471_amd import inputs
from tests.gpu_util import log, run_plan

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tc():
    from paper_2104_11471_amd import tcfft
    return tcfft


@pytest.mark.parametrize("n", [256, 4096, 16384, 65536, 1 << 20])
def test_split_reaches_fp32_accuracy(tc, n):
    batch = max(1, (1 << 20) // n)
    hi, lo = inputs.to_split(inputs.uniform_f64((batch, n), 51))
    val = oracle.from_split(hi, lo)  # exact FP64 value of each input pair
    f32 = np.stack([val.real, val.imag], -1).astype(np.float32)
    v32 = f32[..., 0].astype(np.float64) + 1j * f32[..., 1].astype(np.float64)
    e_split = oracle.rel_l2(run_plan(tc.Plan((n,), batch, precision="split"), (hi, lo)),
                            oracle.fft(val))
    e_f32 = oracle.rel_l2(run_plan(tc.Plan((n,), batch, precision="fp32_radix2"), f32),
                          oracle.fft(v32))
    log(f"n={n}: split rel L2 mean {e_split.mean():.3e} max {e_split.max():.3e}; "
        f"fp32 radix-2 mean {e_f32.mean():.3e} max {e_f32.max():.3e}")
    assert e_split.mean() <= 2.0 * e_f32.mean()
    assert e_split.max() <= 2.0 * e_f32.max()
