"""The allocation-free grouped launch (tcfft_exec_many_static) through the C
ABI: bitwise equal to tcfft_exec_many on the same jobs, on two calls in a row
(the second with fewer and smaller jobs, so stale tables from the first call
would show), plus the job-count limit."""
import ctypes

import numpy as np
import pytest

from paper_2104_11471_amd import inputs
from tests.gpu_util import log

pytestmark = pytest.mark.gpu


def _jobs(specs, seed):
    import torch
    from paper_2104_11471_amd import tcfft
    plans, xs = [], []
    for i, (dims, batch, prec, flags) in enumerate(specs):
        p = tcfft.Plan(dims, batch, precision=prec, flags=flags)
        shape = p.in_shape()
        if flags & tcfft.FLAG_REAL:
            host = inputs.uniform((batch, dims[0] // 2), seed + i).reshape(batch, dims[0])
        elif prec == "split":
            host = np.stack(inputs.to_split(inputs.uniform_f64(shape[1:-1], seed + i)))
        else:
            host = inputs.uniform(shape[:-1], seed + i)
        plans.append(p)
        xs.append(torch.from_numpy(np.ascontiguousarray(host)).cuda())
    return plans, xs


def _run_both(plans, xs):
    import torch
    from paper_2104_11471_amd import tcfft
    ref = [p.empty_out() for p in plans]
    got = [p.empty_out() for p in plans]
    for o in got:
        o.fill_(7.0)  # every output word must be rewritten
    tcfft.exec_many(plans, xs, ref)
    tcfft.exec_many(plans, xs, got, static=True)
    torch.cuda.synchronize()
    for p, a, b in zip(plans, ref, got):
        assert torch.equal(a.view(torch.int16), b.view(torch.int16)), p.describe()["dims"]


def test_static_grouped_launch_equals_exec_many():
    first = [((256,), 64, "fp16", 0), ((4096,), 37, "fp16", 0), ((1 << 16,), 3, "fp16", 0),
             ((128, 128), 5, "split", 0), ((1 << 20,), 1, "split", 0), ((512,), 9, "split", 0),
             ((64, 64, 64), 2, "fp16", 0), ((8192,), 6, "fp16", 8)]
    second = [((1024,), 3, "fp16", 0), ((64, 32), 2, "fp16", 0)]
    log("case static grouped launch: 8 mixed jobs, then 2 small jobs")
    plans, xs = _jobs(first, 1)
    _run_both(plans, xs)
    plans2, xs2 = _jobs(second, 50)
    _run_both(plans2, xs2)


def test_static_grouped_launch_job_limit():
    import torch
    from paper_2104_11471_amd import tcfft
    p = tcfft.Plan((256,), 1)
    x = torch.zeros(p.in_shape(), dtype=torch.float16, device="cuda")
    outs = [torch.empty_like(x) for _ in range(tcfft.STATIC_MAX_JOBS + 1)]
    with pytest.raises(tcfft.TcfftError) as e:
        tcfft.exec_many([p] * len(outs), [x] * len(outs), outs, static=True)
    assert e.value.status == 1
    # at the limit it runs
    tcfft.exec_many([p] * tcfft.STATIC_MAX_JOBS, [x] * tcfft.STATIC_MAX_JOBS,
                    outs[:tcfft.STATIC_MAX_JOBS], static=True)
    torch.cuda.synchronize()
    assert all(torch.count_nonzero(o) == 0 for o in outs[:4])
