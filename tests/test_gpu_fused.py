"""Fused mixed batches (k_fused.hip) on the GPU, in both modes (one launch per
pass level and class; one launch per class with per-job dependency waits):
bitwise equality with the per-(level, variant) launches and with each job
alone, parity with the oracle, HIP-graph capture and replay, and the bounded
dependency wait forced to give up from the host."""
import os

import numpy as np
import pytest

import oracle
from paper_2104_11471_amd import inputs
from tests.gpu_util import FP16_TOL, SPLIT_TOL, log

pytestmark = pytest.mark.gpu

# every pass of these plans has a fused variant: multi-pass 1D (two-pass
# four-step), 2D row + column, a plane pass, FP16 and split mixed
JOBS = [((256,), 7, "fp16"), ((4096,), 3, "fp16"), ((65536,), 3, "fp16"), ((128, 128), 2, "fp16"),
        ((256, 256), 2, "fp16"), ((512, 512), 1, "fp16"), ((1 << 20,), 1, "fp16"),
        ((16,), 100, "fp16"), ((16384,), 2, "fp16"), ((2048,), 9, "fp16"),
        ((1024,), 5, "split"), ((65536,), 1, "split"), ((256, 256), 1, "split"),
        ((16384,), 1, "split"), ((128, 128), 1, "split")]


def _make(dims, batch, prec, seed):
    if prec == "split":
        return np.stack(inputs.to_split(inputs.uniform_f64((batch, *dims), seed)))
    return inputs.uniform((batch, *dims), seed)


def _bits(t):
    import torch
    return t.view(torch.int16)


class _Env:
    def __init__(self, **kv):
        self.kv = kv

    def __enter__(self):
        self.old = {k: os.environ.get(k) for k in self.kv}
        os.environ.update({k: str(v) for k, v in self.kv.items()})

    def __exit__(self, *a):
        for k, v in self.old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


def _setup(jobs):
    import torch
    from paper_2104_11471_amd import tcfft
    # default plans: choices an earlier test tuned (the cache is per process)
    # may use variants outside the fused table
    tcfft.tune_cache_clear()
    plans, xs = [], []
    for i, (dims, batch, prec) in enumerate(jobs):
        p = tcfft.Plan(dims, batch, precision=prec)
        assert all(q["fused"] == 1 for q in p.describe()["passes"]), (dims, prec)
        plans.append(p)
        xs.append(torch.from_numpy(_make(dims, batch, prec, 40 + i)).cuda())
    return plans, xs


@pytest.mark.parametrize("mode", ["1", "2"])
def test_fused_batch_bitwise_and_parity(mode):
    import torch
    from paper_2104_11471_amd import tcfft
    plans, xs = _setup(JOBS)
    fused = [torch.empty_like(x) for x in xs]
    grouped = [torch.empty_like(x) for x in xs]
    alone = [torch.empty_like(x) for x in xs]
    before = tcfft.fused_wait_failures()
    log(f"fused batch (TCFFT_FUSED={mode}): {len(JOBS)} jobs")
    with _Env(TCFFT_FUSED=mode):
        tcfft.exec_many(plans, xs, fused)
        torch.cuda.synchronize()
    log("grouped batch (TCFFT_FUSED=0)")
    with _Env(TCFFT_FUSED=0):
        tcfft.exec_many(plans, xs, grouped)
        torch.cuda.synchronize()
    for p, x, o in zip(plans, xs, alone):
        p(x, o)
    torch.cuda.synchronize()
    assert tcfft.fused_wait_failures() == before
    for i in range(len(JOBS)):
        assert torch.equal(_bits(fused[i]), _bits(grouped[i])), ("grouped", i, JOBS[i])
        assert torch.equal(_bits(fused[i]), _bits(alone[i])), ("alone", i, JOBS[i])
    for i, (dims, batch, prec) in enumerate(JOBS):
        y = fused[i].cpu().numpy().astype(np.float64)
        if prec == "split":
            z = (y[0, ..., 0] + 2.0 ** -11 * y[1, ..., 0]) + 1j * (y[0, ..., 1] + 2.0 ** -11 * y[1, ..., 1])
            xh = xs[i].cpu().numpy()
            ref_in = oracle.from_split(xh[0], xh[1])
            tol = SPLIT_TOL
        else:
            z = y[..., 0] + 1j * y[..., 1]
            ref_in = oracle.from_half(xs[i].cpu().numpy())
            tol = FP16_TOL
        z = z * 2.0 ** plans[i].scale_log2
        ref = oracle.fft(ref_in) if len(dims) == 1 else oracle.fft2(ref_in)
        e = oracle.rel_l2(z, ref, axis=-1 if len(dims) == 1 else (-2, -1))
        assert e.max() < tol, (i, JOBS[i], float(e.max()))


@pytest.mark.parametrize("mode", ["1", "2"])
def test_fused_static_graph_capture_replays(mode):
    """tcfft_exec_many_static (descriptor tables written by kernels from their
    arguments, no allocation, no memset) captured into one HIP graph; each
    replay, with fresh inputs copied in and eager work between replays,
    matches an eager call bitwise."""
    import torch
    from paper_2104_11471_amd import tcfft
    jobs = [((1024,), 6, "fp16"), ((65536,), 2, "fp16"), ((256, 256), 2, "fp16"),
            ((4096,), 4, "split")]
    plans, xs = _setup(jobs)
    outs = [torch.empty_like(x) for x in xs]
    ref = [torch.empty_like(x) for x in xs]
    with _Env(TCFFT_FUSED=mode):
        tcfft.exec_many(plans, xs, outs, static=True)  # eager first: one-time set-up outside capture
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            with torch.cuda.graph(g, stream=s):
                tcfft.exec_many(plans, xs, outs, static=True)
        torch.cuda.synchronize()
    for rep in range(4):
        log(f"graph replay {rep}")
        for i, (dims, batch, prec) in enumerate(jobs):
            xs[i].copy_(torch.from_numpy(_make(dims, batch, prec, 100 + 10 * rep + i)))
        for o in outs:
            o.fill_(0)
        g.replay()
        torch.cuda.synchronize()
        tcfft.exec_many(plans, xs, ref)
        torch.cuda.synchronize()
        for i in range(len(jobs)):
            assert torch.equal(_bits(outs[i]), _bits(ref[i])), (rep, i, jobs[i])


def test_fused_wait_bound_forced_from_host():
    """Dependency mode (TCFFT_FUSED=2) with a zero wait bound
    (TCFFT_FUSED_WAIT_US=0): the first pass-2 tile that arrives before its
    pass 1 has finished gives up, the launch drains, the failure is counted,
    and the next batch with the default bound is right."""
    import torch
    from paper_2104_11471_amd import tcfft
    jobs = [((65536,), 64, "fp16")]
    plans, xs = _setup(jobs)
    out = torch.empty_like(xs[0])
    ref = torch.empty_like(xs[0])
    before = tcfft.fused_wait_failures()
    with _Env(TCFFT_FUSED=2, TCFFT_FUSED_WAIT_US=0):
        tcfft.exec_many(plans, xs, [out])
        torch.cuda.synchronize()
    after = tcfft.fused_wait_failures()
    log(f"wait failures {before} -> {after}")
    assert after == before + 1
    with _Env(TCFFT_FUSED=2):
        tcfft.exec_many(plans, xs, [out])
    plans[0](xs[0], ref)
    torch.cuda.synchronize()
    assert tcfft.fused_wait_failures() == after
    assert torch.equal(_bits(out), _bits(ref))
