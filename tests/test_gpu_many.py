"""Grouped mixed-size execution and the autotuner on the GPU."""
import numpy as np
import pytest

import oracle
from paper_2104_11471_amd import inputs
from tests.gpu_util import FP16_TOL, log

pytestmark = pytest.mark.gpu

JOBS = [((256,), 7, "fp16"), ((4096,), 3, "fp16"), ((256,), 33, "fp16"), ((65536,), 2, "fp16"),
        ((128, 128), 3, "fp16"), ((512, 512), 1, "split"), ((1 << 20,), 1, "fp16"),
        ((16,), 100, "fp16"), ((16384,), 2, "split"), ((4096,), 5, "fp32_radix2"),
        ((1 << 17,), 1, "split"), ((64, 2048), 2, "fp16")]


def _make(dims, batch, prec, seed):
    if prec == "split":
        return np.stack(inputs.to_split(inputs.uniform_f64((batch, *dims), seed)))
    x = inputs.uniform((batch, *dims), seed)
    return x.astype(np.float32) if prec == "fp32_radix2" else x


def test_exec_many_equals_exec_alone():
    import torch
    from paper_2104_11471_amd import tcfft
    plans, xs, outs_many, outs_alone = [], [], [], []
    for i, (dims, batch, prec) in enumerate(JOBS):
        log(f"job {i}: dims={dims} batch={batch} prec={prec}")
        plans.append(tcfft.Plan(dims, batch, precision=prec))
        x = torch.from_numpy(_make(dims, batch, prec, i)).cuda()
        xs.append(x)
        outs_many.append(torch.empty_like(x))
        outs_alone.append(torch.empty_like(x))
    tcfft.exec_many(plans, xs, outs_many)
    for p, x, o in zip(plans, xs, outs_alone):
        p(x, o)
    torch.cuda.synchronize()
    for i, (a, b) in enumerate(zip(outs_many, outs_alone)):
        assert torch.equal(a.view(torch.int16) if a.dtype == torch.float16 else a.view(torch.int32),
                           b.view(torch.int16) if b.dtype == torch.float16 else b.view(torch.int32)), i
    # and the mixed results are right
    for i, (dims, batch, prec) in enumerate(JOBS):
        if prec != "fp16":
            continue
        y = outs_many[i].cpu().numpy().astype(np.float64)
        z = (y[..., 0] + 1j * y[..., 1]) * 2.0 ** plans[i].scale_log2
        ref_in = oracle.from_half(xs[i].cpu().numpy())
        ref = oracle.fft(ref_in) if len(dims) == 1 else oracle.fft2(ref_in)
        e = oracle.rel_l2(z, ref, axis=-1 if len(dims) == 1 else (-2, -1))
        assert e.max() < FP16_TOL, (i, float(e.max()))


def test_exec_many_repeated_replays():
    """The descriptor tables are rebuilt per call; replays give identical bits."""
    import torch
    from paper_2104_11471_amd import tcfft
    plans = [tcfft.Plan((1024,), 9), tcfft.Plan((2048,), 4), tcfft.Plan((1024,), 2)]
    xs = [torch.from_numpy(inputs.uniform((p.batch, p.dims[0]), 5 + k)).cuda()
          for k, p in enumerate(plans)]
    outs = [torch.empty_like(x) for x in xs]
    tcfft.exec_many(plans, xs, outs)
    torch.cuda.synchronize()
    first = [o.clone() for o in outs]
    for _ in range(3):
        for o in outs:
            o.zero_()
        tcfft.exec_many(plans, xs, outs)
        torch.cuda.synchronize()
        for a, b in zip(outs, first):
            assert torch.equal(a.view(torch.int16), b.view(torch.int16))


@pytest.mark.parametrize("dims,batch", [((4096,), 256), ((65536,), 16), ((256, 256), 8)])
def test_autotuned_plan(dims, batch, tmp_path):
    import torch
    from paper_2104_11471_amd import tcfft
    tcfft.tune_cache_clear()
    p = tcfft.Plan(dims, batch, flags=tcfft.FLAG_TUNE)
    d = p.describe()
    log(f"tuned {dims}: {d['choice']} {d['tuned_us']:.1f} us")
    assert d["tuned"] and d["tuned_us"] > 0
    assert tcfft.tune_cache_size() >= 1
    x = inputs.uniform((batch, *dims), 11)
    y = p(torch.from_numpy(x).cuda()).cpu().numpy().astype(np.float64)
    z = (y[..., 0] + 1j * y[..., 1]) * 2.0 ** p.scale_log2
    ref = oracle.fft(oracle.from_half(x)) if len(dims) == 1 else oracle.fft2(oracle.from_half(x))
    e = oracle.rel_l2(z, ref, axis=-1 if len(dims) == 1 else (-2, -1))
    assert e.max() < FP16_TOL
    path = str(tmp_path / "wisdom.txt")
    tcfft.tune_cache_save(path)
    tcfft.tune_cache_clear()
    assert tcfft.tune_cache_size() == 0
    tcfft.tune_cache_load(path)
    q = tcfft.Plan(dims, batch)   # no TUNE flag: the cached choice is reused
    assert q.describe()["choice"] == d["choice"] and q.describe()["tuned"]


@pytest.mark.parametrize("dims,batch,chunk", [((65536,), 64, 16), ((1 << 20,), 8, 3),
                                              ((256, 256), 32, 5)])
def test_chunked_execution_is_bitwise_equal(dims, batch, chunk, tmp_path):
    """A multi-pass plan run chunk by chunk (workspace reused per chunk, the
    MALL-residency knob) gives the same bits as the whole-batch run."""
    import torch
    from paper_2104_11471_amd import tcfft
    tcfft.tune_cache_clear()
    x = torch.from_numpy(inputs.uniform((batch, *dims), 21)).cuda()
    whole = tcfft.Plan(dims, batch)(x)
    key = f"r{len(dims)}_{dims[0]}x{dims[1] if len(dims) == 2 else 1}_b{int(np.log2(batch))}_p0"
    path = tmp_path / "wisdom.txt"
    path.write_text(f"tcfft-tune 3\n{key} 256 64 0 0 0 0 {chunk} 0 1.0\n")
    tcfft.tune_cache_load(str(path))
    p = tcfft.Plan(dims, batch)
    assert p.describe()["choice"]["chunk"] == chunk
    if len(dims) == 1:  # 2D plans have no workspace
        assert p.workspace_bytes < tcfft.Plan(dims, 1).workspace_bytes * batch
    y = p(x)
    torch.cuda.synchronize()
    assert torch.equal(y.view(torch.int16), whole.view(torch.int16))
    tcfft.tune_cache_clear()


def test_exec_many_rejects_a_workspace_plan_twice():
    """Two jobs of one multi-pass plan would write the plan's workspace inside
    one grouped launch: the call is rejected; single-pass plans may repeat."""
    import torch
    from paper_2104_11471_amd import tcfft
    p = tcfft.Plan((1 << 17,), 1)
    assert p.workspace_bytes > 0
    xs = [torch.from_numpy(inputs.uniform((1, 1 << 17), 30 + k)).cuda() for k in range(2)]
    outs = [torch.empty_like(x) for x in xs]
    with pytest.raises(tcfft.TcfftError) as ei:
        tcfft.exec_many([p, p], xs, outs)
    assert ei.value.status == 1
    q = tcfft.Plan((1024,), 4)
    assert q.workspace_bytes == 0
    ys = [torch.from_numpy(inputs.uniform((4, 1024), 40 + k)).cuda() for k in range(3)]
    many = [torch.empty_like(y) for y in ys]
    tcfft.exec_many([q, q, q], ys, many)
    for y, m in zip(ys, many):
        assert torch.equal(q(y).view(torch.int16), m.view(torch.int16))
