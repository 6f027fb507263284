"""Real-input transforms (R2C forward, C2R inverse) on the GPU against the
oracle's rfft/irfft: single-pass, two-pass and three-pass complex cores, FP16
and split precision, the round trip, in-place use and grouped execution."""
import numpy as np
import pytest

import oracle
from paper_2104_11471_amd import inputs
from tests.gpu_util import FP16_TOL, SPLIT_TOL, log

pytestmark = pytest.mark.gpu

SIZES = [32, 64, 128, 256, 512, 1024, 4096, 8192, 16384, 32768, 65536, 1 << 21, 1 << 24]


@pytest.fixture(scope="module")
def tc():
    from paper_2104_11471_amd import tcfft
    return tcfft


def batch_for(n):
    return max(1, min(5, (1 << 22) // n))


def real_input(n, batch, prec, seed):
    """N reals per transform as M complex words (the library's real layout)."""
    m = n // 2
    if prec == "split":
        hi, lo = inputs.to_split(inputs.uniform_f64((batch, m), seed))
        host = np.stack([hi.reshape(batch, n), lo.reshape(batch, n)])
        val = hi.reshape(batch, n).astype(np.float64) + 2.0 ** -11 * lo.reshape(batch, n).astype(np.float64)
    else:
        host = inputs.uniform((batch, m), seed).reshape(batch, n)
        val = host.astype(np.float64)
    return host, val


def spectrum_input(n, batch, prec, seed):
    m = n // 2
    if prec == "split":
        hi, lo = inputs.to_split(inputs.uniform_f64((batch, m + 1), seed))
        return np.stack([hi, lo]), oracle.from_split(hi, lo)
    x = inputs.uniform((batch, m + 1), seed)
    return x, oracle.from_half(x)


def read_spectrum(out, prec):
    y = out.cpu().numpy().astype(np.float64)
    if prec == "split":
        return (y[0, ..., 0] + 2.0 ** -11 * y[1, ..., 0]) + 1j * (y[0, ..., 1] + 2.0 ** -11 * y[1, ..., 1])
    return y[..., 0] + 1j * y[..., 1]


def read_real(out, prec):
    y = out.cpu().numpy().astype(np.float64)
    return y[0] + 2.0 ** -11 * y[1] if prec == "split" else y


@pytest.mark.parametrize("prec", ["fp16", "split"])
@pytest.mark.parametrize("n", SIZES)
def test_r2c_parity(tc, n, prec):
    import torch
    b = batch_for(n)
    log(f"case r2c n={n} batch={b} prec={prec}")
    p = tc.Plan((n,), b, tc.FORWARD, prec, flags=tc.FLAG_REAL)
    assert p.in_shape()[-1] == n and p.out_shape()[-2:] == (n // 2 + 1, 2)
    host, val = real_input(n, b, prec, 21)
    out = p(torch.from_numpy(host).cuda())
    torch.cuda.synchronize()
    y = read_spectrum(out, prec) * 2.0 ** p.scale_log2
    e = oracle.rel_l2(y, oracle.rfft(val))
    log(f"  max rel L2 = {e.max():.3e}")
    assert e.max() <= (SPLIT_TOL if prec == "split" else FP16_TOL)


@pytest.mark.parametrize("prec", ["fp16", "split"])
@pytest.mark.parametrize("n", SIZES)
def test_c2r_parity(tc, n, prec):
    """A general spectrum (non-real X[0], X[M] included: their imaginary parts
    are ignored, as for the oracle)."""
    import torch
    b = batch_for(n)
    log(f"case c2r n={n} batch={b} prec={prec}")
    p = tc.Plan((n,), b, tc.INVERSE, prec, flags=tc.FLAG_REAL)
    host, X = spectrum_input(n, b, prec, 22)
    out = p(torch.from_numpy(np.ascontiguousarray(host)).cuda())
    torch.cuda.synchronize()
    y = read_real(out, prec) * 2.0 ** p.scale_log2
    e = oracle.rel_l2(y, oracle.irfft(X, n))
    log(f"  max rel L2 = {e.max():.3e}")
    assert e.max() <= (SPLIT_TOL if prec == "split" else FP16_TOL)


@pytest.mark.parametrize("prec", ["fp16", "split"])
@pytest.mark.parametrize("n,batch", [(128, 513), (256, 300), (2048, 37), (32768, 7)])
def test_real_many_lines(tc, n, batch, prec):
    """Fused row passes over several workgroups of lines with a ragged last
    workgroup, both directions."""
    import torch
    log(f"case real lines n={n} batch={batch} prec={prec}")
    tol = SPLIT_TOL if prec == "split" else FP16_TOL
    f = tc.Plan((n,), batch, tc.FORWARD, prec, flags=tc.FLAG_REAL)
    host, val = real_input(n, batch, prec, 24)
    y = read_spectrum(f(torch.from_numpy(host).cuda()), prec) * 2.0 ** f.scale_log2
    assert oracle.rel_l2(y, oracle.rfft(val)).max() <= tol
    i = tc.Plan((n,), batch, tc.INVERSE, prec, flags=tc.FLAG_REAL)
    host, X = spectrum_input(n, batch, prec, 25)
    y = read_real(i(torch.from_numpy(np.ascontiguousarray(host)).cuda()), prec) * 2.0 ** i.scale_log2
    assert oracle.rel_l2(y, oracle.irfft(X, n)).max() <= tol


@pytest.mark.parametrize("n", [64, 4096, 1 << 20])
def test_round_trip(tc, n):
    """C2R(R2C(x)) = N x 2^-(S_f + S_i), with many workgroups of lines."""
    import torch
    b = max(3, (1 << 22) // n)
    log(f"case real round trip n={n} batch={b}")
    f = tc.Plan((n,), b, tc.FORWARD, "fp16", flags=tc.FLAG_REAL)
    i = tc.Plan((n,), b, tc.INVERSE, "fp16", flags=tc.FLAG_REAL)
    host, val = real_input(n, b, "fp16", 23)
    spec = f(torch.from_numpy(host).cuda())
    y = i(spec).cpu().numpy().astype(np.float64)
    y *= 2.0 ** (f.scale_log2 + i.scale_log2)
    e = oracle.rel_l2(y, n * val)
    log(f"  max rel L2 = {e.max():.3e}")
    assert e.max() <= 2 * FP16_TOL


def test_real_tone(tc):
    """A cosine tone: all energy in one bin (closed form N/2)."""
    import torch
    n, f0 = 4096, 37
    p = tc.Plan((n,), 1, tc.FORWARD, "fp16", flags=tc.FLAG_REAL)
    x = np.cos(2 * np.pi * f0 * np.arange(n) / n).astype(np.float16)[None, :]
    y = read_spectrum(p(torch.from_numpy(x).cuda()), "fp16") * 2.0 ** p.scale_log2
    assert abs(y[0, f0] - n / 2) < 1e-2 * n / 2
    y[0, f0] = 0
    assert np.max(np.abs(y)) < 2e-3 * n / 2


def test_real_grouped_matches_single(tc):
    """Real plans (both directions) mixed with a complex plan in one grouped
    call give each job's single-exec bits."""
    import torch
    pf = tc.Plan((4096,), 3, tc.FORWARD, "fp16", flags=tc.FLAG_REAL)
    pi = tc.Plan((65536,), 2, tc.INVERSE, "fp16", flags=tc.FLAG_REAL)
    pc = tc.Plan((1024,), 4)
    xs = [torch.from_numpy(real_input(4096, 3, "fp16", 1)[0]).cuda(),
          torch.from_numpy(spectrum_input(65536, 2, "fp16", 2)[0]).cuda(),
          torch.from_numpy(inputs.uniform((4, 1024), 3)).cuda()]
    plans = [pf, pi, pc]
    singles = [p(x) for p, x in zip(plans, xs)]
    outs = [p.empty_out() for p in plans]
    tc.exec_many(plans, xs, outs)
    torch.cuda.synchronize()
    for a, o in zip(singles, outs):
        assert torch.equal(a.view(torch.int16), o.view(torch.int16))


def test_real_split_grouped_matches_single(tc):
    """Split real plans with the fused epilogue / prologue in one grouped call
    (their grouped kernels run one tile per workgroup) give each job's
    single-exec bits, beside an FP16 real plan of the same size."""
    import torch
    jobs = [(8192, 5, tc.FORWARD, "split"), (1024, 37, tc.INVERSE, "split"),
            (16384, 2, tc.FORWARD, "split"), (256, 300, tc.INVERSE, "split"),
            (8192, 3, tc.FORWARD, "fp16")]
    plans, xs = [], []
    for i, (n, b, d, prec) in enumerate(jobs):
        p = tc.Plan((n,), b, d, prec, flags=tc.FLAG_REAL)
        assert p.describe()["real_kernel"] == "fused"
        host = real_input(n, b, prec, 10 + i)[0] if d == tc.FORWARD else spectrum_input(n, b, prec, 10 + i)[0]
        plans.append(p)
        xs.append(torch.from_numpy(np.ascontiguousarray(host)).cuda().reshape(p.in_shape()))
    singles = [p(x) for p, x in zip(plans, xs)]
    outs = [p.empty_out() for p in plans]
    tc.exec_many(plans, xs, outs)
    torch.cuda.synchronize()
    for i, (a, o) in enumerate(zip(singles, outs)):
        assert torch.equal(a.view(torch.int16), o.view(torch.int16)), jobs[i]


def test_real_rejects_overlap(tc):
    """Lines of M and M + 1 words cannot be rewritten in place: overlapping
    buffers of a real plan are an argument error, nothing is launched."""
    import torch
    s = torch.cuda.current_stream().cuda_stream
    for dirn in (tc.FORWARD, tc.INVERSE):
        p = tc.Plan((4096,), 2, dirn, "fp16", flags=tc.FLAG_REAL)
        buf = torch.empty(2 * 2049 * 2 + 8, dtype=torch.float16, device="cuda")
        for off in (0, 8):  # the same pointer, and a shifted one
            st = tc.lib.tcfft_exec(p.handle, buf.data_ptr(), buf.data_ptr() + 2 * off, s)
            assert st == 1
        hp = (tc.ctypes.c_void_p * 1)(p.handle)
        ip = (tc.ctypes.c_void_p * 1)(buf.data_ptr())
        assert tc.lib.tcfft_exec_many(hp, ip, ip, 1, s) == 1


def test_real_describe(tc):
    p = tc.Plan((8192,), 2, tc.FORWARD, "fp16", flags=tc.FLAG_REAL)
    d = p.describe()
    assert d["real"] == 8192 and d["real_kernel"] == "fused"
    assert [q["L"] for q in d["passes"]] == [4096]
    assert p.input_bytes == 2 * 4096 * 4 and p.output_bytes == 2 * 4097 * 4
    assert p.num_launches == 1
    assert tc.Plan((1 << 16,), 1, tc.FORWARD, "fp16", flags=tc.FLAG_REAL).num_launches == 3
    x, o = p.empty(), p.empty_out()
    assert tc.lib.tcfft_exec_passes(p.handle, x.data_ptr(), o.data_ptr(), 1, None) == 2


@pytest.mark.parametrize("n", [128, 8192, 32768, 65536])
def test_real_no_scale(tc, n):
    """Unnormalised real transforms (S = 0), fused and stand-alone steps."""
    import torch
    b = 2
    f = tc.Plan((n,), b, tc.FORWARD, "fp16", flags=tc.FLAG_REAL | tc.FLAG_NO_SCALE)
    i = tc.Plan((n,), b, tc.INVERSE, "fp16", flags=tc.FLAG_REAL | tc.FLAG_NO_SCALE)
    assert f.scale_log2 == 0 and i.scale_log2 == 0
    host = (inputs.uniform((b, n // 2), 26).astype(np.float32) / 256).astype(np.float16).reshape(b, n)
    spec = f(torch.from_numpy(host).cuda())
    y = read_spectrum(spec, "fp16")
    assert oracle.rel_l2(y, oracle.rfft(host.astype(np.float64))).max() <= FP16_TOL
    back = read_real(i(spec), "fp16")
    assert oracle.rel_l2(back, n * host.astype(np.float64)).max() <= 2 * FP16_TOL
