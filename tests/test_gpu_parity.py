"""GPU path vs the FP64 oracle, element by element, through the C ABI.

Tolerances: relative L2 per transform <= 5e-3 (FP16 storage), <= 2e-5 (split
hi+lo FP16), <= 1e-5 (FP32 radix-2 comparator)."""
import numpy as np
import pytest

import oracle
from paper_2104_11471_amd import inputs
from tests.gpu_util import FP16_TOL, FP32_TOL, SPLIT_TOL, log, reference, rel_err, run_plan

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tc():
    from paper_2104_11471_amd import tcfft
    return tcfft


def _check(tc, dims, batch, prec="fp16", sign=-1, flags=0, seed=0, tol=None, inplace=False):
    rank = len(dims)
    log(f"case dims={dims} batch={batch} prec={prec} sign={sign} flags={flags} seed={seed}")
    if prec == "split":
        x = inputs.to_split(inputs.uniform_f64((batch, *dims), seed))
        tol = tol or SPLIT_TOL
    elif prec == "fp32_radix2":
        x = inputs.uniform((batch, *dims), seed).astype(np.float32)
        tol = tol or FP32_TOL
    else:
        x = inputs.uniform((batch, *dims), seed)
        tol = tol or FP16_TOL
    plan = tc.Plan(dims, batch, direction=sign, precision=prec, flags=flags)
    y = run_plan(plan, x, inplace=inplace)
    ref = reference(x, rank, sign)
    e = rel_err(y, ref, rank)
    log(f"  max rel L2 = {e.max():.3e}  mean = {e.mean():.3e}  S = {plan.scale_log2}")
    assert np.all(np.isfinite(y))
    assert e.max() <= tol, (dims, batch, prec, float(e.max()))
    return e


def test_radix16_block_is_the_dft_matrix(tc):
    """N = 16: one matrix-core block.  Input delta at r must give row r of the
    DFT matrix W_16^{r k} (probes the operand and accumulator layouts)."""
    x = np.zeros((16, 16, 2), np.float16)
    for r in range(16):
        x[r, r, 0] = 1.0
    plan = tc.Plan((16,), 16, flags=tc.FLAG_NO_SCALE)
    y = run_plan(plan, x)
    k = np.arange(16)
    for r in range(16):
        ref = np.exp(-2j * np.pi * ((r * k) % 16) / 16)
        assert np.abs(y[r] - ref).max() < 2e-3, r


@pytest.mark.parametrize("n", [16, 32, 64, 128, 256, 512, 1024, 2048, 4096, 8192, 16384])
def test_single_pass_sizes(tc, n):
    _check(tc, (n,), 37)       # ragged batch: not a multiple of lines per workgroup


@pytest.mark.parametrize("n", [1 << 15, 1 << 16, 1 << 17, 1 << 20, 1 << 22, 1 << 23])
def test_multi_pass_sizes(tc, n):
    _check(tc, (n,), 3 if n <= (1 << 20) else 1)


def test_config1_exact_shape(tc):
    """N=256, batch 64, uniform[-1,1] from seed 0, unnormalised (S = 0)."""
    e = _check(tc, (256,), 64, flags=tc.FLAG_NO_SCALE, seed=0)
    assert e.shape == (64,)


@pytest.mark.parametrize("n", [256, 4096, 1 << 16])
def test_inverse_and_roundtrip(tc, n):
    _check(tc, (n,), 5, sign=1)
    x = inputs.uniform((4, n), 3)
    f = tc.Plan((n,), 4, direction=-1)
    b = tc.Plan((n,), 4, direction=1)
    import torch
    t = torch.from_numpy(x).cuda()
    y = b(f(t))
    torch.cuda.synchronize()
    z = y.cpu().numpy().astype(np.float64)
    z = (z[..., 0] + 1j * z[..., 1]) * 2.0 ** (f.scale_log2 + b.scale_log2)
    e = oracle.rel_l2(z, n * oracle.from_half(x))
    assert e.max() < 2 * FP16_TOL


@pytest.mark.parametrize("dims,batch,sign", [((1 << 15,), 3, -1), ((1 << 15,), 3, 1),
                                             ((128, 256), 4, -1), ((128, 512), 3, 1),
                                             ((1 << 23,), 1, 1)])
def test_128_point_column_passes(tc, dims, batch, sign):
    """Plans with a 128-point FP16 column pass of 64 columns (radix-8 stage,
    then one radix-16 stage): both directions, with the inter-pass twiddle
    and transposed store (its table lookups issued before the HBM reads) and
    without."""
    passes = tc.dry_run(dims, batch, direction=sign)["passes"]
    assert any(p["kernel"] == "col" and p["L"] == 128 and p["C"] == 64 for p in passes), passes
    _check(tc, dims, batch, sign=sign, seed=11)


@pytest.mark.parametrize("dims,batch,sign", [((256, 256), 1, -1), ((256, 256), 129, -1),
                                             ((256, 256), 300, 1), ((1 << 16,), 257, -1),
                                             ((256, 1024), 33, 1)])
def test_pipelined_256_point_column_passes(tc, dims, batch, sign):
    """FP16 256-point column passes run as persistent kernels that prefetch the
    next tile: tile counts below, just above and well above the resident
    grid (ragged last round), both directions, 2D and the second pass of a
    65536-point plan."""
    passes = tc.dry_run(dims, batch, direction=sign)["passes"]
    assert any(p["kernel"] == "col" and p["L"] == 256 and not p["tstore"] for p in passes), passes
    _check(tc, dims, batch, sign=sign, seed=13)


@pytest.mark.parametrize("n,sign", [(1 << 15, -1), (1 << 15, 1), (1 << 23, -1)])
def test_split_early_twiddle_lookups(tc, n, sign):
    """Split plans whose 128-point first pass (radix-8 stage, then one radix-16
    stage with the inter-pass twiddle) loads that twiddle's table entries
    before its HBM reads."""
    passes = tc.dry_run((n,), 1, direction=sign, precision="split")["passes"]
    assert passes[0]["kernel"] == "col" and passes[0]["L"] == 128 and passes[0]["xtw"] == 1, passes
    _check(tc, (n,), 3 if n <= (1 << 15) else 1, prec="split", sign=sign, seed=12)


@pytest.mark.parametrize("dims", [(16, 16), (64, 512), (256, 256), (512, 128), (1024, 1024),
                                  (2048, 16), (128, 128), (256, 64), (32, 512), (16, 1024),
                                  (64, 64), (32, 128), (128, 64), (64, 128), (32, 256)])
def test_2d(tc, dims):
    """From (128, 128) on: arrays of 16384 points (one plane pass per array)
    and, in FP16, of 4096 / 8192 points (4 / 2 arrays per workgroup; batches of
    3, 5 and 7 end inside a workgroup)."""
    _check(tc, dims, 3 if dims[0] * dims[1] <= 65536 else 1)
    if dims[0] * dims[1] < 16384:
        _check(tc, dims, 5)
        _check(tc, dims, 7, sign=1)
    if dims[0] * dims[1] == 16384 and dims[1] >= 64:
        _check(tc, dims, 5, sign=1)
        _check(tc, dims, 2, prec="split")


@pytest.mark.parametrize("dims", [(256,), (4096,), (16384,), (1 << 16,), (1 << 20,), (128, 128),
                                  (512, 512)])
def test_split_precision(tc, dims):
    _check(tc, dims, 3 if np.prod(dims) <= 65536 else 1, prec="split")


@pytest.mark.parametrize("n", [16, 256, 4096, 1 << 16])
def test_fp32_radix2_comparator(tc, n):
    _check(tc, (n,), 5, prec="fp32_radix2")
    _check(tc, (n,), 2, prec="fp32_radix2", inplace=True)


@pytest.mark.parametrize("dims", [(4096,), (1 << 16,), (256, 256)])
def test_in_place(tc, dims):
    _check(tc, dims, 3, inplace=True)


def test_deterministic(tc):
    import torch
    x = torch.from_numpy(inputs.uniform((64, 4096), 1)).cuda()
    p = tc.Plan((4096,), 64)
    a = p(x).cpu().numpy()
    b = p(x).cpu().numpy()
    assert np.array_equal(a.view(np.uint16), b.view(np.uint16))


def test_tone_rows(tc):
    """Unit tones x[n] = exp(+2 pi i f n/N): the peak lands at bin f with |Y_f| 2^S ~ N."""
    n, batch = 4096, 200
    x, tones = inputs.batched_1d(n, batch, seed=0)
    p = tc.Plan((n,), batch)
    y = run_plan(p, x)
    for r, f in zip(tones.rows, tones.freqs):
        assert int(np.argmax(np.abs(y[r]))) == int(f)
        assert abs(abs(y[r, f]) - n) / n < 5e-3
        off = np.delete(np.abs(y[r]) ** 2, f).sum() / (n * n)
        assert off < 1e-4


def _pass1_reference(xc, n1):
    """Eq. 3 per-pass invariant of the four-step split N = N1 * M: pass 1 holds
    Z[m][k1] = W_N^{m k1} * DFT_N1 over n1 of x[n1 M + m] (oracle sub-DFTs,
    FP64 twiddles)."""
    b, n = xc.shape
    m = n // n1
    sub = np.ascontiguousarray(xc.reshape(b, n1, m).transpose(0, 2, 1))  # [b][m][n1]
    z = oracle.fft(sub.reshape(b * m, n1), -1).reshape(b, m, n1)
    mm = np.arange(m, dtype=np.int64)[:, None]
    kk = np.arange(n1, dtype=np.int64)[None, :]
    tw = np.exp(-2j * np.pi * ((mm * kk) % n) / n)
    return z * tw


@pytest.mark.parametrize("prec", ["fp16", "split"])
@pytest.mark.parametrize("n,batch", [(1 << 16, 3), (1 << 20, 2), (1 << 23, 1)])
def test_pass1_intermediate(tc, n, batch, prec):
    """The first pass of a multi-pass plan alone: its output equals the oracle's
    N1-point sub-DFTs times W_N twiddles, transposed to [m][k1] (Eq. 3)."""
    import torch
    log(f"case pass1 n={n} batch={batch} prec={prec}")
    if prec == "split":
        x = inputs.to_split(inputs.uniform_f64((batch, n), 5))
        host = np.stack([x[0], x[1]])
        tol = SPLIT_TOL
    else:
        x = inputs.uniform((batch, n), 5)
        host = x
        tol = FP16_TOL
    p = tc.Plan((n,), batch, precision=prec)
    d = p.describe()
    assert len(d["passes"]) >= 2
    n1 = d["passes"][0]["L"]
    s1 = d["passes"][0]["scale"]
    t = torch.from_numpy(np.ascontiguousarray(host)).cuda()
    out = p.run_passes(t, 1)
    torch.cuda.synchronize()
    y = out.cpu().numpy().astype(np.float64)
    if prec == "split":
        z = (y[0, ..., 0] + 2.0 ** -11 * y[1, ..., 0]) + 1j * (y[0, ..., 1] + 2.0 ** -11 * y[1, ..., 1])
    else:
        z = y[..., 0] + 1j * y[..., 1]
    z = z.reshape(batch, n // n1, n1) * 2.0 ** s1
    from tests.gpu_util import to_complex
    ref = _pass1_reference(to_complex(x).reshape(batch, n), n1)
    e = np.linalg.norm((z - ref).reshape(batch, -1), axis=1) / np.linalg.norm(
        ref.reshape(batch, -1), axis=1)
    log(f"  N1={n1} s1={s1} max rel L2 = {e.max():.3e}")
    assert e.max() <= tol
    # all passes through the same entry point is the whole transform
    full = p.run_passes(t, len(d["passes"]))
    ref_full = p(t)
    torch.cuda.synchronize()
    assert torch.equal(full.view(torch.int16), ref_full.view(torch.int16))


def test_2d_row_pass_intermediate(tc):
    """The row pass of a 2D plan alone: natural-order row transforms."""
    import torch
    nx, ny, batch = 64, 512, 3
    x = inputs.uniform((batch, nx, ny), 6)
    p = tc.Plan((nx, ny), batch)
    s1 = p.describe()["passes"][0]["scale"]
    t = torch.from_numpy(x).cuda()
    y = p.run_passes(t, 1).cpu().numpy().astype(np.float64)
    z = (y[..., 0] + 1j * y[..., 1]) * 2.0 ** s1
    from tests.gpu_util import to_complex
    ref = oracle.fft(to_complex(x).reshape(batch * nx, ny), -1).reshape(batch, nx, ny)
    e = np.linalg.norm((z - ref).reshape(batch * nx, -1), axis=1) / np.linalg.norm(
        ref.reshape(batch * nx, -1), axis=1)
    assert e.max() <= FP16_TOL


@pytest.mark.parametrize("dims", [(4096,), (1 << 20,), (256, 256)])
def test_parseval_on_gpu_output(tc, dims):
    """Parseval: N * sum|x|^2 = sum|X|^2 per transform, on the GPU result
    (2^S restored), within the FP16 storage error."""
    batch = 4
    x = inputs.uniform((batch, *dims), 9)
    p = tc.Plan(dims, batch)
    y = run_plan(p, x)
    from tests.gpu_util import to_complex
    xc = to_complex(x).reshape(batch, -1)
    n = xc.shape[1]
    lhs = n * np.sum(np.abs(xc) ** 2, axis=1)
    rhs = np.sum(np.abs(y.reshape(batch, -1)) ** 2, axis=1)
    assert np.all(np.abs(rhs - lhs) / lhs <= 2 * FP16_TOL)
