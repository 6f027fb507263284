"""Two-pass plans whose second pass is a row pass with a transposed store
(pass 1 stores in natural order), against the oracle and the default plan."""
import os
import tempfile

import numpy as np
import pytest

from paper_2104_11471_amd import inputs
from tests.gpu_util import FP16_TOL, SPLIT_TOL, log, reference, rel_err, run_plan

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tc():
    from paper_2104_11471_amd import tcfft
    return tcfft


def forced_plan(tc, n, batch, n1, n2, prec="fp16", cmax=32, chunk=0, sign=-1):
    lg = (batch - 1).bit_length()
    pc = 0 if prec == "fp16" else 1
    fd, path = tempfile.mkstemp(suffix=".txt")
    with os.fdopen(fd, "w") as fh:
        fh.write(f"tcfft-tune 3\nr1_{n}x1_b{lg}_p{pc} 256 {cmax} 2 {n1} {n2} 0 {chunk} 1 1.0\n")
    tc.tune_cache_clear()
    tc.tune_cache_load(path)
    os.unlink(path)
    p = tc.Plan((n,), batch, direction=sign, precision=prec, flags=tc.FLAG_TUNE)
    tc.tune_cache_clear()
    d = p.describe()
    assert [(q["kernel"], q["L"], q["tstore"]) for q in d["passes"]] == [("col", n1, 0), ("row", n2, 1)], d
    return p


@pytest.mark.parametrize("prec", ["fp16", "split"])
@pytest.mark.parametrize("n,n1,n2,batch", [(1 << 16, 256, 256, 3), (1 << 15, 64, 512, 5),
                                           (1 << 20, 1024, 1024, 2), (1 << 19, 2048, 256, 1)])
def test_p2row_parity(tc, n, n1, n2, batch, prec):
    log(f"case p2row n={n} = {n1} x {n2} batch={batch} prec={prec}")
    if prec == "split":
        x = inputs.to_split(inputs.uniform_f64((batch, n), 11))
        tol = SPLIT_TOL
    else:
        x = inputs.uniform((batch, n), 11)
        tol = FP16_TOL
    for sign in (-1, 1):
        p = forced_plan(tc, n, batch, n1, n2, prec, sign=sign)
        y = run_plan(p, x)
        e = rel_err(y, reference(x, 1, sign), 1)
        log(f"  sign={sign} max rel L2 = {e.max():.3e}")
        assert e.max() <= tol


def test_p2row_chunked_and_grouped(tc):
    """Chunked execution and the grouped launch give the unchunked single
    launch's bits."""
    import torch
    n, batch = 1 << 16, 16
    x = torch.from_numpy(inputs.uniform((batch, n), 12)).cuda()
    a = forced_plan(tc, n, batch, 256, 256)(x)
    b = forced_plan(tc, n, batch, 256, 256, chunk=4)(x)
    p = forced_plan(tc, n, batch, 256, 256)
    c = torch.empty_like(x)
    tc.exec_many([p], [x], [c])
    torch.cuda.synchronize()
    assert torch.equal(a.view(torch.int16), b.view(torch.int16))
    assert torch.equal(a.view(torch.int16), c.view(torch.int16))


def test_p2row_pass1_intermediate(tc):
    """Pass 1 alone: natural-order [k1][n2] layout of the Eq. 3 intermediate."""
    import oracle
    import torch
    n, n1, n2, batch = 1 << 16, 256, 256, 2
    x = inputs.uniform((batch, n), 13)
    p = forced_plan(tc, n, batch, n1, n2)
    s1 = p.describe()["passes"][0]["scale"]
    out = p.run_passes(torch.from_numpy(x).cuda(), 1)
    y = out.cpu().numpy().astype(np.float64)
    z = (y[..., 0] + 1j * y[..., 1]).reshape(batch, n1, n2) * 2.0 ** s1
    xc = oracle.from_half(x).reshape(batch, n1, n2)
    sub = oracle.fft(np.ascontiguousarray(xc.transpose(0, 2, 1)).reshape(batch * n2, n1), -1)
    sub = sub.reshape(batch, n2, n1).transpose(0, 2, 1)  # [b][k1][n2]
    kk = np.arange(n1, dtype=np.int64)[:, None]
    mm = np.arange(n2, dtype=np.int64)[None, :]
    ref = sub * np.exp(-2j * np.pi * ((kk * mm) % n) / n)
    e = np.linalg.norm((z - ref).reshape(batch, -1), axis=1) / np.linalg.norm(ref.reshape(batch, -1), axis=1)
    assert e.max() <= FP16_TOL
