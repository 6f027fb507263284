"""Shard plans of a distributed four-step transform, without a GPU.

* the planner (tcfft_shard_dry_run): step-1 and step-2 passes, buffer sizes,
  rejected arguments;
* the layout algebra the header documents: steps 1 and 2 written out with the
  oracle's DFTs on the documented layouts, joined by the documented exchange,
  give the N-point DFT (Sec. 2.1, Eq. 3 with n = n1 M + m, k = k1 + N1 k').
  This pins the index bookkeeping the GPU shard tests rely on."""
import numpy as np
import pytest

import oracle
from tests import shard_layout as sl


@pytest.fixture(scope="module")
def tc():
    from paper_2104_11471_amd import tcfft
    return tcfft


@pytest.mark.parametrize("lg,g", [(15, 2), (20, 4), (22, 8), (23, 8), (24, 8), (27, 16)])
def test_shard_plan_geometry(tc, lg, g):
    n = 1 << lg
    d = tc.shard_dry_run(n, 2, g, g - 1)
    n1 = d["shard_n1"]
    m = n // n1
    assert d["nshards"] == g and d["shard"] == g - 1
    assert d["buffer_bytes"] == 2 * (n // g) * 4 and d["workspace_bytes"] == 0
    p = d["passes"]
    # step 1: N1-point column DFTs over the shard's M/G columns, twiddle, blocked store
    assert p[0]["kernel"] == "col" and p[0]["L"] == n1 and p[0]["xtw"] == 1 and p[0]["tstore"] == 1
    assert p[0]["s_in"] == m // g and p[0]["xmod"] == n
    # step 2: the M-point DFTs over m, one column pass or two
    lens = [q["L"] for q in p[1:]]
    assert int(np.prod(lens)) == m and all(q["kernel"] == "col" for q in p[1:])
    assert len(p) == (2 if m <= 2048 else 3)
    assert d["scale_log2"] == sum(q["scale"] for q in p)
    ds = tc.shard_dry_run(n, 2, g, 0, precision="split")
    assert ds["buffer_bytes"] == 2 * (n // g) * 8


@pytest.mark.parametrize("n,g,shard,flags,status", [
    (1 << 20, 3, 0, 0, 1),      # nshards not a power of two
    (1 << 20, 4, 4, 0, 1),      # shard out of range
    (1 << 20, 4, -1, 0, 1),
    (1 << 20, 1, 0, 0, 1),      # one device is not a distributed transform
    (16384, 2, 0, 0, 2),        # single-pass length
    (1 << 20, 512, 0, 0, 2),    # N1 / G < 4
    (1 << 20, 4, 0, 8, 2),      # real input
    (3 << 18, 4, 0, 0, 2),      # not a power of two
])
def test_shard_plan_rejects(tc, n, g, shard, flags, status):
    with pytest.raises(tc.TcfftError) as e:
        tc.shard_dry_run(n, 1, g, shard, flags=flags)
    assert e.value.status == status


def _step1_model(xs, n, n1, g, shard):
    """Step 1 as documented, with the oracle's DFT: xs (B, N1 * ml) ->
    (B, N/G) laid out [G][ml][n1l]."""
    m, n1l, ml = sl.geometry(n, n1, g)
    b = xs.shape[0]
    cols = np.ascontiguousarray(xs.reshape(b, n1, ml).transpose(0, 2, 1))  # [b][m_l][n1]
    z = oracle.fft(cols.reshape(b * ml, n1), -1).reshape(b, ml, n1)
    mg = (shard * ml + np.arange(ml, dtype=np.int64))[:, None]
    k1 = np.arange(n1, dtype=np.int64)[None, :]
    z = z * np.exp(-2j * np.pi * ((mg * k1) % n) / n)
    # [m_l][k1] -> [h][m_l][k1_l]
    return z.reshape(b, ml, g, n1l).transpose(0, 2, 1, 3).reshape(b, n // g)


def _step2_model(r, n, n1, g):
    """Step 2 as documented: (B, N/G) laid out [M][n1l] -> DFT over m."""
    m, n1l, _ = sl.geometry(n, n1, g)
    b = r.shape[0]
    cols = np.ascontiguousarray(r.reshape(b, m, n1l).transpose(0, 2, 1))
    y = oracle.fft(cols.reshape(b * n1l, m), -1).reshape(b, n1l, m)
    return y.transpose(0, 2, 1).reshape(b, n // g)


@pytest.mark.parametrize("n,n1,g", [(1 << 10, 32, 4), (1 << 12, 16, 2), (1 << 12, 64, 16)])
def test_shard_layout_algebra_gives_the_dft(n, n1, g):
    rng = np.random.default_rng(n + g)
    x = rng.standard_normal((2, n)) + 1j * rng.standard_normal((2, n))
    xp = x[None]  # plane axis
    s1 = [_step1_model(sl.slab(xp, n1, g, s)[0], n, n1, g, s)[None] for s in range(g)]
    recv = sl.exchange(s1, n, n1, g, lambda parts: np.concatenate(parts, axis=2))
    out = [_step2_model(r[0], n, n1, g)[None] for r in recv]
    y = sl.assemble(out, n, n1, g)[0]
    ref = oracle.fft(x, -1)
    assert np.abs(y - ref).max() <= 1e-10 * np.abs(ref).max()


def test_shard_layout_catches_a_wrong_exchange(tc):
    """The check above is sensitive to the bookkeeping: swapping two devices'
    chunks in the exchange breaks it."""
    n, n1, g = 1 << 10, 32, 4
    rng = np.random.default_rng(3)
    x = (rng.standard_normal((1, n)) + 1j * rng.standard_normal((1, n)))[None]
    s1 = [_step1_model(sl.slab(x, n1, g, s)[0], n, n1, g, s)[None] for s in range(g)]
    s1[0], s1[1] = s1[1], s1[0]
    recv = sl.exchange(s1, n, n1, g, lambda parts: np.concatenate(parts, axis=2))
    y = sl.assemble([_step2_model(r[0], n, n1, g)[None] for r in recv], n, n1, g)[0]
    assert np.abs(y - oracle.fft(x[0], -1)).max() > 1e-3
