"""Shard plans of a distributed four-step transform on one GPU, through the
C ABI (tcfft_plan_create_shard / tcfft_exec_shard).

* step 1 of one shard at the workload's real shape (N = 2^24, G = 8) against
  the oracle's N1-point sub-DFTs of that shard's columns times FP64 twiddles
  W_N^{m k1} at the columns' global index m (Sec. 2.1, Eq. 3);
* every shard's step 1, the all-to-all emulated by copies on the GPU, every
  shard's step 2: the assembled result equals the oracle's N-point DFT
  (two-factor and three-factor splits, FP16 and split, both directions).
Tolerance: relative L2 per transform 5e-3 (FP16), 2e-5 (split)."""
import numpy as np
import pytest

import oracle
from paper_2104_11471_amd import inputs
from tests import shard_layout as sl
from tests.gpu_util import FP16_TOL, SPLIT_TOL, log

pytestmark = pytest.mark.gpu


def _host_input(n, batch, split, seed):
    if split:
        hi, lo = inputs.to_split(inputs.uniform_f64((batch, n), seed))
        return np.stack([hi, lo]), oracle.from_split(hi, lo)
    x = inputs.uniform((batch, n), seed)
    return x[None], oracle.from_half(x)


def _to_tensor(a, split):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a)).cuda()
    return t if split else t[0]


def _complex(y, split):
    """tensor (P?, B, pts, 2) -> complex128 (B, pts)."""
    z = y.cpu().numpy().astype(np.float64)
    if split:
        return (z[0, ..., 0] + 2.0 ** -11 * z[1, ..., 0]) + 1j * (z[0, ..., 1] + 2.0 ** -11 * z[1, ..., 1])
    return z[..., 0] + 1j * z[..., 1]


@pytest.mark.parametrize("prec", ["fp16", "split"])
@pytest.mark.parametrize("shard", [0, 3, 7])
def test_shard_step1_at_2_24(shard, prec):
    import torch
    from paper_2104_11471_amd import tcfft
    n, g, batch = 1 << 24, 8, 1
    split = prec == "split"
    log(f"case shard step1 N=2^24 G={g} shard={shard} prec={prec}")
    host, xc = _host_input(n, batch, split, 11)
    p = tcfft.ShardPlan(n, batch, g, shard, precision=prec)
    d = p.describe()
    n1 = d["shard_n1"]
    s1 = d["passes"][0]["scale"]
    m, n1l, ml = sl.geometry(n, n1, g)
    xs = sl.slab(host, n1, g, shard)
    y = p.step1(_to_tensor(xs, split))
    torch.cuda.synchronize()
    z = _complex(y, split) * 2.0 ** s1                      # [h][m_l][k1_l]
    z = z.reshape(batch, g, ml, n1l).transpose(0, 2, 1, 3).reshape(batch, ml, n1)  # [m_l][k1]
    # oracle: N1-point DFTs over n1 of the shard's columns, FP64 twiddles
    cols = xc.reshape(batch, n1, m)[:, :, shard * ml:(shard + 1) * ml]
    sub = oracle.fft(np.ascontiguousarray(cols.transpose(0, 2, 1)).reshape(batch * ml, n1), -1)
    mg = (shard * ml + np.arange(ml, dtype=np.int64))[:, None]
    k1 = np.arange(n1, dtype=np.int64)[None, :]
    ref = sub.reshape(batch, ml, n1) * np.exp(-2j * np.pi * ((mg * k1) % n) / n)
    e = np.linalg.norm((z - ref).reshape(batch, -1), axis=1) / np.linalg.norm(
        ref.reshape(batch, -1), axis=1)
    log(f"  N1={n1} M/G={ml} s1={s1} rel L2 {e.max():.3e}")
    assert e.max() <= (SPLIT_TOL if split else FP16_TOL)


@pytest.mark.parametrize("prec", ["fp16", "split"])
@pytest.mark.parametrize("n,g,batch,direction", [
    (1 << 20, 4, 2, -1),     # N1 x M = 1024 x 1024: step 2 is one pass
    (1 << 20, 8, 1, 1),      # inverse
    (1 << 23, 8, 1, -1),     # 128 x (256 x 256): step 2 is two passes
    (1 << 16, 16, 3, -1),
])
def test_shard_end_to_end(n, g, batch, direction, prec):
    import torch
    from paper_2104_11471_amd import tcfft
    split = prec == "split"
    log(f"case shard end-to-end N={n} G={g} batch={batch} dir={direction} prec={prec}")
    host, xc = _host_input(n, batch, split, 12)
    plans = [tcfft.ShardPlan(n, batch, g, s, direction=direction, precision=prec)
             for s in range(g)]
    n1 = plans[0].describe()["shard_n1"]
    scale = plans[0].scale_log2
    assert all(p.describe()["shard_n1"] == n1 and p.scale_log2 == scale for p in plans)
    xt = torch.from_numpy(np.ascontiguousarray(host)).cuda()          # (P, B, N, 2)
    step1 = []
    for s, p in enumerate(plans):
        xs = sl.slab(xt, n1, g, s).contiguous()
        y = p.step1(xs if split else xs[0])
        step1.append(y if split else y[None])
    recv = sl.exchange(step1, n, n1, g, lambda parts: torch.cat(parts, dim=2))
    out = []
    for p, r in zip(plans, recv):
        y = p.step2(r.contiguous() if split else r[0].contiguous())
        out.append((y if split else y[None]).cpu().numpy())
    torch.cuda.synchronize()
    full = sl.assemble(out, n, n1, g)                                   # (P, B, N, 2)
    z = _complex(torch.from_numpy(full if split else full[0]), split) * 2.0 ** scale
    ref = oracle.fft(xc, direction)
    e = oracle.rel_l2(z, ref)
    log(f"  N1={n1} S={scale} passes={[q['L'] for q in plans[0].describe()['passes']]} "
        f"max rel L2 {e.max():.3e}")
    assert e.max() <= (SPLIT_TOL if split else FP16_TOL)


def test_shard_plan_refuses_plain_exec():
    import torch
    from paper_2104_11471_amd import tcfft
    p = tcfft.ShardPlan(1 << 20, 1, 4, 0)
    x = torch.zeros(p.in_shape(), dtype=torch.float16, device="cuda")
    with pytest.raises(tcfft.TcfftError) as e:
        p.exec_raw(x.data_ptr(), torch.empty_like(x).data_ptr(), 0)
    assert e.value.status == 2
    with pytest.raises(tcfft.TcfftError):
        p.step1(x, x)  # in == out
