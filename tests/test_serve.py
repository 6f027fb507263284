"""Serving loop: continuous batching, memory admission, alone-vs-mix results."""
import numpy as np
import pytest

from paper_2104_11471_amd import inputs


@pytest.mark.gpu
@pytest.mark.parametrize("graphs,window", [(False, 0), (True, 100)])
def test_stream_results_equal_alone(graphs, window):
    """A short Poisson stream of the mixed population: every request completes,
    and sampled results are bitwise the results of the same request run alone,
    with direct launches and with HIP-graph replay plus a batching window."""
    import torch
    from paper_2104_11471_amd import serve, tcfft
    tcfft.tune_cache_clear()
    reqs = inputs.serving_stream(rate_hz=20000, duration_s=0.1, seed=3)
    # keep 2^20 requests few to bound the test's memory
    pool = serve.PayloadPool(reqs, slots=16)
    srv = serve.Server(nslots=4, mem_budget_bytes=8 << 30, max_batch_jobs=128,
                       use_graphs=graphs, batch_window_us=window)
    srv.prepare({(r.rank, tuple(r.dims), -1, "split" if r.split else "fp16") for r in reqs})
    rng = np.random.default_rng(0)
    check = set(rng.choice([r.rid for r in reqs], size=min(40, len(reqs)), replace=False).tolist())
    t0 = serve.now_ns()
    recs, keep = serve.run_stream(srv, reqs, pool, check_tags=check)
    wall = (serve.now_ns() - t0) / 1e9
    st = srv.stats()
    summary = serve.summarize(recs, wall)
    print(summary, st)
    assert st["completed"] == len(reqs) and st["rejected"] == 0
    assert summary["requests"] == len(reqs)
    assert st["max_inflight_bytes"] <= 8 << 30
    byid = {r.rid: r for r in reqs}
    # each checked request again, alone on the idle server (same plans, no
    # other request in its batch): bitwise the result it got in the mix
    for tag, got in keep.items():
        r = byid[tag]
        k = serve.shape_class(r)
        out = torch.empty_like(pool.out[k][0])
        assert srv.submit(r.rank, r.dims, r.batch, -1, k[2], pool.inp[k].data_ptr(),
                          out.data_ptr(), tag) == 0
        srv.wait_idle(20000)
        done = srv.poll()
        assert [d[0] for d in done] == [tag] and done[0][1] == 0
        torch.cuda.synchronize()
        alone = serve.PayloadPool.view(out, k, r.batch)
        got = serve.PayloadPool.view(got, k, r.batch)
        assert torch.equal(got.view(torch.int16), alone.view(torch.int16)), (tag, k)
        # and it is the DFT: a sampled transform against the oracle
        x = serve.PayloadPool.view(pool.inp[k], k, r.batch)
        _check_against_oracle(r, k, x, alone)
    srv.close()


def _check_against_oracle(r, k, x, y):
    import oracle
    from tests.gpu_util import FP16_TOL, SPLIT_TOL
    xs = x.cpu().numpy().astype(np.float64)
    ys = y.cpu().numpy().astype(np.float64)
    if k[2] == "split":
        xc = (xs[0, 0, ..., 0] + 2.0 ** -11 * xs[1, 0, ..., 0]) + 1j * (xs[0, 0, ..., 1] + 2.0 ** -11 * xs[1, 0, ..., 1])
        yc = (ys[0, 0, ..., 0] + 2.0 ** -11 * ys[1, 0, ..., 0]) + 1j * (ys[0, 0, ..., 1] + 2.0 ** -11 * ys[1, 0, ..., 1])
        tol = SPLIT_TOL
    else:
        xc = xs[0, ..., 0] + 1j * xs[0, ..., 1]
        yc = ys[0, ..., 0] + 1j * ys[0, ..., 1]
        tol = FP16_TOL
    ref = oracle.fft(xc, -1) if r.rank == 1 else oracle.fft2(xc, -1)
    d = tcfft_scale(r, k)
    err = np.linalg.norm(yc * 2.0 ** d - ref) / np.linalg.norm(ref)
    assert err <= tol, (r.dims, r.batch, k, err)


def tcfft_scale(r, k):
    """Scale of the server's plan for this shape: the server tunes its
    multi-pass 1D single-transform plans, and the same key hits the same
    cached choice."""
    from paper_2104_11471_amd import tcfft
    flags = tcfft.FLAG_TUNE if (r.rank == 1 and r.dims[0] > 16384) else 0
    return tcfft.Plan(r.dims, 1, precision=k[2], flags=flags).scale_log2


@pytest.mark.gpu
def test_admission_by_memory():
    """With a budget that fits one request at a time, requests still all
    complete, never more than the budget is in flight, and a request larger
    than the budget is refused."""
    import torch
    from paper_2104_11471_amd import serve, tcfft
    n, b = 4096, 16
    one = 2 * n * b * 4
    srv = serve.Server(nslots=4, mem_budget_bytes=one + 1024, max_batch_jobs=64)
    x = torch.from_numpy(inputs.uniform((b, n), 1)).cuda()
    outs = [torch.empty_like(x) for _ in range(12)]
    for i, o in enumerate(outs):
        assert srv.submit(1, (n,), b, -1, "fp16", x.data_ptr(), o.data_ptr(), i) == 0
    big = torch.empty((2 * b, n, 2), dtype=torch.float16, device="cuda")
    assert srv.submit(1, (n,), 2 * b, -1, "fp16", big.data_ptr(), big.data_ptr(), 99) == 4
    srv.wait_idle(20000)
    done = srv.poll()
    assert sorted(t for t, *_ in done) == list(range(12))
    st = srv.stats()
    assert st["max_inflight_bytes"] <= one + 1024 and st["max_batch_jobs"] == 1
    assert st["rejected"] == 1
    ref = tcfft.Plan((n,), b)(x)
    torch.cuda.synchronize()
    for o in outs:
        assert torch.equal(o.view(torch.int16), ref.view(torch.int16))
    srv.close()


def test_server_config_validation():
    """Bad configurations are refused before any device work (CPU)."""
    from paper_2104_11471_amd import serve, tcfft
    for cfg in [(0, 1 << 20, 4), (17, 1 << 20, 4), (2, 0, 4), (2, 1 << 20, 0)]:
        with pytest.raises(tcfft.TcfftError) as e:
            serve.Server(nslots=cfg[0], mem_budget_bytes=cfg[1], max_batch_jobs=cfg[2])
        assert e.value.status == 1
