#!/usr/bin/env python3
"""Benchmark of the batched FP16 matrix-core FFT on one MI355X.

Workload (the paper's batched 1D case, Sec. 5.1: inputs uniform in [-1, 1],
batch large enough to fill the GPU): N in {4096, 16384, 65536} with
batch = 2^27 / N (512 MiB of FP16 complex input per size) plus 1 % unit-tone
rows.  One step = one forward transform of each of the three batches.

Metric: GFLOP/s with the 5 N log2 N convention, whole job; also HBM GB/s of the
algorithmic traffic (8 B per point: one read and one write of FP16 complex) as
a fraction of 8 TB/s.  Inputs are resident in HBM before the timed region.

Prints one JSON line (rank 0).  `--gpus N` with N > 1 exits: this build runs on
one GPU.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
SIZES = (4096, 16384, 65536)
TOTAL_POINTS = 1 << 27


def flops(n: int, batch: int) -> float:
    return 5.0 * n * math.log2(n) * batch


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def time_launches(fn, reps: int, stream, warm: int = 5) -> float:
    """Average duration (s) of fn() over reps, HIP events on `stream`, after
    `warm` untimed calls (clocks ramp back up after the GPU idled)."""
    import torch
    for _ in range(warm):
        fn()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for _ in range(reps):
        fn()
    end.record(stream)
    end.synchronize()
    return start.elapsed_time(end) / 1e3 / reps


def time_trials(fn, stream, min_s: float = 0.1, trials: int = 5) -> float:
    """Median over `trials` of the mean duration (s) of R back-to-back calls,
    R chosen so that each trial times at least `min_s` (after 5 warm calls)."""
    est = time_launches(fn, 3, stream, warm=5)
    reps = max(10, int(math.ceil(min_s / max(est, 1e-7))))
    res = sorted(time_launches(fn, reps, stream, warm=0) for _ in range(trials))
    return res[len(res) // 2]


def time_cold(fn, reps: int, stream, flush) -> float:
    """Average duration (s) of fn() with the memory-side cache flushed before
    each call (a 512 MiB buffer rewritten between the timed calls)."""
    import torch
    tot = 0.0
    for _ in range(reps):
        flush.add_(1)
        start = torch.cuda.Event(enable_timing=True)
        end = torch.cuda.Event(enable_timing=True)
        start.record(stream)
        fn()
        end.record(stream)
        end.synchronize()
        tot += start.elapsed_time(end) / 1e3
    return tot / reps


def measured_traffic(kernel_name: str):
    """HBM bytes per launch of `kernel_name` from the committed rocprofv3
    counter summary, or None when the kernel source changed since."""
    import hashlib
    try:
        rec = json.load(open(os.path.join(ROOT, "profiles", "hbm_traffic.json")))
        src = b"".join(open(os.path.join(ROOT, "paper_2104_11471_amd", "csrc", f), "rb").read()
                       for f in ("common.h", "pass_kernels.h"))
    except OSError:
        return None
    if hashlib.sha256(src).hexdigest()[:16] != rec.get("kernels_sha256_16"):
        return None
    k = rec["per_launch_kib"].get(kernel_name)
    if not k:
        return None
    return int(round((k["fetch"] * rec["fetch_factor"] + k["write"] * rec["write_factor"]) * 1024))


def kernel_name(q: dict) -> str:
    """Template name of a pass's kernel from the plan description."""
    r0 = q["radices"][0] if q["radices"][0] != 16 else 1
    if q["kernel"] == "row":
        wgp = q["C"] if q["C"] else 16384  # points per workgroup
        return (f"row_kernel<{q['L']}, {r0}, {q['NT']}, false, {str(bool(q['tstore'])).lower()}, "
                f"{q['real']}, {wgp}>")
    if q["kernel"] == "col":
        return (f"col_kernel<{q['L']}, {r0}, {q['C']}, {q['NT']}, false, "
                f"{str(bool(q['xtw'])).lower()}, {str(bool(q['tstore'])).lower()}>")
    return f"{q['kernel']}_kernel<{q['L']}>"


def pass_times(plan, x, y, stream, reps: int = 10) -> list:
    """HIP-event time (us) of each pass of a multi-pass plan: the first k
    passes timed alone (tcfft_exec_passes), differences of the prefixes."""
    pref = [0.0]
    for _ in range(20):  # steady clocks (the caller may have left the GPU idle)
        plan.run_passes(x, plan.num_launches, out=y, stream=stream)
    for k in range(1, plan.num_launches + 1):
        pref.append(time_launches(lambda: plan.run_passes(x, k, out=y, stream=stream), reps,
                                  stream) * 1e6)
    return [round(pref[k] - pref[k - 1], 2) for k in range(1, len(pref))]


def accuracy_sample(plan, x_dev, y_dev, x_host, tones, rng, nsample=32):
    """Relative L2 of sampled transforms (random rows + every tone row) vs the oracle."""
    import oracle
    batch = x_host.shape[0]
    rows = np.unique(np.concatenate([rng.choice(batch, size=min(nsample, batch), replace=False),
                                     tones.rows]))
    y = y_dev[rows].cpu().numpy().astype(np.float64)
    z = (y[..., 0] + 1j * y[..., 1]) * 2.0 ** plan.scale_log2
    ref = oracle.fft(oracle.from_half(x_host[rows]), -1)
    e = oracle.rel_l2(z, ref)
    # Eq. (5) reading on the uniform rows only (tone rows have exact-zero bins)
    uni = ~np.isin(rows, tones.rows)
    eq5 = oracle.eq5_error(z[uni], ref[uni])
    return float(e.max()), float(np.sqrt(np.mean(e ** 2))), eq5, len(rows)


def cpu_baseline(xs, target_s: float):
    """The FP64 oracle (radix-2, C, OpenMP) on a bounded sample of the same
    workload: the first rows of each size's batch, sized so the whole run takes
    about target_s seconds of wall time."""
    import oracle
    threads = len(os.sched_getaffinity(0))
    # calibration on a small slice
    n0 = list(xs)[0]
    probe = oracle.from_half(xs[n0][0][:64])
    t = time.perf_counter()
    oracle.fft(probe, -1, threads)
    dt = max(time.perf_counter() - t, 1e-4)
    rate = flops(n0, 64) / dt  # flop/s
    sizes = list(xs)
    per_size = target_s / len(sizes)
    total_flop = 0.0
    total_t = 0.0
    parts = []
    for n in sizes:
        want = per_size * rate / flops(n, 1)
        rows = int(max(1, min(xs[n][0].shape[0], want)))
        reps = int(max(1, min(8, round(want / rows))))
        z = oracle.from_half(xs[n][0][:rows])
        t = time.perf_counter()
        for _ in range(reps):
            oracle.fft(z, -1, threads)
        total_t += time.perf_counter() - t
        total_flop += flops(n, rows) * reps
        parts.append(f"N={n} x {rows} rows x {reps}")
    return {"value": round(total_flop / total_t / 1e9, 3), "unit": "GFLOP/s", "cores": threads,
            "kind": "oracle",
            "sample": "FP64 radix-2 oracle on the first rows of each batch (" + ", ".join(parts)
                      + f"), {total_t:.1f} s"}


def other_workloads(stream) -> dict:
    """Timing + sampled accuracy of the other workloads: the N=256 x 64 latency
    case, long 1D (2^20 x 16, 2^22 x 4, 2^24 x 1), batched 2D (256^2 x 1024,
    512^2 x 256, 1024^2 x 64) and batched 3D (128^3 x 64, 256^3 x 8, 512^3 x 1;
    uniform inputs), FP16 and split.  Long 1D is also timed with the
    memory-side cache flushed before each call (its 64 MiB would otherwise stay
    resident between calls).  Not part of `value`."""
    import torch
    import oracle
    from paper_2104_11471_amd import inputs, tcfft
    out = {}
    # latency of the small case (unnormalised, as specified)
    x = torch.from_numpy(inputs.uniform((64, 256), 0)).cuda()
    p = tcfft.Plan((256,), 64, flags=tcfft.FLAG_NO_SCALE)
    y = torch.empty_like(x)
    for _ in range(20):
        p(x, y, stream=stream)
    dt = time_launches(lambda: p(x, y, stream=stream), 200, stream)
    out["1d_256x64"] = {"us": round(dt * 1e6, 2)}
    cases = [("1d", (1 << 20,), 16), ("1d", (1 << 22,), 4), ("1d", (1 << 24,), 1),
             ("2d", (256, 256), 1024), ("2d", (512, 512), 256), ("2d", (1024, 1024), 64),
             ("3d", (128, 128, 128), 64), ("3d", (256, 256, 256), 8), ("3d", (512, 512, 512), 1)]
    for kind, dims, batch in cases:
        for prec in ("fp16", "split"):
            split = prec == "split"
            if kind == "1d":
                xh, _, _ = inputs.long_1d(dims[0], batch, seed=0, as_split=split)
            elif kind == "2d":
                xh = inputs.smooth_2d(dims[0], dims[1], batch, seed=0, as_split=split)
            elif split:
                xh = inputs.to_split(inputs.uniform_f64((batch,) + dims, 0))
            else:
                xh = inputs.uniform((batch,) + dims, 0)
            host = np.stack(xh) if split else xh
            xd = torch.from_numpy(host).cuda()
            yd = torch.empty_like(xd)
            p = tcfft.Plan(dims, batch, precision=prec, flags=tcfft.FLAG_TUNE)
            p(xd, yd, stream=stream)
            dt = time_trials(lambda: p(xd, yd, stream=stream), stream)
            dt_cold = None
            if kind == "1d":  # 64 MiB of data fits the 256 MB memory-side cache: cold variant too
                with torch.cuda.stream(stream):
                    flush = torch.zeros(1 << 27, dtype=torch.int32, device=xd.device)
                    dt_cold = time_cold(lambda: p(xd, yd, stream=stream), 5, stream, flush)
                del flush
            npts = int(np.prod(dims)) * batch
            n = int(np.prod(dims))
            row = 0
            if n > (1 << 24):  # the oracle needs about a minute here; parity tests cover 3D
                err = None
            z = (yd[:, row] if split else yd[row]).cpu().numpy().astype(np.float64)
            if split:
                z = (z[0, ..., 0] + 2.0 ** -11 * z[1, ..., 0]) + 1j * (z[0, ..., 1] + 2.0 ** -11 * z[1, ..., 1])
                zin = oracle.from_split(xh[0][row], xh[1][row])
            else:
                z = z[..., 0] + 1j * z[..., 1]
                zin = oracle.from_half(xh[row])
            if n <= (1 << 24):
                ref = (oracle.fft(zin) if kind == "1d" else oracle.fft2(zin) if kind == "2d"
                       else oracle.fft3(zin[None])[0])
                err = float(oracle.rel_l2(z * 2.0 ** p.scale_log2, ref, axis=None))
            bpp = 16 if split else 8
            key = f"{kind}_{'x'.join(map(str, dims))}x{batch}_{prec}"
            out[key] = {"us": round(dt * 1e6, 1),
                        "us_cold_cache": round(dt_cold * 1e6, 1) if dt_cold else None,
                        "gflops": round(5.0 * n * math.log2(n) * batch / dt / 1e9, 1),
                        "gbs_alg": round(bpp * npts / dt / 1e9, 1),
                        "hbm_frac_alg": round(bpp * npts / dt / 1e9 / HBM_PEAK_GBS, 4),
                        "passes": p.num_launches, "choice": p.describe()["choice"],
                        "rel_l2_row0": err}
            log(f"{key}: {out[key]}")
            del xd, yd, p
            torch.cuda.empty_cache()
    out.update(real_workloads(stream))
    out.update(fp64_workloads(stream))
    return out


def fp64_workloads(stream) -> dict:
    """FP64 matrix-core path: batched 1D N = 4096 x 32768 and 256 x 524288
    (2^27 points, 2 GiB of complex FP64 each way): time, algorithmic HBM
    bytes (16 B read + 16 B written per point) and the FP64 matrix-core work
    (12 v_mfma_f64_16x16x4f64 = 24576 flops per 256 points per radix-16
    stage) against the 78.6 TFLOP/s FP64 peak; row-0 accuracy against the
    oracle.  Not part of `value`."""
    import torch
    import oracle
    from paper_2104_11471_amd import inputs, tcfft
    out = {}
    for n in (4096, 256):
        batch = TOTAL_POINTS // n
        z = inputs.uniform_f64((batch, n), 3)
        xd = torch.from_numpy(np.stack([z.real, z.imag], -1)).cuda()
        yd = torch.empty_like(xd)
        p = tcfft.Plan((n,), batch, tcfft.FORWARD, "fp64")
        dt = time_trials(lambda: p(xd, yd, stream=stream), stream)
        y0 = yd[0].cpu().numpy()
        err = float(oracle.rel_l2(y0[:, 0] + 1j * y0[:, 1], oracle.fft(z[0], -1), axis=None))
        stages = int(round(math.log2(n))) // 4
        mfma_flop = 96.0 * stages * TOTAL_POINTS
        key = f"1d_{n}x{batch}_fp64"
        out[key] = {"us": round(dt * 1e6, 1),
                    "gbs_alg": round(32.0 * TOTAL_POINTS / dt / 1e9, 1),
                    "hbm_frac_alg": round(32.0 * TOTAL_POINTS / dt / 1e9 / HBM_PEAK_GBS, 4),
                    "mfma_tflops": round(mfma_flop / dt / 1e12, 2),
                    "mfma_frac": round(mfma_flop / dt / 1e12 / 78.6, 4),
                    "rel_l2_row0": err}
        log(f"{key}: {out[key]}")
        del xd, yd, p, z
        torch.cuda.empty_cache()
    return out


def real_workloads(stream) -> dict:
    """Real-input transforms (R2C forward, C2R inverse) of N reals stored as
    N/2 complex words, the spectrum as N/2 + 1 bins: timing and row-0 accuracy
    against the oracle's rfft / irfft.  Algorithmic bytes are one read of the
    input and one write of the output.  Not part of `value`."""
    import torch
    import oracle
    from paper_2104_11471_amd import inputs, tcfft
    out = {}
    cases = [(8192, 16384, "fp16"), (8192, 16384, "split"), (32768, 4096, "fp16"),
             (1 << 21, 64, "fp16")]
    for n, batch, prec in cases:
        m = n // 2
        split = prec == "split"
        for dirn, name in ((tcfft.FORWARD, "r2c"), (tcfft.INVERSE, "c2r")):
            p = tcfft.Plan((n,), batch, dirn, prec, flags=tcfft.FLAG_REAL)
            words = m if dirn == tcfft.FORWARD else m + 1
            if split:
                hi, lo = inputs.to_split(inputs.uniform_f64((batch, words), 5))
                host = np.stack([hi, lo])
            else:
                host = inputs.uniform((batch, words), 5)
            xd = torch.from_numpy(host).cuda().reshape(p.in_shape())
            yd = torch.empty(p.out_shape(), dtype=torch.float16, device=xd.device)
            p(xd, yd, stream=stream)
            dt = time_trials(lambda: p(xd, yd, stream=stream), stream)
            y = yd.cpu().numpy().astype(np.float64)
            if split:
                x0 = host[0][0].astype(np.float64) + 2.0 ** -11 * host[1][0].astype(np.float64)
                y0 = y[0][0] + 2.0 ** -11 * y[1][0]
            else:
                x0 = host[0].astype(np.float64)
                y0 = y[0]
            x0c = x0[..., 0] + 1j * x0[..., 1]
            if dirn == tcfft.FORWARD:
                ref = oracle.rfft(x0.reshape(n))
                got = (y0[..., 0] + 1j * y0[..., 1]) * 2.0 ** p.scale_log2
            else:
                ref = oracle.irfft(x0c, n)
                got = y0 * 2.0 ** p.scale_log2
            bpe = 8 if split else 4
            alg = bpe * batch * (2 * m + 1)
            key = f"{name}_{n}x{batch}_{prec}"
            out[key] = {"us": round(dt * 1e6, 1), "gbs_alg": round(alg / dt / 1e9, 1),
                        "hbm_frac_alg": round(alg / dt / 1e9 / HBM_PEAK_GBS, 4),
                        "launches": p.num_launches, "real_kernel": p.describe()["real_kernel"],
                        "rel_l2_row0": float(oracle.rel_l2(got, ref, axis=None))}
            log(f"{key}: {out[key]}")
            del xd, yd, p
            torch.cuda.empty_cache()
    return out


def mixed_batch_leg(stream, single_pass: bool = False) -> dict:
    """One mixed batch of 256 requests drawn from the serving population (with
    `single_pass`, only its 1D requests of <= 16384 points), run by
    tcfft_exec_many as single launches (k_fused.hip; TCFFT_FUSED=1) and as
    per-(level, variant) grouped launches (TCFFT_FUSED=0): time per batch and
    launch counts.  Not part of `value`."""
    import torch
    from paper_2104_11471_amd import inputs, tcfft
    reqs = inputs.serving_stream(rate_hz=20000.0, duration_s=2.0, seed=7)
    if single_pass:
        reqs = [r for r in reqs if r.rank == 1 and r.dims[0] <= 16384]
    reqs = reqs[:256]
    plans, xs, ys = [], [], []
    cache = {}
    groups, classes = set(), set()
    for r in reqs:
        prec = "split" if r.split else "fp16"
        key = (tuple(r.dims), r.batch, prec)
        if key not in cache:
            cache[key] = tcfft.Plan(r.dims, r.batch, precision=prec)
        p = cache[key]
        if p.workspace_bytes > 0 and any(q is p for q in plans):
            continue  # a workspace-holding plan runs once per call
        plans.append(p)
        shape = (r.batch,) + tuple(r.dims)
        host = (np.stack(inputs.to_split(inputs.uniform_f64(shape, len(xs)))) if r.split
                else inputs.uniform(shape, len(xs)))
        xs.append(torch.from_numpy(host).cuda())
        ys.append(torch.empty_like(xs[-1]))
        for lv, q in enumerate(p.describe()["passes"]):
            groups.add((lv, q["kernel"], q["L"], q["C"], q["NT"], q["xtw"], q["tstore"], prec))
            classes.add((lv, prec, q["lds"] > 65536))
    out = {"jobs": len(plans), "transforms": int(sum(p.batch for p in plans))}
    for name, env in (("fused", "1"), ("fused_dep", "2"), ("grouped", "0")):
        old = os.environ.get("TCFFT_FUSED")
        if env is not None:
            os.environ["TCFFT_FUSED"] = env
        try:
            for _ in range(3):
                tcfft.exec_many(plans, xs, ys, stream=stream)
            dt = time_trials(lambda: tcfft.exec_many(plans, xs, ys, stream=stream), stream)
        finally:
            if old is None:
                os.environ.pop("TCFFT_FUSED", None)
            else:
                os.environ["TCFFT_FUSED"] = old
        out[f"{name}_us"] = round(dt * 1e6, 1)
    out["fused_launches"] = len(classes)  # one per (pass level, precision, LDS class)
    out["grouped_launches"] = len(groups)
    out["fused_wait_failures"] = tcfft.fused_wait_failures()
    log(f"mixed batch: {out}")
    return out


def serving_leg(seconds: float) -> dict:
    """Poisson stream (20k req/s) of the mixed request population through the
    continuous-batching scheduler: p50/p99 latency and throughput.  Payloads
    are pre-staged in device memory (at these rates they would exceed PCIe).
    The main figures use immediate dispatch with direct grouped launches; the
    same stream with HIP-graph replay and a 100 us batching window is reported
    beside them."""
    from paper_2104_11471_amd import inputs, serve
    reqs = inputs.serving_stream(rate_hz=20000.0, duration_s=seconds, seed=0)
    pool = serve.PayloadPool(reqs, slots=12)
    shapes = {(r.rank, tuple(r.dims), -1, "split" if r.split else "fp16") for r in reqs}

    def one(use_graphs, window):
        srv = serve.Server(nslots=4, mem_budget_bytes=24 << 30, max_batch_jobs=512,
                           use_graphs=use_graphs, batch_window_us=window)
        srv.prepare(shapes)
        serve.run_stream(srv, reqs[:64], pool)  # warm the kernels
        t0 = serve.now_ns()
        recs, _ = serve.run_stream(srv, reqs, pool)
        wall = (serve.now_ns() - t0) / 1e9
        out = serve.summarize(recs, wall)
        st = srv.stats()
        out.update({"offered_req_per_s": 20000.0, "seconds": seconds, "slots": 4,
                    "graphs": use_graphs, "batch_window_us": window,
                    "batches": st["batches"], "max_batch_jobs": st["max_batch_jobs"],
                    "max_inflight_bytes": st["max_inflight_bytes"],
                    "payload_pool_bytes": pool.nbytes()})
        srv.close()
        return out

    main = one(False, 0)
    alt = one(True, 100)
    keys = ("p50_us", "p99_us", "max_us", "req_per_s", "batches", "max_batch_jobs")
    main["graphs_window100"] = {k: alt[k] for k in keys}
    old = os.environ.get("TCFFT_FUSED")
    os.environ["TCFFT_FUSED"] = "0"
    try:
        grouped = one(False, 0)
    finally:
        if old is None:
            os.environ.pop("TCFFT_FUSED", None)
        else:
            os.environ["TCFFT_FUSED"] = old
    main["grouped_launches"] = {k: grouped[k] for k in keys}
    return main


def parse_run_spec(spec: str):
    """'1d:16384:8192:fp16' | '2d:256x256:1024:split' | '3d:128x128x128:64:fp16'
    -> (kind, dims, batch, precision)."""
    kind, dims, batch, prec = spec.split(":")
    return kind, tuple(int(v) for v in dims.split("x")), int(batch), prec


def run_workloads(specs, reps: int, stream) -> dict:
    """Profiling mode: plans (autotuned, or from a loaded cache) of the listed
    workloads, each executed `reps` times back to back after one warm-up,
    with the HIP-event mean per execution.  Inputs are seeded uniform values."""
    import torch
    from paper_2104_11471_amd import inputs, tcfft
    out = {}
    for spec in specs:
        kind, dims, batch, prec = parse_run_spec(spec)
        log(f"run {spec}")
        split = prec == "split"
        shape = (batch,) + dims
        host = (np.stack(inputs.to_split(inputs.uniform_f64(shape, 0))) if split
                else inputs.uniform(shape, 0))
        xd = torch.from_numpy(host).cuda()
        yd = torch.empty_like(xd)
        p = tcfft.Plan(dims, batch, precision=prec, flags=tcfft.FLAG_TUNE)
        torch.cuda.synchronize()
        p(xd, yd, stream=stream)
        dt = time_launches(lambda: p(xd, yd, stream=stream), reps, stream)
        d = p.describe()
        npts = int(np.prod(dims)) * batch
        bpp = 16 if split else 8
        out[spec] = {"us": round(dt * 1e6, 2), "hbm_frac_alg": round(bpp * npts / dt / 1e12 / 8.0, 4),
                     "choice": d["choice"],
                     "passes": [(q["kernel"], q["L"], q["C"], q["NT"], q["grid"]) for q in d["passes"]]}
        log(f"  {out[spec]}")
        del xd, yd, p
        torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=120)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-comparator", action="store_true")
    ap.add_argument("--only", default="", help="comma-separated subset of the sizes (profiling)")
    ap.add_argument("--no-others", action="store_true", help="skip the other workloads")
    ap.add_argument("--serve-seconds", type=float, default=5.0,
                    help="length of the Poisson serving stream (0 = skip)")
    ap.add_argument("--wisdom", default="",
                    help="load this autotuner cache before planning (skips re-tuning: a profiled "
                         "run then uses the plans of an unprofiled one)")
    ap.add_argument("--save-wisdom", default="", help="save the autotuner cache after planning")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run only a 512 MiB device copy (HBM counter calibration)")
    ap.add_argument("--run", default="",
                    help="profiling mode: comma-separated workloads kind:dims:batch:precision "
                         "(e.g. 1d:16384:8192:fp16,2d:256x256:1024:split), each run --reps times")
    ap.add_argument("--reps", type=int, default=5)
    args = ap.parse_args()
    global SIZES
    if args.only:
        SIZES = tuple(int(v) for v in args.only.split(","))
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); batched transforms "
              "shard by transform with no communication, see DESIGN.md", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2104_11471_amd import inputs, tcfft

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    if args.calib_copy:
        a = torch.empty(TOTAL_POINTS, dtype=torch.int32, device=dev).fill_(1)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calib_copy_bytes": 4 * TOTAL_POINTS, "reps": 3}))
        return
    if args.wisdom:
        tcfft.tune_cache_load(args.wisdom)
    if args.run:
        res = run_workloads(args.run.split(","), args.reps, stream)
        if args.save_wisdom:
            tcfft.tune_cache_save(args.save_wisdom)
        print(json.dumps({"run": res}), flush=True)
        return
    plans, xs, xd, yd = {}, {}, {}, {}
    for n in SIZES:
        batch = TOTAL_POINTS // n
        log(f"generating N={n} batch={batch}")
        x, tones = inputs.batched_1d(n, batch, seed=0)
        xs[n] = (x, tones)
        xd[n] = torch.from_numpy(x).to(dev)
        yd[n] = torch.empty_like(xd[n])
        # autotuned plan (tuning happens at plan creation, outside the timing)
        plans[n] = tcfft.Plan((n,), batch, flags=tcfft.FLAG_TUNE)
        d = plans[n].describe()
        log(f"  plan choice={d['choice']} tuned_us={d['tuned_us']:.1f} {d['passes']}")
    torch.cuda.synchronize()
    if args.save_wisdom:
        tcfft.tune_cache_save(args.save_wisdom)

    def step():
        for n in SIZES:
            plans[n](xd[n], yd[n], stream=stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    total_flop = sum(flops(n, TOTAL_POINTS // n) for n in SIZES)
    ms_per_step = elapsed / args.steps * 1e3
    value = total_flop * args.steps / elapsed / 1e9

    # per-size timing (HIP events on the launch stream) and accuracy
    per = {}
    rng = np.random.default_rng(1)
    for n in SIZES:
        batch = TOTAL_POINTS // n
        # 5 trials of >= 100 ms of back-to-back launches each, median (the
        # accuracy check of the previous size leaves the GPU idle for seconds:
        # 20 untimed launches bring the clocks back up first)
        for _ in range(20):
            plans[n](xd[n], yd[n], stream=stream)
        dt = time_trials(lambda: plans[n](xd[n], yd[n], stream=stream), stream)
        emax, erms, eq5, ns = accuracy_sample(plans[n], xd[n], yd[n], xs[n][0], xs[n][1], rng)
        per[n] = {"us": round(dt * 1e6, 2), "gflops": round(flops(n, batch) / dt / 1e9, 1),
                  "gbs_alg": round(8.0 * TOTAL_POINTS / dt / 1e9, 1),
                  "launches": plans[n].num_launches,
                  "rel_l2_max": emax, "rel_l2_rms": erms, "eq5": eq5, "rows_checked": ns}
        log(f"N={n}: {per[n]}")

    # dominant plan: the size whose plan takes the largest share of the step
    # (a multi-pass plan counts as one unit: its algorithmic bytes are one
    # round trip, 8 B per point, whatever its pass count)
    dom = max(SIZES, key=lambda n: per[n]["us"])
    for n in SIZES:
        per[n]["choice"] = plans[n].describe()["choice"]
        per[n]["kernels"] = [kernel_name(q) for q in plans[n].describe()["passes"]]
        per[n]["hbm_frac_alg"] = round(8.0 * TOTAL_POINTS / (per[n]["us"] * 1e-6) / 1e9 /
                                       HBM_PEAK_GBS, 4)
        if plans[n].num_launches > 1:
            per[n]["pass_us"] = pass_times(plans[n], xd[n], yd[n], stream)
    dom_bytes = 8.0 * TOTAL_POINTS
    knames = per[dom]["kernels"]
    achieved = dom_bytes / (per[dom]["us"] * 1e-6) / 1e9
    traffic = [measured_traffic(k) for k in knames]
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": sum(traffic) if all(t is not None for t in traffic) else None,
                "kernel": " + ".join(knames) + f" N={dom} batch={TOTAL_POINTS // dom}",
                "alg_bytes_per_launch": int(dom_bytes), "launches": len(knames)}

    comparator = None
    if not args.no_comparator:
        n = SIZES[0]
        batch = TOTAL_POINTS // n
        p32 = tcfft.Plan((n,), batch, precision="fp32_radix2")
        x32 = torch.from_numpy(xs[n][0].astype(np.float32)).to(dev)
        y32 = torch.empty_like(x32)
        p32(x32, y32, stream=stream)
        dt = time_launches(lambda: p32(x32, y32, stream=stream), 3, stream)
        comparator = {"N": n, "batch": batch, "us": round(dt * 1e6, 1),
                      "gflops": round(flops(n, batch) / dt / 1e9, 1),
                      "fp16_speedup": round((flops(n, batch) / (per[n]["us"] * 1e-6)) /
                                            (flops(n, batch) / dt), 2)}
        log(f"fp32 radix-2 comparator: {comparator}")
        del x32, y32, p32

    others = None
    mixed = None
    if not args.no_others:
        others = other_workloads(stream)
        mixed = mixed_batch_leg(stream)

    serving = None
    if args.serve_seconds > 0:
        serving = serving_leg(args.serve_seconds)
        log(f"serving: {serving}")

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(xs, args.cpu_seconds)
        log(f"cpu baseline: {cpu}")

    hbm_frac = 8.0 * TOTAL_POINTS * len(SIZES) * args.steps / elapsed / 1e9 / HBM_PEAK_GBS
    line = {
        "metric": "batched FP16 FFT GFLOP/s (5NlogN) & % HBM peak; mixed-size p99 latency",
        "value": round(value, 1), "unit": "GFLOP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "fp16", "data": "synthetic",
        "config": {"workload": "batched 1D complex FFT, N in {4096, 16384, 65536}, batch = 2^27/N "
                               "(512 MiB FP16 each), uniform[-1,1] + 1% unit tones, forward",
                   "points_per_size": TOTAL_POINTS, "precision": "fp16 storage, fp32 accumulate"},
        "hbm_frac_alg": round(hbm_frac, 4),
        "roofline_step": {"achieved": round(8.0 * TOTAL_POINTS * len(SIZES) / (ms_per_step * 1e-3) / 1e9, 1),
                          "frac": round(hbm_frac, 4), "unit": "GB/s",
                          "alg_bytes_per_step": int(8 * TOTAL_POINTS * len(SIZES))},
        "per_size": {str(k): v for k, v in per.items()},
        "roofline": roofline,
        "comparator_fp32_radix2": comparator,
        "serving": serving,
        "mixed_batch": mixed,
        "other_workloads": others,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
