"""Serving driver over the library's continuous-batching scheduler.

The scheduler itself (queue, memory admission, slots = HIP streams, grouped
launches, completion polling) is native code in libtcfft (tcfft_server_*);
this module marshals requests, keeps a device-resident payload pool and turns
completion timestamps into latency statistics.
"""
from __future__ import annotations

import ctypes
import time
from collections import defaultdict

import numpy as np

from . import tcfft as _tc

lib = _tc.lib


class ServerConfig(ctypes.Structure):
    _fields_ = [("nslots", ctypes.c_int), ("max_batch_jobs", ctypes.c_int),
                ("mem_budget_bytes", ctypes.c_size_t), ("arena_bytes", ctypes.c_size_t),
                ("use_graphs", ctypes.c_int), ("batch_window_us", ctypes.c_int),
                ("queue_timeout_us", ctypes.c_int)]


class Request(ctypes.Structure):
    _fields_ = [("rank", ctypes.c_int), ("dims", ctypes.c_int64 * 2), ("batch", ctypes.c_int64),
                ("dir", ctypes.c_int), ("precision", ctypes.c_int), ("inp", ctypes.c_void_p),
                ("out", ctypes.c_void_p), ("tag", ctypes.c_uint64)]


class Completion(ctypes.Structure):
    _fields_ = [("tag", ctypes.c_uint64), ("status", ctypes.c_int), ("batch_jobs", ctypes.c_int),
                ("t_submit_ns", ctypes.c_int64), ("t_start_ns", ctypes.c_int64),
                ("t_done_ns", ctypes.c_int64), ("batch_id", ctypes.c_int)]


class ServerStats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in ("submitted", "completed", "rejected", "batches",
                                              "max_batch_jobs", "max_inflight_bytes",
                                              "inflight_bytes", "queued", "plans")]


_P = ctypes.POINTER
lib.tcfft_server_create.argtypes = [_P(ctypes.c_void_p), _P(ServerConfig)]
lib.tcfft_server_prepare.argtypes = [ctypes.c_void_p, _P(Request), ctypes.c_int]
lib.tcfft_server_submit.argtypes = [ctypes.c_void_p, _P(Request)]
lib.tcfft_server_poll.argtypes = [ctypes.c_void_p, _P(Completion), ctypes.c_int]
lib.tcfft_server_wait_idle.argtypes = [ctypes.c_void_p, ctypes.c_int64]
lib.tcfft_server_get_stats.argtypes = [ctypes.c_void_p, _P(ServerStats)]
lib.tcfft_server_destroy.argtypes = [ctypes.c_void_p]
lib.tcfft_server_cancel.argtypes = [ctypes.c_void_p, ctypes.c_uint64]
lib.tcfft_server_cancel.restype = ctypes.c_int
lib.tcfft_server_now_ns.argtypes = []
lib.tcfft_server_now_ns.restype = ctypes.c_int64
for _f in ("tcfft_server_create", "tcfft_server_prepare", "tcfft_server_submit", "tcfft_server_poll",
           "tcfft_server_wait_idle", "tcfft_server_get_stats", "tcfft_server_destroy"):
    getattr(lib, _f).restype = ctypes.c_int


def now_ns() -> int:
    return int(lib.tcfft_server_now_ns())


def _request(rank, dims, batch, direction, precision, in_ptr=0, out_ptr=0, tag=0) -> Request:
    r = Request()
    r.rank = rank
    r.dims[0] = int(dims[0])
    r.dims[1] = int(dims[1]) if rank == 2 else 1
    r.batch = int(batch)
    r.dir = int(direction)
    r.precision = _tc._prec(precision)
    r.inp = in_ptr
    r.out = out_ptr
    r.tag = tag
    return r


class Server:
    def __init__(self, nslots: int = 4, mem_budget_bytes: int = 16 << 30, max_batch_jobs: int = 256,
                 arena_bytes: int = 0, use_graphs: bool = False, batch_window_us: int = 0,
                 queue_timeout_us: int = 0):
        """Defaults favour latency: immediate dispatch with direct grouped
        launches.  At batches of a few jobs, graph replay and a batching window
        add more latency than they save launch work."""
        cfg = ServerConfig(nslots, max_batch_jobs, mem_budget_bytes, arena_bytes, int(use_graphs),
                           int(batch_window_us), int(queue_timeout_us))
        h = ctypes.c_void_p()
        st = lib.tcfft_server_create(ctypes.byref(h), ctypes.byref(cfg))
        if st != 0:
            raise _tc.TcfftError(st, "tcfft_server_create")
        self._h = h
        self._buf = (Completion * 8192)()

    def prepare(self, shapes):
        """shapes: iterable of (rank, dims, direction, precision)."""
        reqs = [_request(rank, dims, 1, d, p) for rank, dims, d, p in shapes]
        arr = (Request * len(reqs))(*reqs)
        st = lib.tcfft_server_prepare(self._h, arr, len(reqs))
        if st != 0:
            raise _tc.TcfftError(st, "tcfft_server_prepare")

    def submit(self, rank, dims, batch, direction, precision, in_ptr, out_ptr, tag) -> int:
        r = _request(rank, dims, batch, direction, precision, in_ptr, out_ptr, tag)
        return int(lib.tcfft_server_submit(self._h, ctypes.byref(r)))

    def cancel(self, tag: int) -> int:
        """Cancels the queued (not yet launched) requests with this tag."""
        n = lib.tcfft_server_cancel(self._h, int(tag))
        if n < 0:
            raise _tc.TcfftError(-n, "tcfft_server_cancel")
        return int(n)

    def poll(self) -> list:
        out = []
        while True:
            n = lib.tcfft_server_poll(self._h, self._buf, len(self._buf))
            if n < 0:
                raise _tc.TcfftError(-n, "tcfft_server_poll")
            for i in range(n):
                c = self._buf[i]
                out.append((int(c.tag), int(c.status), int(c.t_submit_ns), int(c.t_start_ns),
                            int(c.t_done_ns), int(c.batch_id), int(c.batch_jobs)))
            if n < len(self._buf):
                return out

    def wait_idle(self, timeout_ms: int = 60000) -> None:
        st = lib.tcfft_server_wait_idle(self._h, timeout_ms)
        if st != 0:
            raise _tc.TcfftError(st, "tcfft_server_wait_idle")

    def stats(self) -> dict:
        s = ServerStats()
        lib.tcfft_server_get_stats(self._h, ctypes.byref(s))
        return {n: int(getattr(s, n)) for n, _ in ServerStats._fields_}

    def close(self):
        if getattr(self, "_h", None):
            lib.tcfft_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def shape_class(req) -> tuple:
    """(rank, dims, precision) of a generated request (inputs.Request)."""
    return (req.rank, tuple(req.dims), "split" if req.split else "fp16")


class PayloadPool:
    """Device-resident inputs and outputs per shape class, sized for the class's
    largest batch.  `slots` buffers per class; an output buffer is reused only
    after the request that wrote it has completed.  Buffers are flat: a request
    of batch b uses the first b*N points (2*b*N for split: hi plane then lo
    plane) in the ABI layout of batch b (`view`)."""

    def __init__(self, requests, slots: int = 8, seed: int = 0):
        import torch
        from . import inputs
        self.slots = slots
        self.max_batch = defaultdict(int)
        for r in requests:
            k = shape_class(r)
            self.max_batch[k] = max(self.max_batch[k], r.batch)
        self.inp, self.out, self.free = {}, {}, {}
        for i, (k, b) in enumerate(sorted(self.max_batch.items())):
            rank, dims, prec = k
            if prec == "split":
                x = np.stack(inputs.to_split(inputs.uniform_f64((b, *dims), seed + i)))
            else:
                x = inputs.uniform((b, *dims), seed + i)
            t = torch.from_numpy(x).cuda().reshape(-1)
            self.inp[k] = t
            self.out[k] = [torch.empty_like(t) for _ in range(slots)]
            self.free[k] = list(range(slots))
        torch.cuda.synchronize()

    @staticmethod
    def view(flat, k, b):
        """The first request-sized part of a flat class buffer, shaped for batch b."""
        rank, dims, prec = k
        n = int(np.prod(dims))
        if prec == "split":
            return flat[: 2 * b * n * 2].view(2, b, *dims, 2)
        return flat[: b * n * 2].view(b, *dims, 2)

    def nbytes(self) -> int:
        return sum(t.numel() * t.element_size() * (1 + self.slots) for t in self.inp.values())


def run_stream(server: Server, requests, pool: PayloadPool, time_scale: float = 1.0,
               check_tags=()):
    """Submits `requests` at their arrival times (scaled), polls completions
    and returns per-request records.  Latency = completion - scheduled arrival,
    so any wait for a free payload buffer counts against the server."""
    import gc

    import torch
    gc_was_enabled = gc.isenabled()
    gc.disable()  # a collection pause would delay submissions by tens of ms
    recs = {}
    busy = {}                 # tag -> (class, out index)
    keep = {}                 # tag -> output copy for checked tags
    check_tags = set(check_tags)
    t0 = now_ns() + 20_000_000  # start 20 ms from now
    i = 0
    n = len(requests)
    pending = 0

    def drain():
        nonlocal pending
        for tag, st, ts, tb, td, bid, bj in server.poll():
            k, oi = busy.pop(tag)
            if tag in check_tags:
                keep[tag] = pool.out[k][oi].clone()
            pool.free[k].append(oi)
            recs[tag]["status"] = st
            recs[tag]["t_submit"] = ts
            recs[tag]["t_start"] = tb
            recs[tag]["t_done"] = td
            recs[tag]["batch_id"] = bid
            recs[tag]["batch_jobs"] = bj
            pending -= 1

    while i < n:
        r = requests[i]
        t_arr = t0 + int(r.t_arrival * time_scale * 1e9)
        while now_ns() < t_arr:
            drain()
        k = shape_class(r)
        while not pool.free[k]:
            drain()
        oi = pool.free[k].pop()
        xin = pool.inp[k]
        xout = pool.out[k][oi]
        rank, dims, prec = k
        recs[r.rid] = {"arrival": t_arr, "rank": rank, "dims": dims, "batch": r.batch,
                       "prec": prec, "out_index": oi}
        busy[r.rid] = (k, oi)
        st = server.submit(rank, dims, r.batch, -1, prec, xin.data_ptr(), xout.data_ptr(), r.rid)
        if st != 0:
            busy.pop(r.rid)
            pool.free[k].append(oi)
            recs[r.rid]["status"] = st
            recs[r.rid]["t_done"] = None
        else:
            pending += 1
        i += 1
    while pending > 0:
        drain()
    torch.cuda.synchronize()
    if gc_was_enabled:
        gc.enable()
    return recs, keep


def summarize(recs, wall_s: float) -> dict:
    lat = []
    by_class = defaultdict(list)
    pts = 0
    flop = 0.0
    for r in recs.values():
        if r.get("status") != 0 or r.get("t_done") is None:
            continue
        l_us = (r["t_done"] - r["arrival"]) / 1e3
        lat.append(l_us)
        n = int(np.prod(r["dims"]))
        pts += n * r["batch"]
        flop += 5.0 * n * np.log2(n) * r["batch"]
        cls = "2d" if r["rank"] == 2 else ("1d_2^20" if r["dims"][0] >= (1 << 20) else "1d_small")
        by_class[cls].append(l_us)
    lat = np.array(lat)

    def pct(a):
        a = np.asarray(a)
        return {"p50_us": round(float(np.percentile(a, 50)), 1),
                "p99_us": round(float(np.percentile(a, 99)), 1),
                "max_us": round(float(a.max()), 1), "n": int(a.size)} if a.size else {}

    # when did the slow requests arrive (relative to the first arrival)?
    ok = [r for r in recs.values() if r.get("status") == 0 and r.get("t_done") is not None]
    t_first = min(r["arrival"] for r in ok) if ok else 0
    slow = sorted(((r["arrival"] - t_first) / 1e6, (r["t_done"] - r["arrival"]) / 1e3) for r in ok
                  if (r["t_done"] - r["arrival"]) > 5_000_000)
    slow_info = {"n_over_5ms": len(slow),
                 "first_arrival_ms": round(slow[0][0], 2) if slow else None,
                 "last_arrival_ms": round(slow[-1][0], 2) if slow else None}
    # where the time goes (medians): client submit after the scheduled arrival,
    # queueing until the batch launch, and launch-to-completion
    def med(key_a, key_b):
        v = [(r[key_b] - r[key_a]) / 1e3 for r in ok if r.get(key_a) is not None]
        return round(float(np.median(v)), 1) if v else None
    parts = {"submit_after_arrival_us": med("arrival", "t_submit"),
             "queued_us": med("t_submit", "t_start"), "launch_to_done_us": med("t_start", "t_done")}
    return {"requests": int(lat.size), "failed": int(len(recs) - lat.size), "slow": slow_info,
            "median_parts": parts,
            "req_per_s": round(lat.size / wall_s, 1), "points_per_s": round(pts / wall_s, 1),
            "gflops": round(flop / wall_s / 1e9, 1), **pct(lat),
            "by_class": {k: pct(v) for k, v in sorted(by_class.items())}}
