"""Thin ctypes binding of libtcfft.so (argument marshalling only).

Every step of a transform runs in the library's HIP kernels; torch provides
device memory and the current stream, nothing else.  Importing this module
loads the library and raises ``RuntimeError`` when it is missing: there is no
fallback of any kind.
"""
from __future__ import annotations

import ctypes
import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtcfft.so")

FORWARD = -1
INVERSE = 1
PREC_FP16 = 0
PREC_SPLIT_FP16 = 1
PREC_FP32_RADIX2 = 2
PREC_FP64 = 3
FLAG_NO_SCALE = 1
FLAG_TUNE = 4
FLAG_REAL = 8
_PREC = {"fp16": PREC_FP16, "split": PREC_SPLIT_FP16, "split_fp16": PREC_SPLIT_FP16,
         "fp32_radix2": PREC_FP32_RADIX2, "fp32": PREC_FP32_RADIX2, "fp64": PREC_FP64}

STATUS = {0: "ok", 1: "invalid argument", 2: "unsupported", 3: "no device", 4: "alloc",
          5: "launch", 6: "internal", 7: "timeout", 8: "cancelled"}

# every symbol include/tcfft.h declares
EXPORTS = ["tcfft_plan_create", "tcfft_plan_1d", "tcfft_plan_2d", "tcfft_exec", "tcfft_exec_many",
           "tcfft_exec_passes", "tcfft_plan_destroy", "tcfft_plan_scale_log2",
           "tcfft_plan_buffer_bytes", "tcfft_plan_input_bytes", "tcfft_plan_output_bytes",
           "tcfft_plan_workspace_bytes", "tcfft_plan_num_launches", "tcfft_plan_describe",
           "tcfft_plan_dry_run", "tcfft_status_string", "tcfft_version", "tcfft_tune_candidates",
           "tcfft_tune_cache_size", "tcfft_tune_cache_save", "tcfft_tune_cache_load",
           "tcfft_tune_cache_clear", "tcfft_server_create", "tcfft_server_prepare",
           "tcfft_server_submit", "tcfft_server_poll", "tcfft_server_wait_idle",
           "tcfft_server_get_stats", "tcfft_server_destroy", "tcfft_server_now_ns",
           "tcfft_plan_create_shard", "tcfft_exec_shard", "tcfft_shard_dry_run",
           "tcfft_exec_many_static", "tcfft_server_cancel", "tcfft_fused_wait_failures"]


class TcfftError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: {STATUS.get(status, status)} (status {status})")
        self.status = status


def _load() -> ctypes.CDLL:
    # One HIP runtime per process: torch ships its own libamdhip64, and the
    # streams and device pointers the binding passes come from it, so torch
    # (when installed) is loaded first and libtcfft binds to that runtime.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m "
                           "paper_2104_11471_amd.build` (there is no fallback path)")
    lib = ctypes.CDLL(LIB_PATH)
    i64 = ctypes.c_int64
    vp = ctypes.c_void_p
    P = ctypes.POINTER
    lib.tcfft_plan_create.argtypes = [P(vp), ctypes.c_int, P(i64), i64, ctypes.c_int, ctypes.c_int,
                                      ctypes.c_uint]
    lib.tcfft_plan_1d.argtypes = [P(vp), i64, i64]
    lib.tcfft_plan_2d.argtypes = [P(vp), i64, i64, i64]
    lib.tcfft_exec.argtypes = [vp, vp, vp, vp]
    lib.tcfft_exec_many.argtypes = [P(vp), P(vp), P(vp), ctypes.c_int, vp]
    lib.tcfft_exec_many_static.argtypes = [P(vp), P(vp), P(vp), ctypes.c_int, vp]
    lib.tcfft_exec_many_static.restype = ctypes.c_int
    lib.tcfft_fused_wait_failures.argtypes = [P(ctypes.c_uint)]
    lib.tcfft_fused_wait_failures.restype = ctypes.c_int
    lib.tcfft_exec_passes.argtypes = [vp, vp, vp, ctypes.c_int, vp]
    lib.tcfft_plan_destroy.argtypes = [vp]
    lib.tcfft_plan_scale_log2.argtypes = [vp]
    lib.tcfft_plan_buffer_bytes.argtypes = [vp]
    lib.tcfft_plan_buffer_bytes.restype = ctypes.c_size_t
    lib.tcfft_plan_input_bytes.argtypes = [vp]
    lib.tcfft_plan_input_bytes.restype = ctypes.c_size_t
    lib.tcfft_plan_output_bytes.argtypes = [vp]
    lib.tcfft_plan_output_bytes.restype = ctypes.c_size_t
    lib.tcfft_plan_workspace_bytes.argtypes = [vp]
    lib.tcfft_plan_workspace_bytes.restype = ctypes.c_size_t
    lib.tcfft_plan_num_launches.argtypes = [vp]
    lib.tcfft_plan_describe.argtypes = [vp, ctypes.c_char_p, ctypes.c_size_t]
    lib.tcfft_plan_dry_run.argtypes = [ctypes.c_int, P(i64), i64, ctypes.c_int, ctypes.c_int,
                                       ctypes.c_uint, ctypes.c_char_p, ctypes.c_size_t]
    lib.tcfft_status_string.argtypes = [ctypes.c_int]
    lib.tcfft_status_string.restype = ctypes.c_char_p
    lib.tcfft_version.argtypes = []
    lib.tcfft_version.restype = ctypes.c_char_p
    lib.tcfft_tune_candidates.argtypes = [ctypes.c_int, P(i64), i64, ctypes.c_int, ctypes.c_char_p,
                                          ctypes.c_size_t]
    lib.tcfft_tune_candidates.restype = ctypes.c_int
    lib.tcfft_tune_cache_size.argtypes = []
    lib.tcfft_tune_cache_size.restype = ctypes.c_int
    lib.tcfft_tune_cache_save.argtypes = [ctypes.c_char_p]
    lib.tcfft_tune_cache_save.restype = ctypes.c_int
    lib.tcfft_tune_cache_load.argtypes = [ctypes.c_char_p]
    lib.tcfft_tune_cache_load.restype = ctypes.c_int
    lib.tcfft_tune_cache_clear.argtypes = []
    lib.tcfft_tune_cache_clear.restype = None
    lib.tcfft_plan_create_shard.argtypes = [P(vp), i64, i64, ctypes.c_int, ctypes.c_int,
                                            ctypes.c_int, ctypes.c_int, ctypes.c_uint]
    lib.tcfft_plan_create_shard.restype = ctypes.c_int
    lib.tcfft_exec_shard.argtypes = [vp, ctypes.c_int, vp, vp, vp]
    lib.tcfft_exec_shard.restype = ctypes.c_int
    lib.tcfft_shard_dry_run.argtypes = [i64, i64, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                        ctypes.c_int, ctypes.c_uint, ctypes.c_char_p,
                                        ctypes.c_size_t]
    lib.tcfft_shard_dry_run.restype = ctypes.c_int
    for name in ("tcfft_plan_create", "tcfft_plan_1d", "tcfft_plan_2d", "tcfft_exec",
                 "tcfft_exec_many", "tcfft_exec_passes", "tcfft_plan_destroy",
                 "tcfft_plan_scale_log2", "tcfft_plan_num_launches", "tcfft_plan_describe",
                 "tcfft_plan_dry_run"):
        getattr(lib, name).restype = ctypes.c_int
    return lib


lib = _load()


def _prec(p) -> int:
    return _PREC[p] if isinstance(p, str) else int(p)


def dry_run(dims, batch: int, direction: int = FORWARD, precision="fp16", flags: int = 0) -> dict:
    """Planner only (no device): the JSON plan the arguments would produce."""
    dims = tuple(int(d) for d in dims)
    arr = (ctypes.c_int64 * len(dims))(*dims)
    buf = ctypes.create_string_buffer(8192)
    n = lib.tcfft_plan_dry_run(len(dims), arr, int(batch), int(direction), _prec(precision),
                               int(flags), buf, len(buf))
    if n < 0:
        raise TcfftError(-n, "tcfft_plan_dry_run")
    return json.loads(buf.value.decode())


def tune_candidates(dims, batch: int, precision="fp16") -> list:
    """The planner candidates the autotuner times (no device)."""
    dims = tuple(int(d) for d in dims)
    arr = (ctypes.c_int64 * len(dims))(*dims)
    buf = ctypes.create_string_buffer(1 << 20)
    n = lib.tcfft_tune_candidates(len(dims), arr, int(batch), _prec(precision), buf, len(buf))
    if n < 0:
        raise TcfftError(-n, "tcfft_tune_candidates")
    return json.loads(buf.value.decode())


def tune_cache_save(path: str) -> None:
    st = lib.tcfft_tune_cache_save(path.encode())
    if st != 0:
        raise TcfftError(st, "tcfft_tune_cache_save")


def tune_cache_load(path: str) -> None:
    st = lib.tcfft_tune_cache_load(path.encode())
    if st != 0:
        raise TcfftError(st, "tcfft_tune_cache_load")


def tune_cache_size() -> int:
    return int(lib.tcfft_tune_cache_size())


def tune_cache_clear() -> None:
    lib.tcfft_tune_cache_clear()


class Plan:
    """A tcFFT plan: ``Plan((n,), batch)`` or ``Plan((nx, ny), batch)``.

    Tensors (torch, on the plan's device):
      * fp16: ``float16`` of shape ``(batch, *dims, 2)`` (interleaved re, im);
      * split: ``float16`` of shape ``(2, batch, *dims, 2)`` -- hi plane then lo
        plane, value = hi + 2^-11 lo;
      * fp32_radix2: ``float32`` of shape ``(batch, n, 2)``;
      * fp64: ``float64`` of shape ``(batch, n, 2)`` (FP64 matrix-core path).
    The output holds DFT(x) * 2^-scale_log2 in the same layout.

    Real plans (``flags`` with FLAG_REAL, 1D, N = 2M): the real side is
    ``float16`` of shape ``(batch, N)`` (split: ``(2, batch, N)``), the
    spectrum side ``(batch, M + 1, 2)`` (split: ``(2, batch, M + 1, 2)``) with
    bins 0..M.  FORWARD maps real -> spectrum, INVERSE spectrum -> real (N x
    the sequence, times 2^-scale_log2)."""

    def __init__(self, dims, batch: int, direction: int = FORWARD, precision="fp16",
                 flags: int = 0):
        self.dims = tuple(int(d) for d in dims)
        self.batch = int(batch)
        self.direction = int(direction)
        self.precision = _prec(precision)
        self.flags = int(flags)
        arr = (ctypes.c_int64 * len(self.dims))(*self.dims)
        h = ctypes.c_void_p()
        st = lib.tcfft_plan_create(ctypes.byref(h), len(self.dims), arr, self.batch,
                                   self.direction, self.precision, self.flags)
        if st != 0:
            raise TcfftError(st, "tcfft_plan_create")
        self._h = h

    @property
    def handle(self):
        return self._h

    @property
    def scale_log2(self) -> int:
        return int(lib.tcfft_plan_scale_log2(self._h))

    @property
    def buffer_bytes(self) -> int:
        return int(lib.tcfft_plan_buffer_bytes(self._h))

    @property
    def workspace_bytes(self) -> int:
        return int(lib.tcfft_plan_workspace_bytes(self._h))

    @property
    def num_launches(self) -> int:
        return int(lib.tcfft_plan_num_launches(self._h))

    def describe(self) -> dict:
        buf = ctypes.create_string_buffer(8192)
        lib.tcfft_plan_describe(self._h, buf, len(buf))
        return json.loads(buf.value.decode())

    @property
    def input_bytes(self) -> int:
        return int(lib.tcfft_plan_input_bytes(self._h))

    @property
    def output_bytes(self) -> int:
        return int(lib.tcfft_plan_output_bytes(self._h))

    @property
    def real(self) -> bool:
        return bool(self.flags & FLAG_REAL)

    def _side(self, real_side: bool) -> tuple:
        if real_side:
            core = (self.batch, self.dims[0])
        elif self.real:
            core = (self.batch, self.dims[0] // 2 + 1, 2)
        else:
            core = (self.batch, *self.dims, 2)
        return (2, *core) if self.precision == PREC_SPLIT_FP16 else core

    def in_shape(self) -> tuple:
        return self._side(self.real and self.direction == FORWARD)

    def out_shape(self) -> tuple:
        return self._side(self.real and self.direction == INVERSE)

    def shape(self) -> tuple:
        """The input shape (equal to the output shape for complex plans)."""
        return self.in_shape()

    def dtype(self):
        import torch
        if self.precision == PREC_FP64:
            return torch.float64
        return torch.float32 if self.precision == PREC_FP32_RADIX2 else torch.float16

    def empty(self, device=None):
        import torch
        return torch.empty(self.in_shape(), dtype=self.dtype(), device=device or "cuda")

    def empty_out(self, device=None):
        import torch
        return torch.empty(self.out_shape(), dtype=self.dtype(), device=device or "cuda")

    def _check(self, t, name):
        import torch
        if not isinstance(t, torch.Tensor) or not t.is_cuda:
            raise ValueError(f"{name} must be a CUDA (HIP) tensor")
        if t.dtype != self.dtype() or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous {self.dtype()} tensor")
        need = self.input_bytes if name == "input" else self.output_bytes
        if t.numel() * t.element_size() != need:
            raise ValueError(f"{name} holds {t.numel() * t.element_size()} bytes, "
                             f"the plan needs {need}")

    def exec_raw(self, in_ptr: int, out_ptr: int, stream_ptr: int) -> None:
        st = lib.tcfft_exec(self._h, ctypes.c_void_p(in_ptr), ctypes.c_void_p(out_ptr),
                            ctypes.c_void_p(stream_ptr))
        if st != 0:
            raise TcfftError(st, "tcfft_exec")

    def __call__(self, x, out=None, stream=None):
        import torch
        self._check(x, "input")
        if out is None:
            out = torch.empty(self.out_shape(), dtype=x.dtype, device=x.device)
        self._check(out, "output")
        s = stream if stream is not None else torch.cuda.current_stream(x.device)
        self.exec_raw(x.data_ptr(), out.data_ptr(), s.cuda_stream)
        return out

    def run_passes(self, x, npasses: int, out=None, stream=None):
        """The first `npasses` passes only (the intermediate of Eq. 3)."""
        import torch
        self._check(x, "input")
        if out is None:
            out = torch.empty_like(x)
        self._check(out, "output")
        s = stream if stream is not None else torch.cuda.current_stream(x.device)
        st = lib.tcfft_exec_passes(self._h, ctypes.c_void_p(x.data_ptr()),
                                   ctypes.c_void_p(out.data_ptr()), int(npasses),
                                   ctypes.c_void_p(s.cuda_stream))
        if st != 0:
            raise TcfftError(st, "tcfft_exec_passes")
        return out

    def close(self):
        if getattr(self, "_h", None):
            lib.tcfft_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


STATIC_MAX_JOBS = 1024


def exec_many(plans, xs, outs, stream=None, static: bool = False) -> None:
    """Runs plans[j] on (xs[j], outs[j]) for all j in one call
    (tcfft_exec_many, or tcfft_exec_many_static with ``static``)."""
    import torch
    n = len(plans)
    VP = ctypes.c_void_p
    hp = (VP * n)(*[p.handle for p in plans])
    ip = (VP * n)(*[x.data_ptr() for x in xs])
    op = (VP * n)(*[o.data_ptr() for o in outs])
    for p, x, o in zip(plans, xs, outs):
        p._check(x, "input")
        p._check(o, "output")
    s = stream if stream is not None else torch.cuda.current_stream()
    fn = lib.tcfft_exec_many_static if static else lib.tcfft_exec_many
    st = fn(hp, ip, op, n, VP(s.cuda_stream))
    if st != 0:
        raise TcfftError(st, "tcfft_exec_many_static" if static else "tcfft_exec_many")


def fused_wait_failures() -> int:
    """Dependency waits of single-launch batches that ran out (current device)."""
    v = ctypes.c_uint(0)
    st = lib.tcfft_fused_wait_failures(ctypes.byref(v))
    if st != 0:
        raise TcfftError(st, "tcfft_fused_wait_failures")
    return v.value


def shard_dry_run(n: int, batch: int, nshards: int, shard: int, direction: int = FORWARD,
                  precision="fp16", flags: int = 0) -> dict:
    """Planner only (no device): the JSON plan of one shard."""
    buf = ctypes.create_string_buffer(8192)
    r = lib.tcfft_shard_dry_run(int(n), int(batch), int(direction), _prec(precision),
                                int(nshards), int(shard), int(flags), buf, len(buf))
    if r < 0:
        raise TcfftError(-r, "tcfft_shard_dry_run")
    return json.loads(buf.value.decode())


class ShardPlan(Plan):
    """One device's share of a distributed N-point transform over `nshards`
    devices (tcfft_plan_create_shard): ``step1`` before the caller's
    all-to-all, ``step2`` after it.  Tensors hold ``batch * N / nshards``
    points: ``(batch, N // nshards, 2)`` float16 (split: ``(2, ...)``)."""

    def __init__(self, n: int, batch: int, nshards: int, shard: int, direction: int = FORWARD,
                 precision="fp16", flags: int = 0):
        self.dims = (int(n),)
        self.batch = int(batch)
        self.direction = int(direction)
        self.precision = _prec(precision)
        self.flags = int(flags)
        self.nshards = int(nshards)
        self.shard = int(shard)
        h = ctypes.c_void_p()
        st = lib.tcfft_plan_create_shard(ctypes.byref(h), int(n), self.batch, self.direction,
                                         self.precision, self.nshards, self.shard, self.flags)
        if st != 0:
            raise TcfftError(st, "tcfft_plan_create_shard")
        self._h = h

    def _side(self, real_side: bool) -> tuple:
        core = (self.batch, self.dims[0] // self.nshards, 2)
        return (2, *core) if self.precision == PREC_SPLIT_FP16 else core

    def _step(self, step: int, x, out, stream):
        import torch
        self._check(x, "input")
        if out is None:
            out = torch.empty_like(x)
        self._check(out, "output")
        s = stream if stream is not None else torch.cuda.current_stream(x.device)
        st = lib.tcfft_exec_shard(self._h, int(step), ctypes.c_void_p(x.data_ptr()),
                                  ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(s.cuda_stream))
        if st != 0:
            raise TcfftError(st, "tcfft_exec_shard")
        return out

    def step1(self, x, out=None, stream=None):
        return self._step(1, x, out, stream)

    def step2(self, x, out=None, stream=None):
        return self._step(2, x, out, stream)

    def __call__(self, x, out=None, stream=None):
        raise TcfftError(2, "a shard plan runs step1 and step2 around an exchange")
