"""Builds libtcfft.so (HIP kernels + C ABI) in-tree for gfx950.

The kernel variants are split over several translation units that compile in
parallel; every unit gets the same flags.  Usage: ``python -m
paper_2104_11471_amd.build`` or :func:`build` (always recompiles)."""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libtcfft.so")
ARCH = "gfx950"
FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
         # packed FP32 instructions are kept out of the generated code
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         # no implicit multiply-add fusion: results depend only on the source,
         # not on how a kernel body was inlined
         "-ffp-contract=off",
         # matrix-core results go straight to VGPRs (no accumulator-register
         # copies: the kernels consume every MFMA result on the vector ALU)
         "-mllvm", "-amdgpu-mfma-vgpr-form",
         "-Wno-unused-command-line-argument"]
UNITS = ["k_row.hip", "k_col_small.hip", "k_col_256.hip", "k_col_large.hip", "k_big.hip", "k_real.hip", "k_row_real.hip", "k_plane.hip", "k_misc.hip", "k_static.hip", "k_fused.hip", "k_f64.hip",
         "registry.cpp", "tcfft.cpp", "serve.cpp"]


def _hipcc() -> str:
    p = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(p):
        raise RuntimeError("hipcc not found: the HIP toolchain is required to build libtcfft")
    return p


def _compile(src: str, obj: str) -> None:
    cmd = [_hipcc(), *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr[-4000:]}")


def build(verbose: bool = False) -> str:
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    objs = [os.path.join(objdir, os.path.splitext(u)[0] + ".o") for u in UNITS]
    jobs = min(len(UNITS), int(os.environ.get("MAX_JOBS", os.cpu_count() or 4)))
    with cf.ThreadPoolExecutor(max_workers=max(1, jobs)) as ex:
        futs = [ex.submit(_compile, u, o) for u, o in zip(UNITS, objs)]
        for f in futs:
            f.result()
    tmp = LIB + ".tmp"
    cmd = [_hipcc(), *FLAGS, "-shared", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr[-4000:]}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
