"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (no GPU).

The planner, the autotuner's candidate list and wisdom file, the shard
planner, argument validation of every device entry point and the serving
configuration checks (tcfft.cpp, serve.cpp) are compiled for the host only,
with -fsanitize=address,undefined, linked with the library's other objects,
and driven by tests/host_sanitize_driver.cpp over every supported and many
unsupported shapes.  Any sanitizer report or failed check fails the test."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2104_11471_amd", "csrc")
OBJ = os.path.join(ROOT, "paper_2104_11471_amd", "_build")
ROCM = "/opt/rocm"
CXX = os.path.join(ROCM, "llvm", "bin", "clang++")
DEVICE_UNITS = ["k_row", "k_col_small", "k_col_256", "k_col_large", "k_big", "k_real",
                "k_row_real", "k_plane", "k_misc", "k_static", "k_fused", "k_f64", "registry"]
SAN = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-fno-sanitize-recover=all"]


def test_planner_and_abi_under_host_sanitizers(tmp_path):
    if not os.path.exists(CXX):
        pytest.skip("ROCm clang++ not available")
    if not all(os.path.exists(os.path.join(OBJ, u + ".o")) for u in DEVICE_UNITS):
        from paper_2104_11471_amd import build
        build.build()
    objs = []
    host_flags = ["-x", "c++", "-std=c++17", "-O1", "-g", "-D__HIP_PLATFORM_AMD__",
                  f"-I{ROCM}/include", "-Wno-unused-result", "-Wno-unused-value", *SAN]
    for src in ("tcfft.cpp", "serve.cpp"):
        o = str(tmp_path / (src + ".o"))
        subprocess.run([CXX, *host_flags, "-c", os.path.join(CSRC, src), "-o", o], check=True)
        objs.append(o)
    drv = str(tmp_path / "driver.o")
    subprocess.run([CXX, "-std=c++17", "-O1", "-g", *SAN, "-c",
                    os.path.join(ROOT, "tests", "host_sanitize_driver.cpp"), "-o", drv], check=True)
    exe = str(tmp_path / "driver")
    subprocess.run([CXX, *SAN, "-o", exe, drv, *objs,
                    *[os.path.join(OBJ, u + ".o") for u in DEVICE_UNITS],
                    f"-L{ROCM}/lib", "-lamdhip64", f"-Wl,-rpath,{ROCM}/lib", "-lpthread"],
                   check=True)
    env = dict(os.environ)
    # the HIP runtime keeps allocations until exit: leak checking is left off;
    # a preloaded library may come before the ASan runtime
    env["ASAN_OPTIONS"] = "verify_asan_link_order=0:detect_leaks=0:abort_on_error=0"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    r = subprocess.run([exe, str(tmp_path)], env=env, capture_output=True, text=True, timeout=300)
    print(r.stdout[-2000:], r.stderr[-4000:])
    assert r.returncode == 0, r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
    assert "0 failed checks" in r.stdout
