"""The C-ABI library on a machine without a GPU: it loads, exports every
symbol include/tcfft.h declares, validates arguments, plans without a device
and reports the absence of a device -- no compute calls."""
import ctypes
import json
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tcfft.h")


@pytest.fixture(scope="module")
def tc():
    from paper_2104_11471_amd import tcfft
    return tcfft


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tcfft_[a-z0-9_]+)\s*\(", text)))


def test_header_and_binding_agree(tc):
    assert declared_functions() == sorted(tc.EXPORTS)


def test_every_declared_symbol_is_exported(tc):
    lib = ctypes.CDLL(tc.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_status_strings_and_version(tc):
    for s in range(7):
        assert tc.lib.tcfft_status_string(s)
    assert b"tcfft" in tc.lib.tcfft_version()


@pytest.mark.parametrize("dims,batch,dirn,prec,flags,status", [
    ((12,), 1, -1, 0, 0, 2),          # not a power of two
    ((8,), 1, -1, 0, 0, 2),           # below 16
    ((1 << 28,), 1, -1, 0, 0, 2),     # above 2^27
    ((256,), 0, -1, 0, 0, 1),         # batch <= 0
    ((256,), 1, 0, 0, 0, 1),          # bad direction
    ((256,), 1, -1, 7, 0, 1),         # bad precision
    ((256,), 1, -1, 0, 64, 1),        # unknown flag
    ((4096, 64), 1, -1, 0, 0, 2),     # 2D first dim above 2048
    ((64, 64), 1, -1, 2, 0, 2),       # FP32 comparator is 1D only
    ((1 << 20,), 4096, -1, 0, 0, 2),  # more than 2^31 points per plan
])
def test_dry_run_rejects(tc, dims, batch, dirn, prec, flags, status):
    with pytest.raises(tc.TcfftError) as e:
        tc.dry_run(dims, batch, dirn, prec, flags)
    assert e.value.status == status


def _radices(p):
    r = 1
    for x in p["radices"]:
        r *= x
    return r


@pytest.mark.parametrize("lg", range(4, 28))
def test_plan_factorises_every_1d_size(tc, lg):
    n = 1 << lg
    d = tc.dry_run((n,), 1)
    prod = 1
    for p in d["passes"]:
        assert _radices(p) == p["L"]
        prod *= p["L"]
        assert p["lds"] <= 160 * 1024
        assert set(p["radices"]) <= {2, 4, 8, 16}
        assert p["radices"].count(16) == len(p["radices"]) - (p["radices"][0] != 16)
    assert prod == n
    # static scale: 2 per radix-16 stage, 1 for radix 2/4, 2 for radix 8
    s = sum(2 * p["radices"].count(16) + {1: 0, 2: 1, 4: 1, 8: 2}[
        p["radices"][0] if p["radices"][0] != 16 else 1] for p in d["passes"])
    assert d["scale_log2"] == s
    assert len(d["passes"]) == (1 if n <= 16384 else (2 if n <= (1 << 22) else 3))


def plane_plan(pts, nz, prec):
    """16384 points per workgroup: one plane, or (FP16) 2 or 4 smaller ones."""
    return nz >= 64 and (pts == 16384 or (prec == "fp16" and pts in (4096, 8192)))


@pytest.mark.parametrize("prec", ["fp16", "split"])
@pytest.mark.parametrize("dims", [(16, 16), (256, 256), (512, 512), (1024, 1024), (2048, 64),
                                  (128, 16384), (128, 128), (256, 64), (16, 1024), (512, 32),
                                  (64, 64), (32, 128), (64, 128), (128, 64), (32, 256), (16, 64)])
def test_plan_2d(tc, dims, prec):
    d = tc.dry_run(dims, 2, precision=prec)
    if plane_plan(dims[0] * dims[1], dims[1], prec):  # one workgroup per 16384 points
        assert [p["kernel"] for p in d["passes"]] == ["plane"]
        assert d["passes"][0]["L"] == dims[1] and d["passes"][0]["C"] == dims[0]
    else:
        assert [p["kernel"] for p in d["passes"]] == ["row", "col"]
        assert d["passes"][0]["L"] == dims[1] and d["passes"][1]["L"] == dims[0]
    for p in d["passes"]:
        assert p["lds"] <= 160 * 1024
    assert d["buffer_bytes"] == 2 * dims[0] * dims[1] * (4 if prec == "fp16" else 8)


def test_multi_pass_layout(tc):
    d = tc.dry_run((1 << 20,), 4)
    p1, p2 = d["passes"]
    assert p1["xtw"] == 1 and p1["tstore"] == 1 and p1["dst"] == 2   # to workspace
    assert p2["xtw"] == 0 and p2["src"] == 2 and p2["dst"] == 1
    assert d["workspace_bytes"] == d["buffer_bytes"]
    d3 = tc.dry_run((1 << 24,), 1)
    assert [p["xtw"] for p in d3["passes"]] == [1, 1, 0]
    assert [(p["src"], p["dst"]) for p in d3["passes"]] == [(0, 2), (2, 1), (1, 1)]


def test_no_scale_flag(tc):
    assert tc.dry_run((256,), 1, flags=tc.FLAG_NO_SCALE)["scale_log2"] == 0
    assert tc.dry_run((256,), 1)["scale_log2"] == 4


def test_plan_create_without_device(tc):
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("a GPU is present")
    except ImportError:
        pass
    with pytest.raises(tc.TcfftError) as e:
        tc.Plan((256,), 4)
    assert e.value.status == 3  # TCFFT_ERR_NO_DEVICE


def test_null_arguments(tc):
    lib = tc.lib
    assert lib.tcfft_exec(None, None, None, None) == 1
    assert lib.tcfft_plan_destroy(None) == 0
    assert lib.tcfft_plan_scale_log2(None) == -1
    assert lib.tcfft_plan_buffer_bytes(None) == 0
    assert lib.tcfft_plan_num_launches(None) == -1
    assert lib.tcfft_exec_many(None, None, None, -1, None) == 1
    assert lib.tcfft_exec_many(None, None, None, 0, None) == 0
    assert lib.tcfft_exec_passes(None, None, None, 1, None) == 1
    h = ctypes.c_void_p()
    assert lib.tcfft_plan_create(ctypes.byref(h), 4, (ctypes.c_int64 * 4)(16, 16, 16, 16), 1, -1, 0, 0) == 1
    assert lib.tcfft_plan_create(None, 1, (ctypes.c_int64 * 1)(16), 1, -1, 0, 0) == 1


def test_tune_candidates_are_valid_plans(tc):
    for dims in [(4096,), (16384,), (65536,), (1 << 20,), (1 << 24,), (256, 256), (1024, 1024),
                 (128, 128), (64, 64, 64), (16, 128, 128)]:
        cands = tc.tune_candidates(dims, 8)
        assert len(cands) >= 1
        n = 1
        for v in dims:
            n *= v
        kinds = set()
        for d in cands:
            prod = 1
            for p in d["passes"]:
                # a plane pass covers its nz (L) and ny (C) dimensions
                prod *= p["L"] * (p["C"] if p["kernel"] == "plane" else 1)
                assert p["lds"] <= 160 * 1024
                kinds.add(p["kernel"])
            assert prod == n
        if len(dims) >= 2 and dims[-1] * dims[-2] == 16384:
            assert "plane" in kinds and "row" in kinds  # both plans are timed


def test_tune_cache_file_errors(tc, tmp_path):
    bad = tmp_path / "bad.txt"
    bad.write_text("not a cache\n")
    with pytest.raises(tc.TcfftError):
        tc.tune_cache_load(str(bad))
    with pytest.raises(tc.TcfftError):
        tc.tune_cache_load(str(tmp_path / "missing.txt"))
    tc.tune_cache_clear()
    assert tc.tune_cache_size() == 0
    good = tmp_path / "good.txt"
    good.write_text("tcfft-tune 3\nr1_4096x1_b8_p0 512 64 0 0 0 0 0 0 123.000\n")
    tc.tune_cache_load(str(good))
    assert tc.tune_cache_size() == 1
    tc.tune_cache_save(str(tmp_path / "out.txt"))
    assert "r1_4096x1_b8_p0 512 64" in (tmp_path / "out.txt").read_text()
    tc.tune_cache_clear()


@pytest.mark.parametrize("n", [32, 64, 128, 4096, 32768, 65536, 1 << 24])
def test_real_plan_layout(tc, n):
    """A real plan is the N/2-point complex plan plus one elementwise pass;
    its buffers are M and M+1 words per transform."""
    m, b = n // 2, 3
    c = tc.dry_run((m,), b)
    fused = 64 <= m <= 16384  # single row pass: the real step is its epilogue / prologue
    for dirn, kern, ib, ob, rk in [(tc.FORWARD, "r2c_post", m, m + 1, 1),
                                   (tc.INVERSE, "c2r_pre", m + 1, m, 2)]:
        d = tc.dry_run((n,), b, dirn, flags=tc.FLAG_REAL)
        assert d["real"] == n and d["real_kernel"] == ("fused" if fused else kern)
        assert d["dims"] == [n]
        assert [(p["kernel"], p["L"]) for p in d["passes"]] == [(p["kernel"], p["L"]) for p in c["passes"]]
        assert [p["real"] for p in d["passes"]] == ([rk] if fused else [0] * len(c["passes"]))
        assert d["scale_log2"] == c["scale_log2"]
        assert d["input_bytes"] == b * ib * 4 and d["output_bytes"] == b * ob * 4
        assert d["buffer_bytes"] == b * (m + 1) * 4
        assert d["workspace_bytes"] == c["workspace_bytes"] + (0 if fused else b * m * 4)
    s = tc.dry_run((n,), b, precision="split", flags=tc.FLAG_REAL)
    assert s["input_bytes"] == b * m * 8 and s["output_bytes"] == b * (m + 1) * 8
    assert tc.dry_run((m,), b)["real"] == 0


@pytest.mark.parametrize("dims,prec", [((16,), "fp16"), ((64, 64), "fp16"), ((256,), "fp32")])
def test_real_plan_rejects(tc, dims, prec):
    with pytest.raises(tc.TcfftError) as e:
        tc.dry_run(dims, 1, precision=prec, flags=tc.FLAG_REAL)
    assert e.value.status == 2


@pytest.mark.parametrize("prec", ["fp16", "split"])
@pytest.mark.parametrize("dims", [(16, 16, 16), (64, 64, 64), (128, 32, 256), (2048, 16, 16),
                                  (16, 2048, 16384), (128, 128, 128), (16, 256, 64),
                                  (32, 64, 256), (16, 32, 512), (2048, 16, 1024), (16, 512, 32),
                                  (64, 64, 64), (16, 32, 128), (16, 128, 64), (32, 64, 128),
                                  (16, 32, 256)])
def test_plan_3d(tc, dims, prec):
    """A plane pass (ny nz = 16384, nz >= 64: both in one workgroup) or a row
    pass over nz and a column pass over ny; then a column pass over nx, in
    place in the output."""
    b = 2
    d = tc.dry_run(dims, b, precision=prec)
    assert d["dims"] == list(dims)
    if plane_plan(dims[1] * dims[2], dims[2], prec):
        assert [p["kernel"] for p in d["passes"]] == ["plane", "col"]
        assert [p["L"] for p in d["passes"]] == [dims[2], dims[0]]
        npl = 16384 // (dims[1] * dims[2])  # planes per workgroup
        assert d["passes"][0]["C"] == dims[1] and d["passes"][0]["grid"] == -(-b * dims[0] // npl)
        assert [(p["src"], p["dst"]) for p in d["passes"]] == [(0, 1), (1, 1)]
    else:
        assert [p["kernel"] for p in d["passes"]] == ["row", "col", "col"]
        assert [p["L"] for p in d["passes"]] == [dims[2], dims[1], dims[0]]
        assert [(p["src"], p["dst"]) for p in d["passes"]] == [(0, 1), (1, 1), (1, 1)]
        assert d["passes"][1]["s_in"] == dims[2]
    assert d["passes"][-1]["s_in"] == dims[1] * dims[2]
    for p in d["passes"]:
        assert p["lds"] <= 160 * 1024
    assert d["workspace_bytes"] == 0
    n = dims[0] * dims[1] * dims[2]
    assert d["buffer_bytes"] == b * n * (4 if prec == "fp16" else 8)
    assert d["scale_log2"] == sum(p["scale"] for p in d["passes"])


@pytest.mark.parametrize("dims,status", [((8, 16, 16), 2), ((4096, 16, 16), 2), ((16, 4096, 16), 2),
                                         ((16, 16, 32768), 2), ((16, 16, 24), 2)])
def test_plan_3d_rejects(tc, dims, status):
    with pytest.raises(tc.TcfftError) as e:
        tc.dry_run(dims, 1)
    assert e.value.status == status
    with pytest.raises(tc.TcfftError) as e:
        tc.dry_run((64, 64, 64), 1, precision="fp32")
    assert e.value.status == 2


def test_unknown_flag_bits_are_rejected(tc):
    for bad in (2, 16, 1 << 31):
        with pytest.raises(tc.TcfftError) as e:
            tc.dry_run((256,), 1, flags=bad)
        assert e.value.status == 1  # INVALID_ARG
