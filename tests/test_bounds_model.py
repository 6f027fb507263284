"""Host model of every pass's HBM address range (no GPU).

From the plan description (tcfft_plan_dry_run / tcfft_shard_dry_run), the
index arithmetic of the row and column kernels is evaluated for every
workgroup, and the lowest and highest element each pass reads and writes --
including the lo plane of split data, npts * batch words above the hi plane --
must lie inside the buffer that pass reads or writes (user input, user output
or workspace).  This checks the planner's geometry against the buffers the
caller and the plan provide before anything runs on a device."""
import numpy as np
import pytest


@pytest.fixture(scope="module")
def tc():
    from paper_2104_11471_amd import tcfft
    return tcfft


def _ilog2(v):
    return int(v).bit_length() - 1


def pass_ranges(p):
    """(min, max) element index read and written by one pass, in one plane."""
    L, grid = p["L"], p["grid"]
    if p["kernel"] == "col":
        C, blocks = p["C"], p["blocks"]
        wg = np.arange(grid, dtype=np.int64)
        outer = wg >> _ilog2(blocks)
        i0 = (wg & (blocks - 1)) * C
        in_base = outer * p["in_outer"] + i0
        rd = (int(in_base.min()), int((in_base + (L - 1) * p["s_in"] + C - 1).max()))
        if p["tstore"]:
            tb = p["tblk"]
            tbl = _ilog2(tb)
            base = outer * p["out_outer"] + (i0 << tbl)
            top = base + ((L - 1) >> tbl) * p["tblk_stride"] + ((C - 1) << tbl) + ((L - 1) & (tb - 1))
        else:
            q = p["q"]
            base = outer * p["out_outer"] + (i0 >> _ilog2(q)) * p["qstride"] + (i0 & (q - 1))
            top = base + (L - 1) * p["s_out"] + C - 1
        return rd, (int(base.min()), int(top.max()))
    if p["kernel"] in ("row", "plane"):
        lines = p["lines"]
        span = lines * (L if p["kernel"] == "row" else L)
        if p["kernel"] == "row" and p["tstore"]:
            q = p["q"]
            assert lines % q == 0
            last = lines - 1
            top = (last >> _ilog2(q)) * q * L + (q - 1) + (L - 1) * q
            return (0, span - 1), (0, int(top))
        return (0, span - 1), (0, span - 1)
    raise AssertionError(p["kernel"])


def check_plan(d, batch):
    split = d["precision"] == "split_fp16"
    elt = 8 if split else 4
    plane = d["points"] * batch
    sizes = {0: d["input_bytes"] // elt, 1: d["output_bytes"] // elt,
             2: d["workspace_bytes"] // elt}
    # every buffer holds exactly one plane of npts * batch points per half
    assert sizes[0] == plane and sizes[1] == plane
    for i, p in enumerate(d["passes"]):
        (r0, r1), (w0, w1) = pass_ranges(p)
        for (lo, hi), buf in (((r0, r1), p["src"]), ((w0, w1), p["dst"])):
            assert lo >= 0 and hi < sizes[buf], (i, p, lo, hi, sizes[buf])
            if split:  # the lo plane: plane words above the hi plane, same buffer
                assert hi + plane < 2 * sizes[buf], (i, p)


@pytest.mark.parametrize("prec", ["fp16", "split"])
@pytest.mark.parametrize("lg", list(range(4, 28)))
def test_1d_passes_stay_in_their_buffers(tc, lg, prec):
    for batch in (1, 3):
        if (1 << lg) * batch > (1 << 31):
            continue
        check_plan(tc.dry_run((1 << lg,), batch, precision=prec), batch)


@pytest.mark.parametrize("prec", ["fp16", "split"])
@pytest.mark.parametrize("dims", [(16, 16), (64, 512), (256, 256), (1024, 1024), (2048, 16384),
                                  (128, 128), (16, 2048, 32), (128, 128, 128), (512, 512, 512)])
def test_2d_3d_passes_stay_in_their_buffers(tc, dims, prec):
    check_plan(tc.dry_run(dims, 2, precision=prec), 2)


@pytest.mark.parametrize("prec", ["fp16", "split"])
@pytest.mark.parametrize("lg,g", [(15, 2), (16, 16), (20, 4), (20, 8), (22, 8), (23, 8),
                                  (24, 8), (26, 4), (27, 16)])
def test_shard_passes_stay_in_their_buffers(tc, lg, g, prec):
    for shard in (0, g - 1):
        d = tc.shard_dry_run(1 << lg, 3, g, shard, precision=prec)
        assert d["points"] == (1 << lg) // g
        check_plan(d, 3)


def test_model_catches_a_plane_offset_past_the_buffer(tc):
    """A shard plan described with the full length as its point count (the
    lo plane then starts past the shard's buffer) fails the check."""
    d = tc.shard_dry_run(1 << 20, 2, 4, 1, precision="split")
    d["points"] = 1 << 20
    with pytest.raises(AssertionError):
        check_plan(d, 2)
