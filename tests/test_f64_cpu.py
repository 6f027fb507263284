"""FP64 matrix-core plans on the host (no device): planner output, buffer
sizes and the supported range."""
import pytest

from paper_2104_11471_amd import tcfft


@pytest.mark.parametrize("n", [16, 32, 64, 128, 256, 512, 1024, 2048, 4096])
def test_fp64_plan(n):
    d = tcfft.dry_run((n,), 5, precision="fp64")
    assert d["precision"] == "fp64"
    assert d["scale_log2"] == 0
    assert d["input_bytes"] == d["output_bytes"] == 16 * n * 5
    assert d["workspace_bytes"] == 0
    (q,) = d["passes"]
    assert q["kernel"] == "f64_row" and q["L"] == n
    r0 = 1 << ((n.bit_length() - 1) % 4)
    assert q["R0"] == r0 and r0 * 16 ** q["stages16"] == n


@pytest.mark.parametrize("dims,flags", [((8192,), 0), ((1 << 20,), 0), ((64, 64), 0),
                                        ((4096,), 8)])
def test_fp64_unsupported(dims, flags):
    with pytest.raises(tcfft.TcfftError) as e:
        tcfft.dry_run(dims, 1, precision="fp64", flags=flags)
    assert e.value.status == 2  # UNSUPPORTED


def test_fp64_has_no_tuner_candidates():
    assert tcfft.tune_candidates((1024,), 64, precision="fp64") == []
