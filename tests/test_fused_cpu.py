"""Coverage of the fused batch kernels (no device): every pass of the default
plans of the serving population and of the common 1D / 2D sizes is one of
their compiled variants, so tcfft_exec_many runs such batches as fused
launches (one per pass level, precision and LDS class)."""
import pytest

from paper_2104_11471_amd import tcfft


SHAPES = ([((1 << e,), b) for e in range(4, 23) for b in (1, 16, 64)] +
          [((s, s), b) for s in (64, 128, 256, 512, 1024, 2048) for b in (1, 8, 32)])


@pytest.mark.parametrize("prec", ["fp16", "split"])
def test_default_plans_are_fused(prec):
    missing = []
    for dims, batch in SHAPES:
        d = tcfft.dry_run(dims, batch, precision=prec)
        for q in d["passes"]:
            if not q["fused"]:
                missing.append((dims, batch, q["kernel"], q["L"], q["C"], q["NT"]))
    assert not missing, missing


def test_serving_population_is_fused():
    from paper_2104_11471_amd import inputs
    reqs = inputs.serving_stream(rate_hz=20000.0, duration_s=0.05, seed=3)
    assert len(reqs) > 500
    seen = set()
    for r in reqs:
        key = (tuple(r.dims), r.batch, r.split)
        if key in seen:
            continue
        seen.add(key)
        d = tcfft.dry_run(r.dims, r.batch, precision="split" if r.split else "fp16")
        assert all(q["fused"] for q in d["passes"]), (r.dims, r.batch, r.split)


def test_unfused_variants_fall_back():
    """Real plans with the spectrum step in the row pass and the single-pass
    65536 kernel are not fused variants (their batches use per-variant
    launches)."""
    d = tcfft.dry_run((4096,), 8, flags=tcfft.FLAG_REAL)
    assert any(not q["fused"] for q in d["passes"])
