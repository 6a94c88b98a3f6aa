"""The peak probes (libnnp_peaks.so) on the GPU: each launches, the copy is
exact, and the measured rates lie within physical bounds of the part."""
import pytest

pytestmark = pytest.mark.gpu


def test_peak_probes_run_and_are_plausible():
    from paper_2002_00054_amd import peaks

    r = peaks.measure(reps=1, copy_mib=256)
    print(r, flush=True)
    assert r["compute_units"] > 0
    for key in ("fp32_fma_tflops", "fp64_fma_tflops", "fp32_exp_tops"):
        assert 0.5 < r[key] < 200.0, (key, r[key])
    assert 100.0 < r["copy_gbps"] < 10000.0
