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
    # matrix cores: below the datasheet's dense peaks (157.3 / 78.6 / 2500 TFLOP/s)
    # and above a tenth of them
    for key, peak in (("mfma_fp32_tflops", 157.3), ("mfma_fp64_tflops", 78.6), ("mfma_bf16_tflops", 2500.0)):
        assert 0.1 * peak < r[key] < 1.05 * peak, (key, r[key])
