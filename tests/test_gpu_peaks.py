"""The library's matrix-core and HBM microbenchmarks run and report rates below the
published MI355X peaks (dense fp32 157.3, fp64 78.6 TFLOP/s; 8 TB/s)."""
import pytest

pytestmark = pytest.mark.gpu


def test_measured_peaks_are_plausible():
    import paper_2508_01266_amd as lr
    p = lr.measure_peaks(0)
    print(f"measured: {p}", flush=True)
    assert 0 < p["mfma_f32_tflops"] < 1.1 * 157.3
    assert 0 < p["mfma_f64_tflops"] < 1.1 * 157.3
    assert 0 < p["hbm_copy_gbs"] < 1.1 * 8000
