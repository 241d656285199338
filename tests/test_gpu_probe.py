"""The peak-rate microbenchmarks (comet_probe_peaks) return rates in the range the
device's published figures allow: FP32 vector FMA up to 157.3 TFLOP/s, FP64 up to 78.6,
dense BF16 matrix-core products up to 2.5 PFLOP/s, HBM copies up to 8 TB/s (each at least
a tenth of its peak, so a probe that measured nothing fails)."""
import pytest

pytestmark = pytest.mark.gpu


def test_probe_rates_are_within_the_published_peaks():
    from paper_2609_21803_amd import native
    p = native.probe_peaks()
    print(p)
    assert 15.7 <= p["fp32_fma_tflops"] <= 157.3 * 1.05
    assert 7.86 <= p["fp64_fma_tflops"] <= 78.6 * 1.05
    assert 250.0 <= p["bf16_mfma_tflops"] <= 2500.0 * 1.05
    assert 800.0 <= p["copy_gbs"] <= 8000.0 * 1.05
