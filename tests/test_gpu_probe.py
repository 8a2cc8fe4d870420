"""Measurement probes: achievable copy bandwidth and arithmetic peaks land in a plausible
range below MI355X's published figures (8 TB/s HBM; 157.3 TFLOP/s FP32 for the matrix cores
and the vector ALUs; 78.6 TFLOP/s FP64 vector; 2.5 PFLOP/s dense BF16 matrix cores)."""
import pytest

from paper_2007_03800_amd import api

pytestmark = pytest.mark.gpu


def test_hbm_copy_rate():
    gbs = api.probe_hbm_copy(1 << 28, reps=3)
    print("copy GB/s", gbs)
    assert 500.0 < gbs < 8000.0


@pytest.mark.parametrize("kind,lo,hi", [("fp32_fma", 10.0, 160.0), ("fp32_mfma_16x16x4", 30.0, 160.0),
                                        ("fp32_mfma_4x4x1", 30.0, 160.0), ("fp64_fma", 5.0, 80.0),
                                        ("bf16_mfma_4x4x4", 50.0, 2600.0), ("bf16_mfma_16x16x16", 100.0, 2600.0),
                                        ("bf16_mfma_16x16x32", 100.0, 2600.0)])
def test_peaks(kind, lo, hi):
    tf = api.probe_peak(kind, reps=3)
    print(kind, "TFLOP/s", tf)
    assert lo < tf < hi
