"""The measured vector FMA rates (hc_measure_vector_peak) against MI355X's
published vector peaks: FP64 78.6 TFLOP/s, FP32 157.3 TFLOP/s with packed FP32
(two values per lane and instruction), so 78.6 for the plain FP32 FMAs this
library is built with.  A rate above the published peak would mean a wrong
FLOP count; one far below it a broken measurement."""
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_2112_03444_amd as hc
    c = hc.Context(0)
    yield c
    c.close()


def test_measured_vector_peaks(ctx):
    f32 = ctx.measure_vector_peak(False)
    f64 = ctx.measure_vector_peak(True)
    print(f"measured FMA rates: FP32 plain {f32:.1f}, FP64 {f64:.1f} TFLOP/s")
    assert 0.3 * 78.6 < f32 <= 1.1 * 157.3
    assert 0.3 * 78.6 < f64 <= 1.1 * 78.6
