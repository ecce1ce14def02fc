"""The multiply-rate measurement (hk_mul_rate) behind the roofline's
denominators: every kind returns a positive rate below its nominal
ceiling, and a shader clock within the chip's range."""
import pytest

from tests.gpu_util import log

pytestmark = pytest.mark.gpu

NOMINAL_LANE_OPS = 256 * 64 * 2.4e9          # one operation per lane per clock
NOMINAL_I8_MACS = 256 * 4 * 1024 * 2.4e9     # 1024 int8 multiply-adds per SIMD per clock


@pytest.mark.parametrize("kind,ceiling", [(0, NOMINAL_LANE_OPS), (3, NOMINAL_LANE_OPS), (4, NOMINAL_I8_MACS)])
def test_rate_positive_and_below_nominal(hk, kind, ceiling):
    rate, clk = hk.mul_rate(kind)
    log("rate kind %d: %.4e /s at %.3f GHz" % (kind, rate, clk / 1e9))
    assert 0.05 * ceiling < rate <= 1.02 * ceiling
    assert 0.5e9 < clk < 3.0e9
