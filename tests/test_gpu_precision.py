"""The library's precision-failure path forced on the GPU: with too few bits
the Secant iteration of the paper ('The Secant Algorithm') cannot make
progress, and hk_smallest_eig must say so (HK_EPRECISION) rather than return
a value.  Each case is one where the oracle's Secant, with the same stopping
rules, gives up for the same reason."""
import pytest

from oracle.drivers import PrecisionError, secant
from tests.gpu_util import log

pytestmark = pytest.mark.gpu

HK_EPRECISION = 3

# (N, beta, K, the reason both sides give)
CASES = [(32, (1, 1), 128, "ratio"), (40, (1, 2), 128, "ratio"), (32, (1, 1), 320, "shrink")]


@pytest.mark.parametrize("N,beta,K,why", CASES)
def test_secant_reports_exhausted_precision(hk, N, beta, K, why):
    with pytest.raises(PrecisionError, match=why):
        secant(N, beta, K, max_iter=60)
    log("starved Secant N=%d beta=%d/%d K=%d" % (N, beta[0], beta[1], K))
    with pytest.raises(hk.HKError) as e:
        hk.smallest_eig(N, beta, K, method=hk.HK_SECANT, digits=45)
    assert e.value.status == HK_EPRECISION, str(e.value)
    assert why in str(e.value), str(e.value)
    log("  %s" % e.value)
    # with 512 more bits the same call succeeds and verifies
    dec, rep = hk.smallest_eig(N, beta, K + 512, method=hk.HK_SECANT, digits=45)
    assert rep["verified"] == 1, dec
