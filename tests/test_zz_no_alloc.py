"""The allocation-free entry point hk_smallest_eig_static (workspace in the
library's fixed device array) gives what hk_smallest_eig gives with a caller
buffer: two calls in a row, the second on a smaller instance (the array
keeps the first call's contents), every report field that does not time
anything equal, and lambda_1 within 1e-40 of the oracle."""
import pytest

from oracle.drivers import inverse_iteration, rel_digits
from tests.gpu_util import log

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("method", ["secant", "inverse"])
def test_static_equals_caller_buffer(hk, method):
    m = hk.HK_SECANT if method == "secant" else hk.HK_INVERSE
    for N, beta, K in [(100, (7, 4), 1536), (32, (1, 1), 512)]:
        log("static workspace %s N=%d beta=%s K=%d" % (method, N, beta, K))
        d1, r1 = hk.smallest_eig_static(N, beta, K, method=m, digits=45)
        d2, r2 = hk.smallest_eig(N, beta, K, method=m, digits=45)
        assert d1 == d2 and r1["verified"] == r2["verified"] == 1
        for k in ("status", "bits_used", "factorizations", "solves", "digits_verified", "limb_macs", "lambda_dec",
                  "lambda"):
            assert r1[k] == r2[k], k
        lam_o, _ = inverse_iteration(N, beta, K)
        assert rel_digits(r1["lambda"], lam_o) > 40


def test_static_rejects_oversize(hk):
    # N = 500, K = 6144 needs far more than the fixed array: a clear error,
    # found on the host before any device work
    assert hk.lib().hk_static_workspace_limit() == 64 << 20
    with pytest.raises(hk.HKError) as ei:
        hk.smallest_eig_static(500, (1, 1), 6144, method=hk.HK_SECANT)
    assert ei.value.status == 1 and "workspace" in str(ei.value)
