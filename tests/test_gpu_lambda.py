"""GPU end-to-end: lambda_1 from the library's Secant driver agrees with the
oracle to 1e-40 relative and passes the inertia bracket."""
from fractions import Fraction

import pytest

from oracle.drivers import inverse_iteration, rel_digits, secant
from tests.gpu_util import log

pytestmark = pytest.mark.gpu


def parse_dec(s):
    m, e = s.split("e")
    return Fraction(m) * Fraction(10) ** int(e)


@pytest.mark.parametrize("N,beta,K", [(32, (1, 1), 512), (60, (7, 4), 1280)])
def test_secant_lambda(hk, N, beta, K):
    log("secant N=%d beta=%s K=%d" % (N, beta, K))
    dec, rep = hk.smallest_eig(N, beta, K, method=hk.HK_SECANT, digits=45)
    assert rep["verified"] == 1
    lam_o, _ = inverse_iteration(N, beta, K)
    assert rel_digits(parse_dec(dec), lam_o) > 40
