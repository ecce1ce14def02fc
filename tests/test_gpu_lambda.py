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


@pytest.mark.parametrize("method", ["secant", "inverse"])
def test_lambda_binary_value(hk, method):
    # lambda_1 is reported as a decimal string and as an hk_mpf; at K = 512
    # the binary value is the whole fixed-point result (at most 512 bits),
    # within 1e-40 of the oracle and consistent with the decimal string
    N, beta, K = 32, (1, 1), 512
    m = hk.HK_SECANT if method == "secant" else hk.HK_INVERSE
    dec, rep = hk.smallest_eig(N, beta, K, method=m, digits=45)
    lam = rep["lambda"]
    assert rep["verified"] == 1 and lam > 0
    assert (lam * (1 << K)).denominator == 1          # exactly K fractional bits or fewer
    assert rel_digits(lam, parse_dec(dec)) > 43.5   # the string is truncated to 45 digits
    lam_o, _ = inverse_iteration(N, beta, K)
    assert rel_digits(lam, lam_o) > 40


def test_lambda_binary_value_batched(hk):
    insts = [(24, (7, 4), 640), (40, (1, 2), 768)]
    res, rep = hk.eig_batched(insts, digits=45, panel=2)
    for (N, beta, K), (st, dec, ver, nf), lam in zip(insts, res, rep["lambda"]):
        assert st == 0 and ver == 1
        assert rel_digits(lam, parse_dec(dec)) > 43.5   # the string is truncated to 45 digits
        lam_o, _ = inverse_iteration(N, beta, K)
        assert rel_digits(lam, lam_o) > 40
