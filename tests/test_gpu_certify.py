"""GPU parity of the rigorous inertia (hk_certify; the paper's 'Interval
Verification' in midpoint-radius form): on the same factorisation the
library's radius recursion (host, (double, exponent) numbers rounded up,
entry magnitudes bounded on the GPU) and the oracle's (integers in units of
2^-(K+32), rounded up) give the same per-pivot margins log2(|d_k| /
radius_k) to 1e-6 bits and the same verdict; hk_smallest_eig with
HK_FLAG_CERTIFY proves the 45-digit bracket once K is raised to the
precision it reports."""
import math

import pytest

import oracle
from oracle.certify import radii
from oracle.moments import moments
from tests.gpu_util import log

pytestmark = pytest.mark.gpu


def oracle_margins(N, K, X, xf):
    h = K // 2
    piv, eD, G = radii(N, K, X, xf)
    out = []
    for d, e in zip(piv, eD):
        if e is None:
            break
        out.append(math.log2(abs(d)) + (G - h) - math.log2(e) if d else -math.inf)
    return out


@pytest.mark.parametrize("N,beta,K,xn", [(32, (1, 1), 512, 0), (32, (1, 1), 1024, 0), (24, (7, 4), 768, -5),
                                         (40, (3, 2), 1024, 3), (20, (1, 2), 640, 0)])
def test_certify_margins_match_oracle(hk, N, beta, K, xn):
    xf = xn << (K // 2)
    X = moments(N, beta, K)
    om = oracle_margins(N, K, X, xf)
    log("certify N=%d beta=%s K=%d: oracle least margin %.2f bits" % (N, beta, K, min(om)))
    m = hk.Matrix(N, beta, K)
    m.factor(xf)
    nn, ok, mm, margins = m.certify()
    assert nn == 0
    assert ok == (len(om) == N and min(om) > 0)
    for k, v in enumerate(om):
        assert abs(margins[k] - v) < 1e-6, (k, margins[k], v)
    assert abs(mm - min(om)) < 1e-6


def test_smallest_eig_certified_bracket(hk):
    # N = 32, beta = 1: at K = 512 the 45-digit bracket passes the plain
    # inertia check but is not proved; the reported precision proves it
    N, beta = 32, (1, 1)
    dec, rep = hk.smallest_eig(N, beta, 512, method=hk.HK_SECANT, digits=45, flags=hk.HK_FLAG_CERTIFY)
    assert rep["verified"] == 1 and rep["certified"] == 0
    K2 = rep["certify_bits"]
    log("certify: margin %.1f bits at K=512, proposed K=%d" % (rep["certify_margin_bits"], K2))
    assert 768 < K2 <= 1024
    dec2, rep2 = hk.smallest_eig(N, beta, K2, method=hk.HK_SECANT, digits=45, flags=hk.HK_FLAG_CERTIFY)
    assert rep2["verified"] == 1 and rep2["certified"] == 1 and rep2["certify_margin_bits"] > 0
    assert dec2 == dec
