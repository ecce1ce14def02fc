"""GPU parity of the triangular solves: y = (L D L^T)^{-1} b from hk_solve
equals the oracle's solve digit for digit (vectors with K + g fractional
bits), and inverse iteration on the GPU reaches the oracle's lambda_1 to
1e-40 relative with a verified inertia bracket."""
import random
from fractions import Fraction

import pytest

import oracle
from oracle.drivers import inverse_iteration, rel_digits, secant, solve_guard_bits
from oracle.moments import moments
from tests.gpu_util import log

pytestmark = pytest.mark.gpu


def parse_dec(s):
    m, e = s.split("e")
    return Fraction(m) * Fraction(10) ** int(e)


@pytest.mark.parametrize("N,beta,K,xn,panel,seed", [
    (32, (1, 1), 512, 0, 4, 1),
    (33, (7, 4), 384, -3, 1, 2),
    (70, (3, 2), 640, 11, 3, 3),
    (65, (1, 3), 768, 0, 8, 4),
    (130, (1, 2), 1024, 5, 4, 5),
    (200, (7, 4), 2048, 0, 1, 6),      # the N = 200 workload, every digit
    (200, (7, 4), 2048, -9, 4, 7),
])
def test_solve_parity(hk, N, beta, K, xn, panel, seed):
    log("solve N=%d beta=%s K=%d panel=%d" % (N, beta, K, panel))
    rng = random.Random(9020852 + seed)
    X = moments(N, beta, K)
    xf = xn << (K // 2)
    of = oracle.factor_from_moments(X, N, K, xf)
    g = solve_guard_bits(N, K, X)
    # right-hand side: K fractional bits, |b_i| <= 1, structured and random
    b = [rng.randrange(-(1 << K), (1 << K) + 1) for _ in range(N)]
    b[0] = 1 << K
    b[-1] = 0
    y_o = oracle.solve(of, b, 3, g)
    m = hk.Matrix(N, beta, K)
    m.set_panel(panel)
    m.factor(xf)
    assert m.info().solve_guard_bits == g
    vb, vx = m.new_vec(), m.new_vec()
    m.vec_import(b, vb)
    m.solve(vb, vx)
    y_g = m.vec_export(vx)
    assert y_g == y_o


@pytest.mark.parametrize("N,beta,K", [(32, (1, 1), 512), (100, (1, 3), 1024), (60, (7, 4), 1280)])
def test_inverse_iteration_lambda(hk, N, beta, K):
    log("inverse N=%d beta=%s K=%d" % (N, beta, K))
    dec, rep = hk.smallest_eig(N, beta, K, method=hk.HK_INVERSE, digits=45)
    assert rep["verified"] == 1
    lam_o, _ = secant(N, beta, K)
    assert rel_digits(parse_dec(dec), lam_o) > 40


def test_config2_inverse_equals_secant(hk):
    N, beta, K = 200, (7, 4), 2048
    log("config2 inverse vs secant")
    d1, r1 = hk.smallest_eig(N, beta, K, method=hk.HK_INVERSE, digits=45)
    d2, r2 = hk.smallest_eig(N, beta, K, method=hk.HK_SECANT, digits=45)
    assert r1["verified"] == 1 and r2["verified"] == 1
    assert rel_digits(parse_dec(d1), parse_dec(d2)) > 40
    assert abs(float(parse_dec(d1)) / 3.9264554677562985943e-76 - 1) < 1e-15
