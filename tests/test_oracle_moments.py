"""Pins for the oracle's correctly rounded moments X_n = RNE(2^K mu_n),
mu_n = (1/beta) Gamma((n+1)/beta) (paper, Introduction and 'Properties of M')."""
import json
import math
import os
from fractions import Fraction

import mpmath
import pytest

from oracle.moments import gamma_frac_bounds, moments, rne_div

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def mp_moment_fixed(n, p, q, K, prec):
    """Independent reference: mpmath Gamma at `prec` bits, then RNE."""
    with mpmath.workprec(prec):
        v = mpmath.mpf(q) / p * mpmath.gamma(mpmath.mpf(q * (n + 1)) / p) * mpmath.mpf(2) ** K
        fl = int(mpmath.floor(v))
        frac = v - fl
        if frac > 0.5:
            return fl + 1
        if frac < 0.5:
            return fl
        raise AssertionError("tie at this precision")


def test_beta_one_factorials():
    # beta = 1: M_ij = (i+j)!  (paper's first worked example)
    K = 96
    X = moments(20, (1, 1), K)
    assert X == [math.factorial(n) << K for n in range(39)]


def test_beta_half_exact():
    # beta = 1/2: mu_n = 2 (2n+1)!
    K = 64
    X = moments(10, (1, 2), K)
    assert X == [(2 * math.factorial(2 * n + 1)) << K for n in range(19)]


def test_beta_one_third_exact():
    K = 40
    X = moments(6, (1, 3), K)
    assert X == [(3 * math.factorial(3 * n + 2)) << K for n in range(11)]


def test_paper_worked_example_beta_7_4():
    ex = json.load(open(os.path.join(GOLD, "paper_examples_4x4.json")))
    K = 200
    X = moments(4, (7, 4), K)
    num, den = ex["beta_7_4_prefactor"]
    for i in range(4):
        for j in range(4):
            a = ex["beta_7_4_gamma_numerator_over_7"][i][j]
            with mpmath.workprec(600):
                v = mpmath.mpf(num) / den * mpmath.gamma(mpmath.mpf(a) / 7)
                got = mpmath.mpf(X[i + j]) / mpmath.mpf(2) ** K
                assert abs(got - v) <= mpmath.mpf(2) ** (-K)
    fa = ex["beta_1_factorial_arg"]
    Y = moments(4, (1, 1), 8)
    for i in range(4):
        for j in range(4):
            assert Y[i + j] == math.factorial(fa[i][j]) << 8


@pytest.mark.parametrize("beta", [(2, 1), (7, 4), (3, 2), (5, 3), (8, 3), (1, 1), (2, 7)])
def test_against_mpmath(beta):
    p, q = Fraction(*beta).numerator, Fraction(*beta).denominator
    N, K = 12, 300
    X = moments(N, beta, K)
    for n in range(2 * N - 1):
        assert X[n] == mp_moment_fixed(n, p, q, K, 2 * K + 400), (beta, n)


def test_gamma_half_is_sqrt_pi():
    F = 2000
    lo, hi = gamma_frac_bounds(1, 2, F)
    assert 0 <= hi - lo < 2 ** 40
    with mpmath.workprec(F + 200):
        ref = mpmath.sqrt(mpmath.pi) * mpmath.mpf(2) ** F
        assert lo <= ref <= hi


@pytest.mark.parametrize("p", [3, 4, 5, 7, 8])
def test_gauss_multiplication(p):
    # prod_{r=1}^{p-1} Gamma(r/p) = (2 pi)^{(p-1)/2} / sqrt(p)
    F = 800
    lo, hi = 1, 1
    for r in range(1, p):
        a, b = gamma_frac_bounds(r, p, F)
        lo, hi = lo * a, hi * b
    with mpmath.workprec(F * p + 200):
        ref = (2 * mpmath.pi) ** (mpmath.mpf(p - 1) / 2) / mpmath.sqrt(p) * mpmath.mpf(2) ** (F * (p - 1))
        assert lo <= ref <= hi
    assert (hi - lo) * 2 ** 30 < lo  # interval is tight


def test_reflection():
    # Gamma(1/3) Gamma(2/3) = pi / sin(pi/3) = 2 pi / sqrt(3)
    F = 600
    a0, a1 = gamma_frac_bounds(1, 3, F)
    b0, b1 = gamma_frac_bounds(2, 3, F)
    with mpmath.workprec(2 * F + 100):
        ref = 2 * mpmath.pi / mpmath.sqrt(3) * mpmath.mpf(2) ** (2 * F)
        assert a0 * b0 <= ref <= a1 * b1


@pytest.mark.parametrize("beta", [(7, 4), (2, 7), (5, 3)])
def test_rounding_stable_under_more_guard(beta):
    # the Gamma enclosures at 64 and at 320 guard bits must decide every
    # rounding the same way: each X_n is the correctly rounded value, so a
    # bound that failed to enclose Gamma would show as a differing X_n
    X1 = moments(30, beta, 512, guard=64)
    X2 = moments(30, beta, 512, guard=320)
    assert X1 == X2
    assert all(x > 0 for x in X1)
