"""Pins for the oracle's eigenvalue drivers: brute-force eigen-solves for
N <= 12, the paper's lambda_1 and condition-number tables, the agreement of
the Secant iteration ('The Secant Algorithm') with inverse iteration, the
sign bracket of 'Interval Verification', and precision-exhaustion detection."""
import json
import os
from fractions import Fraction

import mpmath
import pytest

import oracle
from oracle.drivers import (PrecisionError, inverse_iteration, rel_digits, secant,
                            solve_guard_bits, verify)
from oracle.moments import moments

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def eigsy_lambda1(N, beta, prec=4000):
    p, q = Fraction(*beta).numerator, Fraction(*beta).denominator
    with mpmath.workprec(prec):
        M = mpmath.matrix(N, N)
        for i in range(N):
            for j in range(N):
                M[i, j] = mpmath.mpf(q) / p * mpmath.gamma(mpmath.mpf(q * (1 + i + j)) / p)
        ev = mpmath.eigsy(M, eigvals_only=True)
        return min(ev)


def mp_rel_digits(lam, ref):
    with mpmath.workprec(4000):
        a = mpmath.mpf(lam.numerator) / lam.denominator
        return -mpmath.log10(abs(a - ref) / ref)


@pytest.mark.parametrize("beta,N", [((1, 1), 12), ((7, 4), 10), ((1, 2), 8), ((3, 2), 12),
                                    ((2, 1), 11), ((5, 3), 9)])
def test_brute_force_eigsy(beta, N):
    K = 1536
    lam_ref = eigsy_lambda1(N, beta)
    X = moments(N, beta, K)
    lam_s, _ = secant(N, beta, K, X=X)
    lam_i, _ = inverse_iteration(N, beta, K, X=X)
    assert mp_rel_digits(lam_s, lam_ref) > 44
    assert mp_rel_digits(lam_i, lam_ref) > 44


def test_sylvester_bisection_exact_rational():
    # exact-rational LDL^T of the dyadic-rounded M: count negative pivots at
    # rational x and bisect; must bracket the oracle's lambda
    N, K, beta = 8, 512, (7, 4)
    X = moments(N, beta, K)
    A0 = [[Fraction(X[r + c], 1 << K) for c in range(N)] for r in range(N)]

    def negs(x):
        A = [row[:] for row in A0]
        for i in range(N):
            A[i][i] -= x
        n = 0
        for k in range(N):
            d = A[k][k]
            if d < 0:
                n += 1
            for c in range(k + 1, N):
                for r in range(c, N):
                    A[r][c] -= A[r][k] * A[c][k] / d
                    A[c][r] = A[r][c]
        return n

    lam, _ = inverse_iteration(N, beta, K)
    lo, hi = Fraction(0), Fraction(1)
    while negs(hi) == 0:
        hi *= 2
    for _ in range(120):
        mid = (lo + hi) / 2
        if negs(mid) == 0:
            lo = mid
        else:
            hi = mid
    assert lo <= lam * (1 + Fraction(1, 10 ** 30)) and lam <= hi * (1 + Fraction(1, 10 ** 30))
    assert rel_digits(lam, lo) > 30


def _parse(s):
    s = s.replace("x10^", "e")
    return mpmath.mpf(s)


@pytest.mark.parametrize("col,K", [(0, 1024), (1, 1024), (2, 1024), (3, 1536)])
def test_paper_lambda_table_N100(col, K):
    tab = json.load(open(os.path.join(GOLD, "paper_lambda_table.json")))
    beta = tuple(tab["columns_beta"][col])
    ref = _parse(tab["rows"]["100"][col])
    lam, info = secant(100, beta, K)
    with mpmath.workprec(200):
        got = mpmath.mpf(lam.numerator) / lam.denominator
        # 5 significant digits as printed
        assert abs(got - ref) <= ref * mpmath.mpf("0.51e-4")
    # cond(M) >= (1/beta) Gamma((2N-1)/beta) / lambda_1, printed to 3 digits
    ct = json.load(open(os.path.join(GOLD, "paper_cond_table.json")))
    m, e = ct["rows"]["100"][col].split("e")
    p, q = beta
    with mpmath.workprec(300):
        cond = mpmath.mpf(q) / p * mpmath.gamma(mpmath.mpf(q * 199) / p) / got
        lead = cond / mpmath.mpf(10) ** int(e)
        assert abs(lead - mpmath.mpf(m)) <= mpmath.mpf("0.0051")


@pytest.mark.slow
@pytest.mark.parametrize("col,K", [(2, 2048), (3, 2560)])
def test_paper_lambda_table_N300(col, K):
    tab = json.load(open(os.path.join(GOLD, "paper_lambda_table.json")))
    beta = tuple(tab["columns_beta"][col])
    ref = _parse(tab["rows"]["300"][col])
    lam, _ = inverse_iteration(300, beta, K, threads=0)
    with mpmath.workprec(200):
        got = mpmath.mpf(lam.numerator) / lam.denominator
        assert abs(got - ref) <= ref * mpmath.mpf("0.51e-4")


def test_secant_equals_inverse_iteration_config1():
    N, K, beta = 32, 512, (1, 1)
    lam_i, info_i = inverse_iteration(N, beta, K)
    lam_s, info_s = secant(N, beta, K)
    assert rel_digits(lam_i, lam_s) > 40
    assert abs(float(lam_i) - 5.2027073259163599130749e-8) < 1e-20
    ok, (nlo, nhi, D, e) = verify(N, beta, K, lam_i)
    assert ok and nlo == 0 and nhi == 1


def test_secant_equals_inverse_iteration_beta_7_4():
    N, K, beta = 60, 1280, (7, 4)
    X = moments(N, beta, K)
    lam_i, _ = inverse_iteration(N, beta, K, X=X)
    lam_s, _ = secant(N, beta, K, X=X)
    assert rel_digits(lam_i, lam_s) > 40
    assert verify(N, beta, K, lam_s, X=X)[0]


def test_precision_exhaustion_detected():
    # far too few bits: the iteration must report it rather than return garbage
    with pytest.raises((PrecisionError, ArithmeticError)):
        secant(100, (7, 4), 400, max_iter=60)


def test_verify_rejects_wrong_value():
    N, K, beta = 32, 512, (1, 1)
    lam, _ = inverse_iteration(N, beta, K)
    ok, _ = verify(N, beta, K, lam * Fraction(101, 100))
    assert not ok
    ok, _ = verify(N, beta, K, lam * Fraction(99, 100))
    assert not ok


def test_solve_residual_and_exact_factor():
    # beta = 1, x = 0: the factors are exact, so A y = b holds up to the
    # rounding of the three solve steps only; check the residual exactly
    N, K = 16, 256
    X = moments(N, (1, 1), K)
    f = oracle.factor_from_moments(X, N, K, 0)
    b = [((-1) ** i * (i + 3)) << (K - 2) for i in range(N)]
    g = solve_guard_bits(N, K, X)
    y = oracle.solve(f, b, 3, g)          # K + g fractional bits
    A = [[Fraction(X[r + c], 1 << K) for c in range(N)] for r in range(N)]
    yf = [Fraction(t, 1 << (K + g)) for t in y]
    for i in range(N):
        r = Fraction(b[i], 1 << K) - sum(A[i][j] * yf[j] for j in range(N))
        assert abs(r) <= Fraction(1, 1 << (K // 4))
    # stage-1 output: L z = b exactly up to one rounding per entry
    z = oracle.solve(f, b, 1, g)
    Ls = f.all_L()
    for i in range(N):
        acc = Fraction(b[i], 1 << K) - sum(Fraction(Ls[k][i - k - 1], 1 << (K // 2)) * Fraction(z[k], 1 << (K + g))
                                           for k in range(i))
        assert abs(acc - Fraction(z[i], 1 << (K + g))) <= Fraction(1, 1 << (K + g + 1))
