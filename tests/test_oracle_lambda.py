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
from oracle.drivers import (PrecisionError, bracket_root, inverse_iteration, rel_digits, secant,
                            solve_guard_bits, to_fixed, verify)
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


def exact_negative_pivots(X, N, K, x):
    """Negative pivots of the exact-rational LDL^T of the dyadic-rounded
    M - xI (Sylvester's inertia: the number of eigenvalues below x)."""
    A = [[Fraction(X[r + c], 1 << K) for c in range(N)] for r in range(N)]
    for i in range(N):
        A[i][i] -= x
    n = 0
    for k in range(N):
        d = A[k][k]
        if d == 0:
            raise ZeroDivisionError("singular leading block at this shift")
        if d < 0:
            n += 1
        for c in range(k + 1, N):
            for r in range(c, N):
                A[r][c] -= A[r][k] * A[c][k] / d
                A[c][r] = A[r][c]
    return n


def exact_bisection(X, N, K, steps=160):
    """lambda_1 of the dyadic-rounded matrix bracketed by bisection on the
    exact inertia: (lo, hi) with no eigenvalue below lo and one below hi."""
    lo, hi = Fraction(0), Fraction(1, 3)      # (1/3: not a point where a pivot vanishes)
    while exact_negative_pivots(X, N, K, hi) == 0:
        hi *= 2
    for _ in range(steps):
        mid = (lo + hi) / 2
        if exact_negative_pivots(X, N, K, mid) == 0:
            lo = mid
        else:
            hi = mid
    return lo, hi


def test_sylvester_bisection_exact_rational():
    # exact-rational LDL^T of the dyadic-rounded M: count negative pivots at
    # rational x and bisect; must bracket the oracle's lambda
    N, K, beta = 8, 512, (7, 4)
    X = moments(N, beta, K)
    lam, _ = inverse_iteration(N, beta, K)
    lo, hi = exact_bisection(X, N, K, 120)
    assert lo <= lam * (1 + Fraction(1, 10 ** 30)) and lam <= hi * (1 + Fraction(1, 10 ** 30))
    assert rel_digits(lam, lo) > 30


@pytest.mark.parametrize("N,beta,K,mult", [(8, (7, 4), 512, 4), (10, (3, 2), 768, 8), (12, (1, 1), 512, 3)])
def test_bracket_phase_illinois(N, beta, K, mult):
    """The bracketing phase on its own from [0, mult * lambda_1]: the
    function values of the two ends have opposite signs and one end stays
    put for consecutive steps, so the Illinois halving must act (a nonzero
    scale in the trace).  It must land on the root that exact-rational
    bisection of the same dyadic-rounded matrix gives (to the 40 digits the
    fixed-point factorisation at this K resolves), and converge
    superlinearly: plain regula falsi needs over 40 factorisations on the
    first case, bisection about 160, the Illinois form at most 16."""
    X = moments(N, beta, K)
    lo, hi = exact_bisection(X, N, K)
    b = to_fixed(hi * mult, K, "ceil")
    trace = []
    lam, info = bracket_root(N, beta, K, 0, b, X=X, trace=trace)
    assert info["bracketed"] and info["factorizations"] <= 16
    assert any(t[4] > 0 or t[5] > 0 for t in trace)
    # the returned lower end has P > 0, and it lies within the tolerance
    assert rel_digits(lam, lo) > 40


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
