"""Pins for the oracle's rigorous inertia (oracle/certify.py; the paper's
'Interval Verification' in midpoint-radius form): the radii enclose the
exact Schur complements and quotients of the true matrix (exact integers at
beta = 1, mpmath at three times the working precision otherwise), the
certified signs agree with the eigenvalue counts of mpmath's eigsy, verified
brackets are certified, and a starved precision is refused."""
from fractions import Fraction

import mpmath
import pytest

import oracle
from oracle.certify import certified_inertia, certify_bracket, radii
from oracle.drivers import secant, to_fixed, truncate_digits
from oracle.moments import moments


def exact_matrix(N, beta, K, x):
    """True M - xI: Fractions at beta = 1 (M_ij = (i+j)!), else mpmath at 3K bits."""
    import math
    p, q = Fraction(*beta).numerator, Fraction(*beta).denominator
    if (p, q) == (1, 1):
        return [[Fraction(math.factorial(r + c)) - (x if r == c else 0) for c in range(N)] for r in range(N)]
    with mpmath.workprec(3 * K + 200):
        xm = mpmath.mpf(x.numerator) / x.denominator
        return [[mpmath.mpf(q) / p * mpmath.gamma(mpmath.mpf(q * (1 + r + c)) / p) - (xm if r == c else 0)
                 for c in range(N)] for r in range(N)]


@pytest.mark.parametrize("N,beta,K,xn", [(8, (1, 1), 128, 0), (10, (1, 1), 192, 3), (9, (7, 4), 256, -5),
                                         (12, (3, 2), 320, 1), (8, (1, 2), 256, 0)])
def test_radii_enclose_exact_schur_complements(N, beta, K, xn):
    h = K // 2
    xf = xn << h
    X = moments(N, beta, K)
    f = oracle.factor_from_moments(X, N, K, xf)
    piv, eD, G = radii(N, K, X, xf, f)
    # recompute the radii of every C entry and L quotient alongside the exact
    # elimination of the true matrix
    x = Fraction(xf, 1 << K)
    S = exact_matrix(N, beta, K, x)
    exact = isinstance(S[0][0], Fraction)
    ctx = mpmath.workprec(3 * K + 200)
    ctx.__enter__()
    try:
        # the enclosure of the C entries is checked through the pivot radii
        # returned (eD) and, for the other entries, by re-running the
        # recursion here with every radius kept
        from oracle.certify import _ceil_div
        sh = G - h
        half = 1 << (G - h - 1)
        rho = [[1 << (G - K - 1)] * (r + 1) for r in range(N)]
        for k in range(N):
            C = f.column_C(k)
            eC = [rho[r][k] + half for r in range(k, N)]
            assert eC[0] == eD[k]
            for i, r in enumerate(range(k, N)):
                err = abs(S[r][k] - (Fraction(C[i], 1 << h) if exact else mpmath.mpf(C[i]) / 2 ** h))
                assert err <= (Fraction(eC[i], 1 << G) if exact else mpmath.mpf(eC[i]) / 2 ** G)
            if k == N - 1:
                break
            L = f.column_L(k)
            D = C[0] << sh
            assert D > eC[0]
            den = D * (D - eC[0])
            eL = []
            for i in range(1, N - k):
                eq = _ceil_div((eC[i] * D + (abs(C[i]) << sh) * eC[0]) << G, den)
                eL.append(eq + half)
                r = k + i
                qx = S[r][k] / S[k][k]
                err = abs(qx - (Fraction(L[i - 1], 1 << h) if exact else mpmath.mpf(L[i - 1]) / 2 ** h))
                assert err <= (Fraction(eL[-1], 1 << G) if exact else mpmath.mpf(eL[-1]) / 2 ** G)
            # exact elimination step and the radius update
            for c in range(k + 1, N):
                for r in range(c, N):
                    S[r][c] = S[r][c] - S[c][k] * S[r][k] / S[k][k]
                    Cc = abs(C[c - k]) << sh
                    Lr = abs(L[r - k - 1]) << sh
                    ec, el = eC[c - k], eL[r - k - 1]
                    rho[r][c] += _ceil_div(Cc * el + ec * Lr + ec * el, 1 << G)
    finally:
        ctx.__exit__(None, None, None)


@pytest.mark.parametrize("beta,N", [((1, 1), 8), ((7, 4), 7), ((1, 2), 9), ((3, 2), 10)])
def test_certified_inertia_counts_eigenvalues(beta, N):
    K = 1024
    p, q = Fraction(*beta).numerator, Fraction(*beta).denominator
    with mpmath.workprec(3000):
        M = mpmath.matrix(N, N)
        for i in range(N):
            for j in range(N):
                M[i, j] = mpmath.mpf(q) / p * mpmath.gamma(mpmath.mpf(q * (1 + i + j)) / p)
        ev = sorted(mpmath.eigsy(M, eigvals_only=True))
        pts = [(ev[0] / 2, 0), (ev[0] * (1 - mpmath.mpf(10) ** -30), 0), (ev[0] * (1 + mpmath.mpf(10) ** -30), 1)]
        pts = [(int(mpmath.floor(x * mpmath.mpf(2) ** K)), n) for x, n in pts]
    X = moments(N, beta, K)
    for xf, want in pts:
        n, ok = certified_inertia(N, K, X, xf)
        assert ok and n == want, (xf, want, n, ok)


def test_verified_bracket_certified_with_more_bits_config1():
    # N = 32, beta = 1: the 45-digit bracket of the Secant root at K = 512
    # passes the plain inertia check, but the radii (which grow by about 8
    # bits a column here) exceed the last pivot by 2^152 at K = 512, 2^24 at
    # 768; from K = 832 on the same decimal bracket is proved
    N, beta = 32, (1, 1)
    lam, _ = secant(N, beta, 512)
    D, e = truncate_digits(lam, 45)
    lo_d, hi_d = Fraction(D) * Fraction(10) ** e, Fraction(D + 1) * Fraction(10) ** e
    for K, want in [(512, False), (768, False), (832, True), (1024, True)]:
        X = moments(N, beta, K)
        lo, hi = to_fixed(lo_d, K, "floor"), to_fixed(hi_d, K, "ceil")
        assert certify_bracket(N, beta, K, lo, hi, X=X) == want, K
    # a bracket that misses lambda_1 is not certified
    K = 1024
    X = moments(N, beta, K)
    lo, hi = to_fixed(lo_d, K, "floor"), to_fixed(hi_d, K, "ceil")
    assert not certify_bracket(N, beta, K, hi, hi + (hi - lo), X=X)
    assert not certify_bracket(N, beta, K, lo - (hi - lo), lo, X=X)


def test_starved_precision_is_not_certified():
    # N = 24, beta = 1 at K = 96: the factorisation still has positive pivots
    # at x = 0, but the radii outgrow the small trailing pivots
    N, beta, K = 24, (1, 1), 96
    X = moments(N, beta, K)
    f = oracle.factor_from_moments(X, N, K, 0)
    n, ok = certified_inertia(N, K, X, 0, f)
    assert f.n_negative == 0 and not ok
