"""Pins for the oracle's fixed-point LDL^T (paper, 'The LDL^T Determinant
Algorithm': M entries with K fractional bits, C and CDivDiag with K/2) against
closed forms, exact rational arithmetic and eigenvalue counts."""
import math
import random
from fractions import Fraction

import mpmath
import pytest

import oracle
from oracle.moments import moments


def closed_C(pc, r, h):
    return (math.factorial(r) ** 2 // math.factorial(r - pc)) << h


def closed_L(pc, r, h):
    return (math.comb(r, pc) * math.factorial(r) // math.factorial(pc)) << h


def test_beta1_closed_forms_every_limb_config1():
    # beta = 1, x = 0: A^{(pc)}_{r,pc} = (r!)^2/(r-pc)!, L = C(r,pc) r!/pc!,
    # d_pc = (pc!)^2 -- all exact in the fixed-point format, so every digit of
    # the oracle's output is fixed (N = 32, K = 512 is the small config).
    N, K = 32, 512
    h = K // 2
    f = oracle.factor(N, (1, 1), K, 0)
    assert f.status == 0 and f.first_nonpos == -1 and f.n_negative == 0
    C, L = f.all_C(), f.all_L()
    for pc in range(N):
        assert C[pc] == [closed_C(pc, r, h) for r in range(pc, N)]
    for pc in range(N - 1):
        assert L[pc] == [closed_L(pc, r, h) for r in range(pc + 1, N)]
    # det M = prod (k!)^2
    det = 1
    for d in f.pivots():
        det *= d
    assert det == math.prod(math.factorial(k) ** 2 for k in range(N)) << (h * N)
    assert f.limb_macs == 641306.0


def exact_ldl(Af):
    """Exact rational LDL^T (no pivoting) of a symmetric Fraction matrix."""
    n = len(Af)
    A = [row[:] for row in Af]
    Cs, Ls = [], []
    for k in range(n):
        Cs.append([A[r][k] for r in range(k, n)])
        d = A[k][k]
        Ls.append([A[r][k] / d for r in range(k + 1, n)])
        for c in range(k + 1, n):
            for r in range(c, n):
                A[r][c] -= A[c][k] * A[r][k] / d
                A[c][r] = A[r][c]
    return Cs, Ls


@pytest.mark.parametrize("beta,N,K,xnum", [((7, 4), 10, 400, -3), ((3, 2), 12, 512, 5),
                                           ((2, 1), 9, 256, 0), ((1, 3), 8, 300, 7),
                                           ((5, 8), 11, 350, -1)])
def test_against_exact_rational_ldl(beta, N, K, xnum):
    h = K // 2
    X = moments(N, beta, K)
    x_fixed = xnum << (K - 40)                     # a dyadic shift x = xnum * 2^-40
    Af = [[Fraction(X[r + c] - (x_fixed if r == c else 0), 1 << K) for c in range(N)] for r in range(N)]
    Ce, Le = exact_ldl(Af)
    f = oracle.factor_from_moments(X, N, K, x_fixed)
    C, L = f.all_C(), f.all_L()
    # column 0 has no accumulated error: both rounding points are RNE, i.e.
    # within half a unit of 2^-h of the exact value
    for i, r in enumerate(range(0, N)):
        assert abs(Fraction(C[0][i], 1 << h) - Ce[0][i]) <= Fraction(1, 1 << (h + 1))
    for i in range(N - 1):
        assert abs(Fraction(L[0][i], 1 << h) - Fraction(C[0][i + 1], C[0][0])) <= Fraction(1, 1 << (h + 1))
    # later columns: relative deviation far below 2^-(h/2) (a dropped term, a
    # wrong index or a wrong sign moves them by O(1) relative)
    for k in range(N):
        for i in range(len(Ce[k])):
            ex = Ce[k][i]
            got = Fraction(C[k][i], 1 << h)
            assert abs(got - ex) <= abs(ex) * Fraction(1, 1 << (h // 2)) + Fraction(1, 1 << (h // 2))
    for k in range(N - 1):
        for i in range(len(Le[k])):
            ex = Le[k][i]
            got = Fraction(L[k][i], 1 << h)
            assert abs(got - ex) <= abs(ex) * Fraction(1, 1 << (h // 2)) + Fraction(1, 1 << (h // 2))


def test_rne_ties_are_even():
    # a column-0 entry that is an exact half ulp at h bits must round to even
    N, K = 3, 16
    h = K // 2
    X = [(1 << 20), (5 << 7) + (1 << 7) // 2 * 1, (7 << 12), 9 << 16, 11 << 16]
    X[1] = (2 * 3 + 1) << (h - 1)          # (3 + 1/2) units of 2^h -> 4
    X[2] = (2 * 4 + 1) << (h - 1)          # (4 + 1/2) -> 4
    f = oracle.factor_from_moments(X, N, K, 0)
    C0 = f.column_C(0)
    assert C0[1] == 4 and C0[2] == 4


def test_prefix_invariance():
    # the leading n x n block of M_N is M_n, so the first rows of every column
    # of the N-factorisation equal the n-factorisation
    K = 640
    fa = oracle.factor(24, (7, 4), K, 12345)
    fb = oracle.factor(16, (7, 4), K, 12345)
    Ca, La, Cb, Lb = fa.all_C(), fa.all_L(), fb.all_C(), fb.all_L()
    for k in range(16):
        assert Ca[k][:16 - k] == Cb[k]
    for k in range(15):
        assert La[k][:15 - k] == Lb[k]


def test_partial_factorisation_matches_full():
    K = 512
    fa = oracle.factor(20, (3, 2), K, 0)
    fb = oracle.factor(20, (3, 2), K, 0, ncols=7)
    assert fb.all_C() == fa.all_C(0, 7)
    assert fb.all_L() == fa.all_L(0, 7)


@pytest.mark.parametrize("beta,N", [((1, 1), 8), ((7, 4), 7), ((1, 2), 9), ((3, 2), 10)])
def test_inertia_counts_eigenvalues(beta, N):
    # Sylvester: #negative pivots of M - xI = #eigenvalues below x
    K = 1024
    p, q = Fraction(*beta).numerator, Fraction(*beta).denominator
    with mpmath.workprec(3000):
        M = mpmath.matrix(N, N)
        for i in range(N):
            for j in range(N):
                M[i, j] = mpmath.mpf(q) / p * mpmath.gamma(mpmath.mpf(q * (1 + i + j)) / p)
        ev = sorted(mpmath.eigsy(M, eigvals_only=True))
        pts = []
        for i in range(min(N - 1, 3)):
            pts.append(((ev[i] + ev[i + 1]) / 2, i + 1))
        pts.append((ev[0] / 2, 0))
        pts.append((ev[0] * (1 + mpmath.mpf(10) ** -30), -1))
        pts.append((ev[0] * (1 - mpmath.mpf(10) ** -30), 0))
        pts = [(int(mpmath.floor(x * mpmath.mpf(2) ** K)), n) for x, n in pts]
    X = moments(N, beta, K)
    for xf, want in pts:
        f = oracle.factor_from_moments(X, N, K, xf)
        if want == -1:
            # just above lambda_1 every leading block is still positive
            # definite, so the only negative pivot is the last one
            assert f.n_negative == 1 and f.first_nonpos == N - 1
        else:
            assert f.n_negative == want, (xf, want)


# ---- constructed rounding ties (the shifts of tests/tie_cases.py) ----------
from tests.tie_cases import (beta1_negative_last_pivot_shift, beta1_pivot_tie_shift, general_tie_shift,
                             is_half, rne)


@pytest.mark.parametrize("K,m", [(512, 1), (512, 3), (512, -1), (8192, 1), (16640, 3)])
def test_beta1_pivot_ties(K, m):
    # beta = 1, x_fix = m 2^(h-1): A_00 and A^(1)_11 are exact halves at h
    # bits; the first two columns checked against exact rational arithmetic
    N, h = 6, K // 2
    xf = beta1_pivot_tie_shift(K, m)
    f = oracle.factor(N, (1, 1), K, xf)
    C0, C1, L0 = f.column_C(0), f.column_C(1), f.column_L(0)
    a00 = Fraction((1 << K) - xf, 1 << h)
    assert is_half(a00)
    assert C0[0] == rne(a00) and C0[0] % 2 == 0
    assert C0[1:] == [math.factorial(r) << h for r in range(1, N)]
    assert L0 == [rne(Fraction(C0[i] << h, C0[0])) for i in range(1, N)]
    a11 = Fraction((2 << K) - xf - C0[1] * L0[0], 1 << h)
    assert is_half(a11)
    assert C1[0] == rne(a11) and C1[0] % 2 == 0


@pytest.mark.parametrize("beta,K,D,e", [((3, 2), 640, 1, 0), ((3, 2), 640, 1, 1), ((3, 2), 640, 1, 3),
                                        ((5, 3), 640, 3, 0), ((2, 7), 1024, 5, 0), ((3, 2), 8192, 1, 0)])
def test_general_division_ties(beta, K, D, e):
    # x_fix = X_0 - 2^(K+1) D - e 2^(h-1): the pivot is 2^(h+1) D (e = 0, 1) or
    # 2^(h+1) D + 2 (e = 3), and L_0[r] = RNE(C_0[r] 2^h / d_0) is a tie for
    # every C_0[r] = D mod 2D when e < 3
    N, h = 40, K // 2
    X = moments(N, beta, K)
    xf = general_tie_shift(X[0], K, D, e << (h - 1) if e else 0)
    f = oracle.factor_from_moments(X, N, K, xf)
    C0, L0 = f.column_C(0), f.column_L(0)
    assert C0[0] == (D << (h + 1)) + (2 if e == 3 else 0)
    assert C0[1:] == [rne(Fraction(X[r], 1 << h)) for r in range(1, N)]
    q = [Fraction(C0[i] << h, C0[0]) for i in range(1, N)]
    assert L0 == [rne(v) for v in q]
    ties = sum(is_half(v) for v in q)
    if e < 3:
        assert ties >= 1 and ties == sum(c % (2 * D) == D for c in C0[1:])


def test_beta1_negative_last_pivot_tie():
    # N = 2, beta = 1, x just above the smaller eigenvalue (3 - 5^(1/2))/2 of
    # [[1, 1], [1, 2]]: the last pivot is a negative exact half at h bits
    K = 512
    h = K // 2
    X = moments(2, (1, 1), K)

    def piv(xf):
        return oracle.factor_from_moments(X, 2, K, xf).pivots()
    xf = beta1_negative_last_pivot_shift(K, piv)
    f = oracle.factor_from_moments(X, 2, K, xf)
    d0, d1 = f.pivots()
    assert d0 == rne(Fraction(X[0] - xf, 1 << h)) > 0
    L01 = f.column_L(0)[0]
    assert L01 == rne(Fraction(f.column_C(0)[1] << h, d0))
    a11 = Fraction(X[2] - xf - f.column_C(0)[1] * L01, 1 << h)
    assert a11 < 0 and is_half(a11)
    assert d1 == rne(a11) and d1 % 2 == 0
    assert f.n_negative == 1 and f.first_nonpos == 1
    # x between the two eigenvalues of the 2 x 2 matrix
    x = Fraction(xf, 1 << K)
    assert (3 - 2.2360679775) / 2 < float(x) < 0.9
