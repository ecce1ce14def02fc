"""Shifts that put the two rounding points of the factorisation exactly on a
tie ("The LDL^T Determinant Algorithm": C = A / 2^h and CDivDiag = C 2^h / d,
both rounded to h = K/2 fractional bits; the rule here is round to nearest,
ties to even).  Host-side construction only: every shift is an exact integer
with K fractional bits, built from the moments and, for the negative-pivot
case, from the oracle's own outputs.

  beta = 1, x = m 2^(h-1) / 2^K, m odd: every M entry is a multiple of 2^K,
      so A_00 = 2^K - x_fix sits exactly half-way between two multiples of
      2^h, and so does A^(1)_11 (C_0[1] = 2^h is exact, so the update
      C_0[1] L_0[1] is a multiple of 2^h): C_0[0] and C_1[1] are ties.
  any beta, x_fix = X_0 - 2^(K+1) D - e: A_00 = 2^(K+1) D + e; with e = 0,
      d_0 = 2^(h+1) D and L_0[r] = RNE(C_0[r] / 2D), a tie whenever
      C_0[r] = D mod 2D; with e = 2^(h-1) or 3 2^(h-1) the pivot itself is a
      tie (down to 2^(h+1) D, up to 2^(h+1) D + 2).
  beta = 1, N = 2, inertia mode: x just above the smaller eigenvalue of
      [[1, 1], [1, 2]] with x_fix = j 2^h + 2^(h-1) leaves A^(1)_11 a small
      negative number half-way between two multiples of 2^h: the last pivot
      is a negative tie.
"""
from fractions import Fraction


def rne(v):
    """Round a Fraction to the nearest integer, ties to even (definition)."""
    f = v.numerator // v.denominator
    r = v - f
    if r > Fraction(1, 2) or (r == Fraction(1, 2) and f % 2 == 1):
        return f + 1
    return f


def is_half(v):
    return v - (v.numerator // v.denominator) == Fraction(1, 2)


def beta1_pivot_tie_shift(K, m):
    assert m % 2 == 1
    return m << (K // 2 - 1)


def general_tie_shift(X0, K, D=1, e=0):
    return X0 - (D << (K + 1)) - e


def beta1_negative_last_pivot_shift(K, factor_fn):
    """x_fix = j 2^h + 2^(h-1) with the smallest j for which the oracle's
    last pivot of the N = 2, beta = 1 matrix is negative (A^(1)_11 decreases
    as x grows).  factor_fn(xf) -> pivots list."""
    h = K // 2
    # d_1 > 0 at x = 0 and d_1 < 0 at x = 0.9 (d_0 stays positive there)
    lo, hi = 0, (9 << h) // 10
    while hi - lo > 1:
        mid = (lo + hi) // 2
        if factor_fn((mid << h) + (1 << (h - 1)))[1] < 0:
            hi = mid
        else:
            lo = mid
    return (hi << h) + (1 << (h - 1))
