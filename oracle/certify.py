"""Rigorous inertia of M - xI around the fixed-point factorisation
(TEST INFRASTRUCTURE ONLY; the paper's "Interval Verification" made
rigorous).

The paper checks the signs of det(M - xI) at the truncated root and one unit
above it in fixed-point interval arithmetic.  Here the interval form is
midpoint-radius: the midpoints are the fixed-point factorisation itself
(the C, L and pivots of ``oracle.factor``), and a radius per entry bounds
the distance from the midpoint to the exact value of the same quantity in
exact arithmetic on the true matrix (M with the true moments, x exact):

  A^(0)_rc:  the true entry is within rho = 2^-(K+1) of X_{r+c}/2^K - [r=c] x
             (the moments are correctly rounded);
  column k:  C_k[r] = RNE(A^(k)_rk / 2^h) is within eC = rho_rk + 2^-(h+1) of
             the exact Schur complement entry S_rk; the pivot d_k = C_k[k]
             within eD = eC[k]; when d_k > eD the exact quotient S_rk / S_kk
             is within eQ = (eC[r] + |C_k[r] / d_k| eD) / (d_k - eD) of
             C_k[r] / d_k, so L_k[r] = RNE(C_k[r] 2^h / d_k) is within
             eL = eQ + 2^-(h+1) of it;
  update:    rho_rc += |C_k[c]| eL[r] + eC[c] |L_k[r]| + eC[c] eL[r]
             (the exact update subtracts S_ck (S_rk / S_kk), the fixed-point
             one C_k[c] L_k[r]).

A pivot is certified positive when d_k > eD, negative when d_k < -eD.  All
pivots certified positive prove M - xI positive definite (lambda_1 > x); the
first N - 1 certified positive and the last certified negative prove exactly
one eigenvalue below x (Sylvester), given that a pivot's sign is that of the
exact pivot.  The radii are integers in units of 2^-G (G = K + 32), every
operation rounded up, so each is an upper bound of the exact recursion.
"""
from . import factor_from_moments
from .moments import moments


def _ceil_div(a, b):
    return -((-a) // b)


def radii(N, K, X, x_fixed, f=None, G=None):
    """Run the radius recursion along the oracle's factorisation f of
    M - xI (computed here when not given).  Returns (pivots, eD, G): the
    pivots (h fractional bits) and their radii (units 2^-G), and G."""
    h = K // 2
    G = K + 32 if G is None else G
    f = factor_from_moments(X, N, K, x_fixed) if f is None else f
    sh = G - h                       # C, L, d in units of 2^-G: value << sh
    half = 1 << (G - h - 1)          # 2^-(h+1) in units of 2^-G
    # rho[r][c] for r >= c (lower triangle), units 2^-G; the moments' half ulp
    rho0 = 1 << (G - K - 1)
    rho = [[rho0] * (r + 1) for r in range(N)]
    piv = f.pivots()
    eD = []
    for k in range(N):
        C = f.column_C(k)                      # C_k[r], r = k..N-1
        eC = [rho[r][k] + half for r in range(k, N)]
        d = C[0]
        eD.append(eC[0])
        if k == N - 1:
            break
        D = d << sh
        if D <= eC[0]:
            # the pivot is not certified positive: later radii are not bounded
            eD.extend([None] * (N - 1 - k))
            break
        L = f.column_L(k)                      # L_k[r], r = k+1..N-1
        den = D * (D - eC[0])
        eL = []
        for i in range(1, N - k):
            Cr = abs(C[i]) << sh
            eQ = _ceil_div((eC[i] * D + Cr * eC[0]) << G, den)
            eL.append(eQ + half)
        for ci in range(1, N - k):             # column c = k + ci
            c = k + ci
            Cc = abs(C[ci]) << sh
            ec = eC[ci]
            for ri in range(ci, N - k):        # row r = k + ri >= c
                r = k + ri
                Lr = abs(L[ri - 1]) << sh
                el = eL[ri - 1]
                rho[r][c] += _ceil_div(Cc * el + ec * Lr + ec * el, 1 << G)
    return piv, eD, G


def certified_inertia(N, K, X, x_fixed, f=None):
    """(n_negative, certified): the pivots' signs, and whether every sign is
    certified (the exact pivot has the same sign)."""
    h = K // 2
    piv, eD, G = radii(N, K, X, x_fixed, f)
    sh = G - h
    ok = True
    nneg = 0
    for d, e in zip(piv, eD):
        if e is None:
            ok = False
            continue
        D = d << sh
        if D > e:
            continue
        if D < -e:
            nneg += 1
        else:
            ok = False
    return nneg, ok


def certify_bracket(N, beta, K, lo_fixed, hi_fixed, X=None):
    """True when lambda_1 in (lo, hi) is proved: every pivot at lo certified
    positive, and at hi the first N - 1 certified positive and the last
    certified negative."""
    X = moments(N, beta, K) if X is None else X
    n_lo, ok_lo = certified_inertia(N, K, X, lo_fixed)
    f_hi = factor_from_moments(X, N, K, hi_fixed)
    n_hi, ok_hi = certified_inertia(N, K, X, hi_fixed, f_hi)
    last_neg = f_hi.pivots()[-1] < 0 and f_hi.first_nonpos == N - 1
    return ok_lo and n_lo == 0 and ok_hi and n_hi == 1 and last_neg
