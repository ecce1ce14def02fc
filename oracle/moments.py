"""Oracle: correctly rounded fixed-point moments (TEST INFRASTRUCTURE ONLY).

The matrix is M_ij = (1/beta) Gamma((1+i+j)/beta), i, j = 0..N-1 (paper,
Introduction), i.e. M_ij = mu_{i+j} with mu_n the n-th moment of the weight
exp(-x^beta) on [0, inf) ("Properties of M").  Entries are stored with K bits
after the binary point ("The LDL^T Determinant Algorithm"); the paper does not
say how they are rounded, and the reading used here is round-to-nearest,
ties-to-even of the exact real value, so

    X_n = RNE(2^K mu_n),   n = 0 .. 2N-2.

With beta = p/q in lowest terms, mu_n = (q/p) Gamma(q(n+1)/p).  Writing
q(n+1) = m p + r (0 <= r < p):

  * r = 0:  Gamma(m) = (m-1)!, so X_n is a rounded exact rational;
  * r > 0:  Gamma(m + r/p) = Gamma(r/p) * prod_{j<m} (r + j p) / p^m, so only
            the p-1 constants Gamma(r/p) are transcendental.

Gamma(s), 0 < s < 1, comes from the classical split Gamma(s) = gamma(s, T) +
Gamma(s, T) with the lower incomplete function summed as the confluent series
gamma(s, T) = T^s e^{-T} sum_k T^k / (s (s+1) ... (s+k)) and the upper part
bounded by 0 <= Gamma(s, T) <= T^{s-1} e^{-T} <= e^{-T}.  Choosing T = u^p
(u an integer) makes T^s = u^r exact.  Every quantity is carried as a pair of
integers that bound the true value from below and above (floor / ceiling
chains, the truncated tails bounded explicitly), so X_n is exact whenever the
two rounded bounds agree; otherwise the working precision is doubled (Ziv's
strategy).  Pure Python integers throughout; parity pinned against mpmath and
exact closed forms in tests/test_oracle_moments.py.
"""
import math
from fractions import Fraction
from functools import lru_cache


def reduce_beta(beta):
    """beta given as (num, den), Fraction or int -> (p, q) with beta = p/q."""
    if isinstance(beta, tuple):
        fr = Fraction(beta[0], beta[1])
    else:
        fr = Fraction(beta)
    if fr <= 0:
        raise ValueError("beta must be positive")
    return fr.numerator, fr.denominator


def rne_div(num, den):
    """Round num/den to the nearest integer, ties to even (den != 0)."""
    if den < 0:
        num, den = -num, -den
    neg = num < 0
    a = -num if neg else num
    q, r = divmod(a, den)
    if 2 * r > den or (2 * r == den and (q & 1)):
        q += 1
    return -q if neg else q


def _iroot_ceil(x, p):
    """Smallest integer u >= 1 with u^p >= x."""
    u = max(1, int(round(x ** (1.0 / p))))
    while u ** p < x:
        u += 1
    while u > 1 and (u - 1) ** p >= x:
        u -= 1
    return u


def _series_bounds(G, T, r, p):
    """Bounds (lo, hi) on 2^G * sum_{k>=0} T^k p^{k+1} / prod_{j<=k}(r + j p)
    (the confluent series with s = r/p); floor / ceiling chains."""
    lo_t = (p << G) // r
    hi_t = -((-(p << G)) // r)
    lo_s, hi_s = lo_t, hi_t
    k = 0
    tp = T * p
    while True:
        k += 1
        den = r + k * p
        lo_t = (lo_t * tp) // den
        hi_t = -((-(hi_t * tp)) // den)
        lo_s += lo_t
        hi_s += hi_t
        # remaining terms shrink by a factor <= tp / den' < 1/2 once den' > 2 tp
        if den > 2 * tp and hi_t <= 1:
            hi_s += 1  # geometric tail <= current term <= 1 unit
            return lo_s, hi_s


def _exp_bounds(G, T):
    """Bounds (lo, hi) on 2^G e^T = 2^G sum_k T^k / k!."""
    lo_t = hi_t = 1 << G
    lo_s = hi_s = 1 << G
    k = 0
    while True:
        k += 1
        lo_t = (lo_t * T) // k
        hi_t = -((-(hi_t * T)) // k)
        lo_s += lo_t
        hi_s += hi_t
        if k > 2 * T and hi_t <= 1:
            hi_s += 1
            return lo_s, hi_s


@lru_cache(maxsize=64)
def gamma_frac_bounds(r, p, F):
    """Integers (lo, hi) with lo <= 2^F Gamma(r/p) <= hi, for 0 < r < p."""
    if not 0 < r < p:
        raise ValueError("need 0 < r < p")
    # tail e^{-T} must be below 2^{-F-8}: T > (F + 8) ln 2
    Tmin = (F + 8) * math.log(2.0) + 2.0
    u = _iroot_ceil(Tmin, p)
    T = u ** p
    G = F + 64 + 2 * max(1, int(T).bit_length())
    s_lo, s_hi = _series_bounds(G, T, r, p)
    e_lo, e_hi = _exp_bounds(G, T)
    ur = u ** r
    lo = (ur * s_lo << F) // e_hi
    hi = -((-(ur * s_hi << F)) // e_lo)
    hi += -((-(1 << (F + G))) // e_lo)  # upper incomplete part <= e^{-T}
    return lo, hi


def log2_mu_estimate(n, p, q):
    """Float estimate of log2 mu_n (for choosing precision only)."""
    x = q * (n + 1) / p
    return (math.lgamma(x) + math.log(q / p)) / math.log(2.0)


def moments(N, beta, K, guard=64):
    """X_n = RNE(2^K mu_n), n = 0..2N-2, mu_n = (1/beta) Gamma((n+1)/beta).
    Gamma is enclosed with `guard` bits beyond the ones the result needs; the
    guard doubles until every rounding is decided (the result does not depend
    on the starting guard)."""
    p, q = reduce_beta(beta)
    nmax = 2 * N - 2
    top = max(log2_mu_estimate(n, p, q) for n in range(0, nmax + 1))
    while True:
        F = K + max(0, int(math.ceil(top))) + guard
        out = []
        ok = True
        gam = {}
        prods = {}
        for n in range(nmax + 1):
            a = q * (n + 1)
            m, r = divmod(a, p)
            if r == 0:
                out.append(rne_div((q * math.factorial(m - 1)) << K, p))
                continue
            if r not in gam:
                gam[r] = gamma_frac_bounds(r, p, F)
            # prod_{j<m} (r + j p), extended incrementally per residue
            mm, P = prods.get(r, (0, 1))
            while mm < m:
                P *= r + mm * p
                mm += 1
            prods[r] = (mm, P)
            g_lo, g_hi = gam[r]
            den = p ** (m + 1) << F
            lo = rne_div((q * P * g_lo) << K, den)
            hi = rne_div((q * P * g_hi) << K, den)
            if lo != hi:
                ok = False
                break
            out.append(lo)
        if ok:
            return out
        guard *= 2


def gamma_fixed(r, p, F):
    """Convenience for tests: 2^F Gamma(r/p) rounded to nearest, requiring the
    interval to decide the rounding (raises otherwise)."""
    lo, hi = gamma_frac_bounds(r, p, F + 32)
    a, b = rne_div(lo, 1 << 32), rne_div(hi, 1 << 32)
    if a != b:
        raise ArithmeticError("undecided")
    return a
