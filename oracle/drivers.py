"""Oracle drivers for the smallest eigenvalue (TEST INFRASTRUCTURE ONLY).

All arithmetic here is on Python integers and ``fractions.Fraction``; the
factorisations and solves come from the oracle's C core.  Fixed-point values
are integers with K fractional bits unless stated.

  * ``secant``      -- the paper's Secant root finder on P(x) = det(M - xI)
                       ("The Secant Algorithm"): start at a small negative x1
                       and x2 = 0, iterate x_{i+1} = x_i - (x_i - x_{i-1})
                       P(x_i) / (P(x_i) - P(x_{i-1})), where every P(x) is the
                       product of the LDL^T pivots.
  * ``verify``      -- the two sign checks of "Interval Verification": at x
                       truncated to a number of significant digits det(M - xI)
                       must be positive, one unit higher in the last digit it
                       must be negative.  Checked here through Sylvester's
                       inertia (count of negative pivots).
  * ``inverse_iteration`` -- not in the paper: one factorisation at a shift
                       sigma, then repeated solves; the eigenvalue estimate is
                       sigma + <v,v>/<v,A^{-1}v> from exact integer dots.

Readings of the paper taken here (the paper is silent on them):
  * Secant start: x1 = -2^{-ceil(K/4)}, x2 = 0 ("a small negative value");
    stop when |x_{i+1} - x_i| <= 10^-tol_digits * x_{i+1} (the paper stops
    when 15 digits are stable; 45 are used here); a step that does not
    shrink, a non-increasing iterate or a ratio P_i/P_{i-1} >= 1 means the
    precision K is exhausted (PrecisionError).
  * The ratio r = P(x_i)/P(x_{i-1}) is formed as the product over k of the
    pivot ratios, each floor-rounded to F = K/2 + 64 + bitlen(N) fractional
    bits and the running product truncated to F bits after every factor
    (ascending k).  x_{i+1} is then rounded RNE to K fractional bits.
  * Verification depth: 45 significant digits, lower point floored and upper
    point ceiled to K fractional bits.
  * Inverse iteration: v0 = all ones; v <- RNE(y 2^K / max|y|); stop when
    |lambda_k - lambda_{k-1}| <= 10^-tol_digits lambda_k.  The solve's
    intermediate vectors keep g = solve_guard_bits(N, K, X) extra fractional
    bits: half the bit length of the largest moment, rounded up to 64.
"""
from fractions import Fraction

from . import factor_from_moments, solve
from .moments import moments, rne_div


class PrecisionError(ArithmeticError):
    pass


class NotSPDError(ArithmeticError):
    pass


def to_fixed(x, K, mode="rne"):
    """Fraction -> integer with K fractional bits (rne / floor / ceil)."""
    x = Fraction(x)
    num, den = x.numerator << K, x.denominator
    if mode == "floor":
        return num // den
    if mode == "ceil":
        return -((-num) // den)
    return rne_div(num, den)


def pivot_ratio_fixed(d_new, d_old, F):
    """floor(2^F * prod_k d_new[k]/d_old[k]) with per-factor floor rounding
    and truncation of the running product to F fractional bits."""
    R = 1 << F
    for a, b in zip(d_new, d_old):
        if b == 0:
            raise NotSPDError("zero pivot")
        t = (a << F) // b
        R = (R * t) >> F
    return R


class _Evaluator:
    """P(x) through the pivots of the fixed-point LDL^T of M - xI; counts the
    factorisations."""

    def __init__(self, N, K, X, threads):
        self.N, self.K, self.X, self.threads = N, K, X, threads
        self.count = 0

    def __call__(self, x):
        f = factor_from_moments(self.X, self.N, self.K, x, threads=self.threads)
        self.count += 1
        if f.status != 0:
            return None, f
        return f.pivots(), f


def _secant_point(xa, xb, R, ONE):
    """xb - (xb - xa) r / (r - 1) with r = R / ONE, rounded RNE to the grid of
    xa and xb (K fractional bits)."""
    return rne_div(xb * (R - ONE) - (xb - xa) * R, R - ONE)


def _ratio_bits(N, K):
    """Fractional bits F of the pivot-product ratios."""
    return K // 2 + 64 + N.bit_length()


def secant(N, beta, K, tol_digits=45, max_iter=200, X=None, threads=0, trace=None):
    """Smallest eigenvalue by the Secant iteration; returns (Fraction, info).

    Phase 1 is the paper's iteration from the left.  If rounding makes an
    iterate land at or beyond the computed root (some pivot <= 0, which the
    exact iteration never does), the last two points bracket the root and
    phase 2 continues with the same secant formula on the bracket (Illinois
    variant of regula falsi) until the bracket is below the tolerance; the
    returned value is the bracket's lower end (a point with P > 0)."""
    X = moments(N, beta, K) if X is None else X
    F = _ratio_bits(N, K)
    ONE = 1 << F
    q = -(-K // 4)
    tol = Fraction(1, 10 ** tol_digits)
    evaluate = _Evaluator(N, K, X, threads)

    xs = [-(1 << (K - q)), 0]
    piv = []
    for x in xs:
        d, f = evaluate(x)
        if d is None or f.first_nonpos >= 0:
            raise NotSPDError("start point not left of lambda_1")
        piv.append(d)
    prev_step = None
    for it in range(max_iter):
        x0, x1 = xs[-2], xs[-1]
        R = pivot_ratio_fixed(piv[-1], piv[-2], F)
        if R >= ONE:
            raise PrecisionError("ratio >= 1: precision exhausted")
        x2 = _secant_point(x0, x1, R, ONE)
        step = x2 - x1
        if trace is not None:
            trace.append(("secant", x2, R))
        if step <= 0:
            raise PrecisionError("non-increasing iterate")
        if prev_step is not None and step >= prev_step and it > 2:
            raise PrecisionError("step did not shrink")
        prev_step = step
        if Fraction(step) <= tol * x2:
            return Fraction(x2, 1 << K), {"factorizations": evaluate.count, "iterations": it + 1}
        d, f = evaluate(x2)
        if d is not None and f.first_nonpos < 0:
            xs.append(x2)
            piv.append(d)
            continue
        # crossed the computed root: bracket [x1, x2]
        return _bracket(evaluate, x1, piv[-1], x2, d, F, K, tol, max_iter - it, trace)
    raise PrecisionError("no convergence")


def bracket_root(N, beta, K, a, b, tol_digits=45, max_iter=200, X=None, threads=0, trace=None):
    """The bracketing phase of the root finder on its own, from a bracket
    [a, b] of fixed-point shifts (K fractional bits) with P(a) > 0 >= P(b):
    Illinois regula falsi until b - a <= 10^-tol_digits a; returns
    (Fraction(a, 2^K), info) like secant()."""
    X = moments(N, beta, K) if X is None else X
    evaluate = _Evaluator(N, K, X, threads)
    da, fa = evaluate(a)
    if da is None or fa.first_nonpos >= 0:
        raise NotSPDError("lower end not left of lambda_1")
    db, fb = evaluate(b)
    if db is not None and fb.first_nonpos < 0:
        raise ValueError("upper end not right of lambda_1")
    return _bracket(evaluate, a, da, b, db, _ratio_bits(N, K), K, Fraction(1, 10 ** tol_digits),
                    max_iter, trace)


def _bracket(evaluate, a, da, b, db, F, K, tol, budget, trace):
    """Illinois regula falsi on [a, b] with P(a) > 0 >= P(b); P known only
    through pivot lists (db may be None when a zero pivot stopped the
    factorisation, then the midpoint is used).  When the same end survives
    two steps in a row, the function value kept for the other end is halved
    (once more for every further step on that side), which restores
    superlinear convergence where plain regula falsi would keep one end
    fixed."""
    ONE = 1 << F
    scale_a = scale_b = 0       # Illinois halvings applied to P(a), P(b)
    side = 0
    for it in range(budget):
        if Fraction(b - a) <= tol * a:
            return Fraction(a, 1 << K), {"factorizations": evaluate.count, "iterations": it,
                                         "bracketed": True}
        c = None
        if db is not None:
            R = pivot_ratio_fixed(db, da, F)            # P(b)/P(a) <= 0
            R = (R >> scale_b) << scale_a if scale_b <= scale_a else R >> (scale_b - scale_a)
            if R != ONE:
                c = _secant_point(a, b, R, ONE)
        if c is None or c <= a or c >= b:
            c = (a + b) // 2
        if trace is not None:
            trace.append(("bracket", c, a, b, scale_a, scale_b))
        dc, f = evaluate(c)
        if dc is not None and f.first_nonpos < 0:
            a, da = c, dc
            scale_a = 0
            if side == -1:
                scale_b += 1
            side = -1
        else:
            b, db = c, dc
            scale_b = 0
            if side == 1:
                scale_a += 1
            side = 1
    raise PrecisionError("bracketing did not converge")


def inertia(N, K, X, x_fixed, threads=0):
    """Number of negative pivots of M - xI and the first non-positive index."""
    f = factor_from_moments(X, N, K, x_fixed, threads=threads)
    return f.n_negative, f.first_nonpos


def truncate_digits(lam, digits):
    """(D, e) with lam truncated to `digits` significant digits = D * 10^e."""
    lam = Fraction(lam)
    if lam <= 0:
        raise ValueError("positive value expected")
    # find e with 10^(digits-1) <= lam / 10^e < 10^digits
    e = len(str(lam.numerator // lam.denominator)) - digits if lam >= 1 else 0
    while True:
        D = (lam / (Fraction(10) ** e)).__floor__()
        if D >= 10 ** digits:
            e += 1
        elif D < 10 ** (digits - 1):
            e -= 1
        else:
            return D, e


def verify(N, beta, K, lam, digits=45, X=None, threads=0):
    """Sign/inertia bracket around lam: 0 negative pivots at the truncated
    value, exactly one at one unit higher in the last digit."""
    X = moments(N, beta, K) if X is None else X
    D, e = truncate_digits(lam, digits)
    lo = Fraction(D) * Fraction(10) ** e
    hi = Fraction(D + 1) * Fraction(10) ** e
    n_lo, _ = inertia(N, K, X, to_fixed(lo, K, "floor"), threads)
    n_hi, _ = inertia(N, K, X, to_fixed(hi, K, "ceil"), threads)
    return n_lo == 0 and n_hi == 1, (n_lo, n_hi, D, e)


def normalize_inf(y, K):
    """v = RNE(y 2^K / max|y|)."""
    m = max(abs(t) for t in y)
    if m == 0:
        raise ArithmeticError("zero vector")
    return [rne_div(t << K, m) for t in y]


def solve_guard_bits(N, K, X):
    """Guard bits of the solve: ceil(log2(mu_max) / 2) rounded up to 64."""
    top = max(0, X[2 * N - 2].bit_length() - K)
    return 64 * ((top // 2 + 63) // 64)


def inverse_iteration(N, beta, K, sigma_fixed=0, tol_digits=45, max_iter=200, X=None,
                      threads=0, trace=None, guard=None):
    """Smallest eigenvalue by inverse iteration with one factorisation of
    M - sigma I; returns (Fraction, info)."""
    X = moments(N, beta, K) if X is None else X
    g = solve_guard_bits(N, K, X) if guard is None else guard
    f = factor_from_moments(X, N, K, sigma_fixed, threads=threads)
    if f.first_nonpos >= 0:
        raise NotSPDError("shift not below lambda_1 (pivot %d)" % f.first_nonpos)
    sigma = Fraction(sigma_fixed, 1 << K)
    v = [1 << K] * N
    lam_prev = None
    tol = Fraction(1, 10 ** tol_digits)
    for it in range(max_iter):
        y = solve(f, v, 3, g)                     # K + g fractional bits
        vy = sum(a * b for a, b in zip(v, y))     # 2K + g fractional bits
        vv = sum(a * a for a in v)                # 2K fractional bits
        if vy <= 0:
            raise PrecisionError("non-positive Rayleigh quotient")
        lam = sigma + Fraction(vv << g, vy)
        if trace is not None:
            trace.append((v, y, vv, vy))
        if lam_prev is not None and abs(lam - lam_prev) <= tol * lam:
            return lam, {"factorizations": 1, "solves": it + 1, "guard": g}
        lam_prev = lam
        v = normalize_inf(y, K)
    raise PrecisionError("inverse iteration did not converge")


def rel_digits(a, b):
    """Number of agreeing significant decimal digits of two positive values."""
    a, b = Fraction(a), Fraction(b)
    if a == b:
        return 1e9
    import math
    r = abs(a - b) / abs(b)
    return -math.log10(r.numerator) + math.log10(r.denominator)
