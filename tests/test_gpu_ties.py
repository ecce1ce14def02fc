"""GPU parity at the rounding rule's ties: shifts built so that the h-bit
rounding of C ("The LDL^T Determinant Algorithm": the extracted column) and
of the quotient CDivDiag land exactly half-way (tests/tie_cases.py explains
each construction).  Every digit of C, L and d is compared with the oracle,
whose ties-to-even at these same inputs is pinned against exact rational
arithmetic in test_oracle_ldl.py.  The cases cover the three finalisation
forms (2 or 8 digits a lane in registers, and through LDS), short and long
quotients, both schedules (separate update and finalise/divide launches,
and one launch per column), and a negative tie at the last pivot."""
from fractions import Fraction

import pytest

import oracle
from oracle.moments import moments
from tests.gpu_util import log
from tests.test_gpu_factor import compare
from tests.tie_cases import (beta1_negative_last_pivot_shift, beta1_pivot_tie_shift, general_tie_shift,
                             is_half)

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("la", [0, 2])
@pytest.mark.parametrize("N,K,m", [(40, 512, 1), (40, 512, 3), (12, 8192, 1), (6, 16640, 3)])
def test_beta1_pivot_ties(hk, N, K, m, la):
    h = K // 2
    xf = beta1_pivot_tie_shift(K, m)
    assert is_half(Fraction((1 << K) - xf, 1 << h))
    log("pivot ties beta=1 N=%d K=%d x_fix=%d*2^(h-1) look-ahead %d" % (N, K, m, la))
    X = moments(N, (1, 1), K)
    of = oracle.factor_from_moments(X, N, K, xf)
    hm = hk.Matrix(N, (1, 1), K)
    hm.set_panel(3)
    hm.set_lookahead(la)
    st, nneg, fb = hm.factor(xf)
    assert (nneg, fb) == (0, -1)
    compare(hm, of, N)


@pytest.mark.parametrize("la", [0, 2])
@pytest.mark.parametrize("N,beta,K,D,e", [(70, (3, 2), 640, 1, 0), (70, (3, 2), 640, 1, 1),
                                          (70, (3, 2), 640, 1, 3), (70, (5, 3), 640, 3, 0),
                                          (40, (2, 7), 1024, 5, 0), (20, (3, 2), 8192, 1, 0)])
def test_division_ties(hk, N, beta, K, D, e, la):
    h = K // 2
    X = moments(N, beta, K)
    xf = general_tie_shift(X[0], K, D, e << (h - 1) if e else 0)
    of = oracle.factor_from_moments(X, N, K, xf)
    C0 = of.column_C(0)
    ties = sum(is_half(Fraction(c << h, C0[0])) for c in C0[1:])
    log("division ties N=%d beta=%s K=%d D=%d e=%d: %d tied quotients, look-ahead %d"
        % (N, beta, K, D, e, ties, la))
    if e < 3:
        assert ties >= 1
    hm = hk.Matrix(N, beta, K)
    hm.set_panel(4)
    hm.set_lookahead(la)
    hm.factor(xf)
    compare(hm, of, N)


@pytest.mark.parametrize("la", [0, 2])
def test_negative_last_pivot_tie(hk, la):
    N, K = 2, 512
    X = moments(N, (1, 1), K)

    def piv(xf):
        return oracle.factor_from_moments(X, N, K, xf).pivots()
    xf = beta1_negative_last_pivot_shift(K, piv)
    of = oracle.factor_from_moments(X, N, K, xf)
    log("negative last-pivot tie N=2 K=512 look-ahead %d" % la)
    hm = hk.Matrix(N, (1, 1), K)
    hm.set_lookahead(la)
    st, nneg, fb = hm.factor(xf, inertia_mode=1)
    assert st == 0 and nneg == 1
    compare(hm, of, N)
    assert hm.pivots()[1] < 0
