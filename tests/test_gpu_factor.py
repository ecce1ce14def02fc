"""GPU parity: every digit of C, L and the pivots from the HIP factorisation
equals the oracle's, element by element, on seeded configurations (sizes that
span several 64-row tiles and 16-digit blocks with ragged tails), at the small
config (N=32, beta=1, K=512: also the closed forms) and the N=200, beta=7/4,
K=2048 config, for several update ranks (schedule invariance)."""
import math
import random

import pytest

import oracle
from oracle.moments import moments
from tests.gpu_util import log

pytestmark = pytest.mark.gpu


def compare(hm, of, N):
    gC, oC = hm.columns_C(), of.all_C()
    for pc in range(N):
        assert gC[pc] == oC[pc], ("C", pc)
    gL, oL = hm.columns_L(), of.all_L()
    for pc in range(N - 1):
        assert gL[pc] == oL[pc], ("L", pc)
    assert hm.pivots() == of.pivots()


def test_config1_closed_forms(hk):
    N, K = 32, 512
    h = K // 2
    log("config1 N=32 beta=1 K=512")
    m = hk.Matrix(N, (1, 1), K)
    st, nneg, fb = m.factor(0)
    assert (nneg, fb) == (0, -1)
    C, L = m.columns_C(), m.columns_L()
    for pc in range(N):
        assert C[pc] == [(math.factorial(r) ** 2 // math.factorial(r - pc)) << h for r in range(pc, N)]
    for pc in range(N - 1):
        assert L[pc] == [(math.comb(r, pc) * math.factorial(r) // math.factorial(pc)) << h
                         for r in range(pc + 1, N)]
    det = math.prod(m.pivots())
    assert det == math.prod(math.factorial(k) ** 2 for k in range(N)) << (h * N)
    assert m.limb_macs() == oracle.factor(N, (1, 1), K).limb_macs


CASES = [
    # (N, beta, K, shift numerator xn, panel); shift x = xn * 2^-(K/2), far
    # below lambda_1 for these sizes (negative values move the other way)
    (5, (7, 4), 128, 0, 1),
    (33, (7, 4), 384, -3, 4),
    (70, (3, 2), 640, 11, 3),
    (65, (1, 2), 512, 0, 4),
    (97, (5, 3), 768, 7, 8),
    (40, (2, 7), 320, -1, 2),
    (130, (1, 1), 1024, 5, 4),
]


@pytest.mark.parametrize("la", [0, 2])
@pytest.mark.parametrize("N,beta,K,xn,panel", CASES)
def test_parity_vs_oracle(hk, N, beta, K, xn, panel, la):
    log("parity N=%d beta=%s K=%d x=%d*2^-(K/2) panel=%d look-ahead %d" % (N, beta, K, xn, panel, la))
    X = moments(N, beta, K)
    xf = xn << (K - K // 2)
    of = oracle.factor_from_moments(X, N, K, xf)
    m = hk.Matrix(N, beta, K)
    m.set_panel(panel)
    m.set_lookahead(la)
    st, nneg, fb = m.factor(xf)
    compare(m, of, N)


@pytest.mark.parametrize("panel", [1, 4, 16])
def test_schedule_invariance(hk, panel):
    # the update is exact, so every rank gives the same digits
    N, beta, K = 80, (7, 4), 896
    log("schedule panel=%d" % panel)
    m = hk.Matrix(N, beta, K)
    m.set_panel(panel)
    m.factor(0)
    of = oracle.factor(N, beta, K, 0)
    compare(m, of, N)


def test_config2_full_parity(hk):
    N, beta, K = 200, (7, 4), 2048
    log("config2 N=200 beta=7/4 K=2048")
    X = moments(N, beta, K)
    of = oracle.factor_from_moments(X, N, K, 0)
    m = hk.Matrix(N, beta, K)
    m.factor(0)
    compare(m, of, N)
    assert m.limb_macs() == of.limb_macs


def test_shift_above_lambda_reports_not_spd(hk):
    # x far above lambda_1: a pivot turns negative before the last column
    N, beta, K = 40, (3, 2), 512
    m = hk.Matrix(N, beta, K)
    st, nneg, fb = m.factor(1 << K, inertia_mode=0, raise_on_error=False)
    of = oracle.factor(N, beta, K, 1 << K)
    assert st == 2 and fb == of.first_nonpos and 0 <= fb < N - 1


def test_inertia_last_pivot(hk):
    # just above lambda_1: only the last pivot is negative
    from oracle.drivers import inverse_iteration, to_fixed
    from fractions import Fraction
    N, beta, K = 32, (1, 1), 512
    lam, _ = inverse_iteration(N, beta, K)
    m = hk.Matrix(N, beta, K)
    xs = to_fixed(lam * (1 + Fraction(1, 10 ** 30)), K, "ceil")
    st, nneg, fb = m.factor(xs, inertia_mode=1)
    assert st == 0 and nneg == 1 and fb == N - 1
    of = oracle.factor(N, beta, K, xs)
    assert m.pivots() == of.pivots()
    st, nneg, fb = m.factor(xs, inertia_mode=0, raise_on_error=False)
    assert st == 2 and fb == N - 1


def test_graph_replays_equal_eager_and_oracle(hk):
    """hk_factor replays one captured HIP graph per panel width when per-launch
    timing is off: several replays at alternating shifts, with eager (timed,
    stream-launched) factorisations and host work in between, each equal to
    the oracle digit for digit."""
    N, beta, K = 70, (3, 2), 640
    h = K // 2
    X = moments(N, beta, K)
    shifts = [5 << (K - h), 0, 5 << (K - h), 17 << (K - h)]
    ref = {x: oracle.factor_from_moments(X, N, K, x) for x in set(shifts)}
    m = hk.Matrix(N, beta, K)
    for rep, x in enumerate(shifts):
        for timing in (0, 1, 0):
            log("graph replay %d timing %d shift %d" % (rep, timing, x))
            m.set_timing(timing)
            m.factor(x)
            compare(m, ref[x], N)
    m.set_timing(0)
    m.set_panel(2)          # recapture at another width
    m.factor(shifts[0])
    compare(m, ref[shifts[0]], N)


@pytest.mark.parametrize("panel", [1, 3, 8])
def test_lookahead_modes_equal_oracle(hk, panel):
    """The look-ahead schedules (1: next panel's columns first, the rest of
    the trailing update on a second stream; 2: one launch per column with the
    previous column's update inside it) give the same digits as one trailing
    update per panel, eager and through graph replays."""
    N, beta, K = 97, (5, 3), 768
    X = moments(N, beta, K)
    ref = oracle.factor_from_moments(X, N, K, 0)
    m = hk.Matrix(N, beta, K)
    m.set_panel(panel)
    for la in (1, 0, 2, 1, 2):
        for timing in (1, 0, 0):
            log("look-ahead %d panel %d timing %d" % (la, panel, timing))
            m.set_lookahead(la)
            m.set_timing(timing)
            m.factor(0)
            compare(m, ref, N)


EDGE = [
    # degenerate and boundary sizes: one entry, two entries, one full tile,
    # one tile plus one row, the smallest precision
    (1, (1, 1), 64, 0, 4),
    (1, (3, 2), 128, 1, 1),
    (2, (1, 2), 96, 0, 2),
    (64, (2, 1), 64 * 9, 0, 4),
    (65, (1, 1), 640, 0, 3),
    (12, (1, 1), 64, 0, 1),
]


@pytest.mark.parametrize("la", [0, 2])
@pytest.mark.parametrize("N,beta,K,xn,panel", EDGE)
def test_edge_sizes_vs_oracle(hk, N, beta, K, xn, panel, la):
    log("edge N=%d beta=%s K=%d x=%d*2^-(K/2) panel=%d look-ahead %d" % (N, beta, K, xn, panel, la))
    X = moments(N, beta, K)
    xf = xn << (K - K // 2)
    of = oracle.factor_from_moments(X, N, K, xf)
    m = hk.Matrix(N, beta, K)
    m.set_panel(panel)
    m.set_lookahead(la)
    st, nneg, fb = m.factor(xf, inertia_mode=1, raise_on_error=False)
    assert (nneg, fb) == (of.n_negative, of.first_nonpos)
    if fb < 0 or fb == N - 1:
        compare(m, of, N)


@pytest.mark.parametrize("group,la", [(1, 0), (2, 1), (1, 1), (4, 0)])
def test_update_group_invariance(hk, group, la):
    # update items per workgroup change only the launch shape: every digit
    # still equals the oracle's
    N, beta, K, xn = 97, (5, 3), 768, 7
    log("update group %d look-ahead %d" % (group, la))
    X = moments(N, beta, K)
    xf = xn << (K - K // 2)
    of = oracle.factor_from_moments(X, N, K, xf)
    m = hk.Matrix(N, beta, K)
    m.set_panel(3)
    m.set_lookahead(la)
    m.set_update_group(group)
    m.factor(xf)
    compare(m, of, N)


@pytest.mark.parametrize("la", [0, 1])
def test_widest_entries_vs_oracle(hk, la):
    # entries of about 3800 digits: the finalise/divide launch's LDS (pivot,
    # this row's digits, two finalisation regions, then the division over the
    # dead finalisation regions) sits just under what a workgroup may hold
    N, beta, K = 16, (1, 1), 110000
    log("widest entries N=%d K=%d look-ahead %d" % (N, K, la))
    X = moments(N, beta, K)
    of = oracle.factor_from_moments(X, N, K, 0)
    m = hk.Matrix(N, beta, K)
    m.set_panel(4)
    m.set_lookahead(la)
    m.factor(0)
    assert m.info().max_col_digits > 3700
    compare(m, of, N)


def test_lds_limit_reported(hk):
    # the in-kernel look-ahead launch also holds the update's operands in LDS:
    # at these widths it does not fit, and the factorisation says so before
    # launching anything
    m = hk.Matrix(16, (1, 1), 110000)
    m.set_lookahead(2)
    with pytest.raises(hk.HKError, match="LDS"):
        m.factor(0)
    # the same matrix still factors in a mode that fits
    m.set_lookahead(0)
    m.factor(0)
    assert m.pivots()[0] > 0


@pytest.mark.parametrize("engine,la,panel", [(0, 0, 4), (1, 0, 4), (0, 1, 3), (1, 1, 2), (0, 0, 16)])
def test_update_engines_vs_oracle(hk, engine, la, panel):
    # the bulk update on the matrix cores (int8 byte-plane products) and on
    # the vector units: every digit equals the oracle's either way
    N, beta, K, xn = 150, (3, 2), 2048, 5
    log("update engine %d look-ahead %d panel %d" % (engine, la, panel))
    X = moments(N, beta, K)
    xf = xn << (K - K // 2)
    of = oracle.factor_from_moments(X, N, K, xf)
    m = hk.Matrix(N, beta, K)
    m.set_panel(panel)
    m.set_lookahead(la)
    m.set_update_engine(engine)
    assert m.info().update_engine == (1 if engine == hk.HK_UPDATE_MATRIX_CORES else 0)
    m.factor(xf)
    compare(m, of, N)


def test_matrix_core_update_wide_panel(hk):
    # a 16-column panel of 1040-digit columns: C's byte planes of the whole
    # panel no longer fit one workgroup's LDS, so the bulk update takes the
    # one-item-per-wavefront form of the matrix-core kernel
    N, beta, K = 64, (1, 2), 30000
    log("matrix-core update, wide panel N=%d K=%d" % (N, K))
    X = moments(N, beta, K)
    of = oracle.factor_from_moments(X, N, K, 0)
    m = hk.Matrix(N, beta, K)
    assert m.info().max_col_digits * 16 < 32704
    m.set_panel(16)
    m.set_lookahead(0)
    m.factor(0)
    assert m.info().update_engine == 1
    compare(m, of, N)
