"""GPU batched form: instances of uneven (N, beta, K) factored together by the
instance-batched kernels replayed from one captured HIP graph.  Each
instance's lambda_1 matches its oracle value to 1e-40 with a verified bracket,
and equals, digit for digit, what the single-instance (eager) path returns."""
import random
from fractions import Fraction

import pytest

import oracle
from oracle.drivers import inverse_iteration, rel_digits
from tests.gpu_util import log

pytestmark = pytest.mark.gpu


def parse_dec(s):
    m, e = s.split("e")
    return Fraction(m) * Fraction(10) ** int(e)


def test_batched_lambda_matches_oracle(hk):
    insts = [(32, (1, 1), 512), (20, (7, 4), 640), (45, (3, 2), 768), (7, (2, 1), 512),
             (64, (1, 2), 1024), (33, (5, 3), 896)]
    log("batched lambda, %d instances" % len(insts))
    res, rep = hk.eig_batched(insts, digits=45, panel=4)
    assert rep["status"] == 0
    assert rep["graph_launches"] >= 3
    for (N, beta, K), (st, dec, ver, nf) in zip(insts, res):
        assert st == 0 and ver == 1, (N, beta, K, st)
        lam_o, _ = inverse_iteration(N, beta, K)
        assert rel_digits(parse_dec(dec), lam_o) > 40, (N, beta, K, dec)


def test_batched_equals_single_instance(hk):
    # the single-instance path agrees with the batched one instance by instance
    insts = [(25, (7, 4), 512), (40, (1, 1), 640)]
    res, rep = hk.eig_batched(insts, digits=45, panel=2)
    for (N, beta, K), (st, dec, ver, nf) in zip(insts, res):
        d1, r1 = hk.smallest_eig(N, beta, K, method=hk.HK_SECANT, digits=45)
        assert st == 0 and d1 == dec


def test_paired_factorisations_change_nothing(hk):
    # with the paired workspace the Secant's start points and the bracket's
    # ends go two to a launch sequence: two sequences fewer, identical results
    # (a Secant and an inverse-iteration mix, uneven sizes, look-ahead 1)
    insts = [(40, (1, 1), 640), (23, (7, 4), 512), (57, (3, 2), 768)]
    log("paired against unpaired batched factorisations, %d instances" % len(insts))
    for method in (hk.HK_SECANT, hk.HK_INVERSE):
        r1, d1 = hk.eig_batched(insts, digits=45, panel=3, method=method,
                                flags=hk.HK_FLAG_LOOKAHEAD_ON, paired=True)
        r0, d0 = hk.eig_batched(insts, digits=45, panel=3, method=method,
                                flags=hk.HK_FLAG_LOOKAHEAD_ON, paired=False)
        assert r1 == r0, (method, r1, r0)
        assert all(st == 0 and ver == 1 for st, _, ver, _ in r1)
        fewer = 2 if method == hk.HK_SECANT else 1
        assert d1["graph_launches"] == d0["graph_launches"] - fewer, (method, d1["graph_launches"],
                                                                      d0["graph_launches"])


def test_autotune_writes_cache(hk, tmp_path):
    insts = [(24, (1, 1), 384), (30, (7, 4), 512)]
    path = str(tmp_path / "tune.txt")
    b, la, g = hk.autotune(insts, cache_path=path)
    assert b in (1, 2, 4, 8, 16) and la in (0, 1, 2) and g in (1, 2, 4)
    txt = open(path).read()
    assert "panel=%d la=%d ipw=%d" % (b, la, g) in txt


# ---- factor parity of the batched path -------------------------------------
import hashlib  # noqa: E402
import json  # noqa: E402
import os  # noqa: E402

from oracle.moments import moments  # noqa: E402
from tests.golden.canon import canon_bytes, column_digest  # noqa: E402
from tests.test_gpu_factor import compare  # noqa: E402

BATCH_GOLD = os.path.join(os.path.dirname(__file__), "golden", "batch_digests.json")


@pytest.mark.parametrize("panel,la", [(3, 1), (3, 0), (1, 2)])
def test_batched_factors_equal_oracle_uneven(hk, panel, la):
    # uneven instances, shifts of both signs: every digit of every instance
    # against the oracle, under each schedule (second-stream look-ahead, none,
    # one launch per column)
    insts = [(40, (7, 4), 512), (97, (3, 2), 1024), (130, (1, 1), 1536), (70, (2, 7), 768), (5, (5, 3), 256)]
    shifts = [3 << 256, -(5 << 512), 0, 7 << 384, -(1 << 128)]
    log("batched factors, uneven, panel %d look-ahead %d" % (panel, la))
    b = hk.Batch(insts)
    b.set_schedule(panel, la)
    res = b.factor(shifts)
    for i, ((N, beta, K), xf) in enumerate(zip(insts, shifts)):
        assert res[i] == (0, 0, -1), (i, res[i])
        of = oracle.factor_from_moments(moments(N, beta, K), N, K, xf)
        compare(b.member(i), of, N)


@pytest.mark.parametrize("panel,la", [(2, 1), (1, 2)])
def test_batched_factors_match_golden_batch(hk, panel, la):
    # the seeded batch of ten uneven instances up to N = 400, K = 8192
    # (tests/golden/make_batch_digests.py, oracle only): per-column digests
    # of C and L, the pivots and the algorithmic work of every instance
    db = json.load(open(BATCH_GOLD))
    g = db["instances"]
    insts = [(x["N"], tuple(x["beta"]), x["K"]) for x in g]
    log("golden batch of %d, panel %d look-ahead %d" % (len(insts), panel, la))
    b = hk.Batch(insts)
    b.set_schedule(panel, la)
    res = b.factor()
    for i, x in enumerate(g):
        assert res[i] == (0, 0, -1), (i, res[i])
        m = b.member(i)
        N = x["N"]
        bad = []
        for c0 in range(0, N, 50):
            c1 = min(N, c0 + 50)
            Cs = m.columns_C(c0, c1)
            Ls = m.columns_L(c0, min(c1, N - 1))
            for pc in range(c0, c1):
                Lc = Ls[pc - c0] if pc < N - 1 else []
                if column_digest(Cs[pc - c0], Lc) != x["columns"][pc]:
                    bad.append(pc)
        assert bad == [], (i, bad[:5])
        assert hashlib.sha256(canon_bytes(m.pivots())).hexdigest() == x["pivots"]
        assert m.limb_macs() == x["limb_macs"]


def test_batched_workload_64_instances(hk):
    # the batched workload's shape: 64 seeded instances, N uniform in
    # [50, 400], beta = p/q (p, q in 1..8, 1/2 <= beta <= 3), K from 1024 at
    # N = 50 to 8192 at N = 400; every lambda_1 equals the single-instance
    # path's digit for digit, and the four smallest instances the oracle's
    # to 1e-40
    import math
    rng = random.Random(9020852)
    insts = []
    while len(insts) < 64:
        N = rng.randint(50, 400)
        p, q = rng.randint(1, 8), rng.randint(1, 8)
        b = Fraction(p, q)
        if Fraction(1, 2) <= b <= 3:
            insts.append((N, (b.numerator, b.denominator), 64 * math.ceil((1024 + 7168 * (N - 50) / 350) / 64)))
    log("batched workload: 64 instances, N %d..%d" % (min(i[0] for i in insts), max(i[0] for i in insts)))
    res, rep = hk.eig_batched(insts, digits=45)
    assert rep["status"] == 0
    for (N, beta, K), (st, dec, ver, nf) in zip(insts, res):
        assert st == 0 and ver == 1, (N, beta, K)
        d1, r1 = hk.smallest_eig(N, beta, K, method=hk.HK_SECANT, digits=45, flags=hk.HK_FLAG_NO_WORK_COUNT)
        assert d1 == dec, (N, beta, K, d1, dec)
    for N, beta, K in sorted(insts)[:4]:
        lam_o, _ = inverse_iteration(N, beta, K)
        i = insts.index((N, beta, K))
        assert rel_digits(parse_dec(res[i][1]), lam_o) > 40, (N, beta, K)
