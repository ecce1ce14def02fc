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


def test_autotune_writes_cache(hk, tmp_path):
    insts = [(24, (1, 1), 384), (30, (7, 4), 512)]
    path = str(tmp_path / "tune.txt")
    b, la = hk.autotune(insts, cache_path=path)
    assert b in (1, 2, 4, 8, 16) and la in (0, 1, 2)
    txt = open(path).read()
    assert "panel=%d la=%d" % (b, la) in txt
