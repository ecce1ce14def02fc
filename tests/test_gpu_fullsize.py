"""GPU parity at full size: the N=200 (beta=7/4, K=2048) and N=500 (beta in
{1, 2, 3/2, 1/2}, K=6144) factorisations, compared column by column with
SHA-256 digests of the oracle's C and L digits (tests/golden/factor_digests.json,
written by tests/golden/make_factor_digests.py, which calls only the oracle)."""
import hashlib
import json
import os

import pytest

from tests.golden.canon import canon_bytes, column_digest
from tests.gpu_util import log

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden", "factor_digests.json")


def _db():
    return json.load(open(GOLD)) if os.path.exists(GOLD) else {}


@pytest.mark.parametrize("name,la", [("N200_b7_4_K2048", -1), ("N500_b1_K6144", -1), ("N500_b2_K6144", -1),
                                     ("N500_b3_2_K6144", -1), ("N500_b1_2_K6144", -1),
                                     ("N200_b7_4_K2048", 0), ("N500_b1_K6144", 2), ("N500_b1_2_K6144", 2)])
def test_fullsize_digests(hk, name, la):
    """la: the look-ahead mode (-1: the one chosen by size)."""
    db = _db()
    if name not in db:
        pytest.skip("digest not generated")
    g = db[name]
    N, beta, K = g["N"], tuple(g["beta"]), g["K"]
    log("full-size parity %s look-ahead %d" % (name, la))
    m = hk.Matrix(N, beta, K)
    m.set_lookahead(la)
    m.factor(0)
    bad = []
    step = 50
    for c0 in range(0, N, step):
        c1 = min(N, c0 + step)
        Cs = m.columns_C(c0, c1)
        Ls = m.columns_L(c0, min(c1, N - 1))
        for pc in range(c0, c1):
            Lc = Ls[pc - c0] if pc < N - 1 else []
            if column_digest(Cs[pc - c0], Lc) != g["columns"][pc]:
                bad.append(pc)
    assert bad == []
    assert hashlib.sha256(canon_bytes(m.pivots())).hexdigest() == g["pivots"]
    assert m.limb_macs() == g["limb_macs"]
