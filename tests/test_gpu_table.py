"""GPU reproduction of the paper's table of smallest eigenvalues (section
'Numerical results', printed to 5 significant digits) at N = 300 and
N = 500 for all four beta, by the library's Secant driver with the inertia
bracket at 45 digits (tests/golden/paper_lambda_table.json).  The precisions
are the smallest K that the training pairs of the learned form put near these
sizes (the bits a 41-digit bracket needs), raised by a third to a half so
that the Secant iteration has room beyond the 45 digits it stops at."""
import json
import os
from fractions import Fraction

import pytest

from tests.gpu_util import log

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden", "paper_lambda_table.json")

# (row N, column, K)
CASES = [(300, 0, 3072), (300, 1, 2048), (300, 2, 2048), (300, 3, 2560),
         (500, 0, 4096), (500, 1, 3072), (500, 2, 4096), (500, 3, 5120)]


def parse_dec(s):
    m, e = (s.split("e") + ["0"])[:2]
    return Fraction(m) * Fraction(10) ** int(e)


@pytest.mark.parametrize("N,col,K", CASES)
def test_paper_lambda_table(hk, N, col, K):
    tab = json.load(open(GOLD))
    beta = tuple(tab["columns_beta"][col])
    ref = parse_dec(tab["rows"][str(N)][col])
    log("lambda table N=%d beta=%d/%d K=%d" % (N, beta[0], beta[1], K))
    dec, rep = hk.smallest_eig(N, beta, K, method=hk.HK_SECANT, digits=45, flags=hk.HK_FLAG_NO_WORK_COUNT)
    assert rep["verified"] == 1, dec
    lam = parse_dec(dec)
    # the paper prints 5 significant digits
    assert abs(lam - ref) <= ref * Fraction(51, 10 ** 6), (dec, str(ref))
    log("  lambda_1 = %s (paper %s), %d factorisations" % (dec, tab["rows"][str(N)][col], rep["factorizations"]))
