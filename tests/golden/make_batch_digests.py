"""Writes tests/golden/batch_digests.json: per-column SHA-256 digests of the
oracle's fixed-point LDL^T factors (C and L of every column, and the pivots)
for a seeded batch of uneven instances shaped like the batched workload
(N uniform in [50, 400], beta = p/q with p, q uniform in 1..8 and
1/2 <= beta <= 3, K = 1024 bits at N = 50 rising linearly to 8192 at
N = 400 in whole 64-bit words), plus the largest such instance
(N = 400, beta = 3/2, K = 8192).  Calls only the oracle.  Run from the
repository root:
    python tests/golden/make_batch_digests.py
"""
import hashlib
import json
import math
import os
import random
import sys
import time
from fractions import Fraction

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from oracle.moments import moments  # noqa: E402
from tests.golden.canon import canon_bytes, column_digest  # noqa: E402

SEED = 9020852
COUNT = 9


def batch_instances(n=COUNT, seed=SEED):
    rng = random.Random(seed)
    out = []
    while len(out) < n:
        N = rng.randint(50, 400)
        p, q = rng.randint(1, 8), rng.randint(1, 8)
        b = Fraction(p, q)
        if Fraction(1, 2) <= b <= 3:
            K = 64 * math.ceil((1024 + 7168 * (N - 50) / 350) / 64)
            out.append((N, (b.numerator, b.denominator), K))
    out.append((400, (3, 2), 8192))
    return out


def main():
    path = os.path.join(HERE, "batch_digests.json")
    insts = []
    for N, beta, K in batch_instances():
        t = time.time()
        X = moments(N, beta, K)
        f = oracle.factor_from_moments(X, N, K, 0)
        cols = [column_digest(f.column_C(pc), f.column_L(pc)) for pc in range(N)]
        insts.append({"N": N, "beta": list(beta), "K": K, "shift": 0, "columns": cols,
                      "pivots": hashlib.sha256(canon_bytes(f.pivots())).hexdigest(),
                      "limb_macs": f.limb_macs})
        print(N, beta, K, "%.1f s" % (time.time() - t), flush=True)
    json.dump({"seed": SEED, "source": "oracle.factor_from_moments at x = 0", "instances": insts},
              open(path, "w"), indent=0)


if __name__ == "__main__":
    main()
