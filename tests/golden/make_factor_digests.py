"""Writes tests/golden/factor_digests.json: per-column SHA-256 digests of the
oracle's fixed-point LDL^T factors (C and L of every column) at full size, for
the GPU parity tests.  Calls only the oracle.  Run from the repository root:
    python tests/golden/make_factor_digests.py [config ...]
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from oracle.moments import moments  # noqa: E402
from tests.golden.canon import canon_bytes, column_digest  # noqa: E402
import hashlib  # noqa: E402

CONFIGS = {
    "N200_b7_4_K2048": (200, (7, 4), 2048),
    "N500_b1_K6144": (500, (1, 1), 6144),
    "N500_b2_K6144": (500, (2, 1), 6144),
    "N500_b3_2_K6144": (500, (3, 2), 6144),
    "N500_b1_2_K6144": (500, (1, 2), 6144),
}


def main(names):
    path = os.path.join(HERE, "factor_digests.json")
    db = json.load(open(path)) if os.path.exists(path) else {}
    for name in names:
        N, beta, K = CONFIGS[name]
        t = time.time()
        X = moments(N, beta, K)
        f = oracle.factor_from_moments(X, N, K, 0)
        cols = []
        for pc in range(N):
            C = f.column_C(pc)
            L = f.column_L(pc)
            cols.append(column_digest(C, L))
        piv = hashlib.sha256(canon_bytes(f.pivots())).hexdigest()
        db[name] = {"N": N, "beta": list(beta), "K": K, "shift": 0, "columns": cols,
                    "pivots": piv, "limb_macs": f.limb_macs,
                    "source": "oracle.factor_from_moments at x = 0"}
        print(name, "%.1f s" % (time.time() - t), flush=True)
        json.dump(db, open(path, "w"), indent=0)


if __name__ == "__main__":
    main(sys.argv[1:] or list(CONFIGS))
