"""What the trained precision network gains over the method without it, on
equal drivers and at an equal standard (not in the paper).  On a seeded
held-out set of instances (a seed the training pairs never used):

  plain   : batched inverse iteration from sigma = 0 at the plain precision
            (1024 bits at N = 50 rising to 8192 at N = 400), then the inertia
            bracket at 40 digits;
  learned : the network's proposed precision b and shift sigma, batched
            inverse iteration at b and 1.25 b, accepted on agreement to
            1e-40, then the same inertia bracket at 40 digits in the accepted
            precision.

Every instance must be accepted, verified and agree with the plain value to
1e-40; the learned form's update work (limb MACs from the cost model
(N^3 - N)/6 (K/64 + 0.0088 log2 mu_{2N-2})^2 per factorisation, with the
factorisations each form actually took) must be below the plain form's.
Counts, not wall time, decide; the two times are logged."""
import math
import time
from fractions import Fraction

import pytest

from tests.gpu_util import log

pytestmark = pytest.mark.gpu


def parse_dec(s):
    m, e = s.split("e")
    return Fraction(m) * Fraction(10) ** int(e)


def work_model(N, beta, K):
    p, q = beta
    log2_mu = (math.lgamma(q * (2 * N - 1) / p) + math.log(q / p)) / math.log(2)
    return (N ** 3 - N) / 6 * (K / 64 + 0.0088 * log2_mu) ** 2


def test_learned_gain_on_equal_drivers(hk):
    import torch
    from paper_0902_0852_amd import learned
    model = learned.load_model()
    insts = learned.sample_instances(8, 20261203, 80, 240)
    plain = [(N, b, learned.plain_bits(N)) for N, b in insts]
    log("learned gain, %d held-out instances, N in [80, 240]" % len(plain))
    torch.cuda.synchronize()
    t0 = time.time()
    res_p, rep_p = hk.eig_batched(plain, digits=40, method=hk.HK_INVERSE)
    torch.cuda.synchronize()
    t_plain = time.time() - t0
    t0 = time.time()
    res_l, rep_l, bits, lns = learned.smallest_eig_learned(model, plain, digits=40)
    ok = hk.bracket_batched([(N, b, r["bits_used"]) for (N, b, _), r in zip(plain, res_l)],
                            [r["lambda_dec"] for r in res_l], digits=40)
    torch.cuda.synchronize()
    t_learned = time.time() - t0
    w_plain = w_learned = 0.0
    for (N, b, K), (st, dec, ver, nf), lam_p, r, good in zip(plain, res_p, rep_p["lambda"], res_l, ok):
        assert st == 0 and ver == 1, (N, b, K)
        assert r["status"] == 0 and r["path"] == 1, (N, b, r)          # accepted, no fallback
        assert good, (N, b, r["bits_used"])                            # verified at 40 digits
        # the binary values of both forms (the decimal strings are truncated)
        a, c = lam_p, r["lambda"]
        assert a > 0 and abs(a - c) <= a * Fraction(1, 10 ** 40), (N, b, dec, r["lambda_dec"])
        w_plain += nf * work_model(N, b, K)
        # the learned form's factorisations: its own (b, 1.25 b, any shift
        # halvings) at their precisions are at most the accepted one's, plus
        # the bracket's two at the accepted precision
        w_learned += (r["factorizations"] + 2) * work_model(N, b, r["bits_used"])
    log("plain %.2f s, learned %.2f s (incl. bracket); modelled work plain %.3e, learned %.3e limb-MACs; "
        "mean bits plain %.0f, proposed %.0f, used %.0f"
        % (t_plain, t_learned, w_plain, w_learned, sum(k for _, _, k in plain) / len(plain),
           sum(bits) / len(bits), sum(r["bits_used"] for r in res_l) / len(res_l)))
    assert w_learned < w_plain
