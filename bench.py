"""Benchmark: smallest eigenvalue of the Hankel moment matrix on one MI355X.

One step = one pass of the whole hot path on one synthetic instance: moments
(Gamma at the working precision) -> LDL^T factorisations (expansion, panel,
trailing update) -> the eigenvalue iteration -> the inertia bracket at 45
digits, i.e. one verified lambda_1.  The default workload is N = 200,
beta = 7/4, K = 2048 fractional bits.

Printed value: algorithmic 32-bit limb MACs per second of the whole job (the
schoolbook count of every factorisation's trailing update, sum over updates
of ceil(bits(C)/32) * ceil(bits(L)/32), divided by the wall time of the timed
steps).  Also printed: lambda_1 solves/s, a roofline record for the kernel
that carries the update work (k_update, or k_column in look-ahead mode 2,
where each column's launch holds its update as well as the finalisation and
division of the column; achieved limb MACs/s from the start and end HIP
events that every such launch records on the library's stream, against one
32-bit multiply per lane per clock on 256 CUs at 2.4 GHz), and the CPU
oracle timed on the host cores.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--config c2]
"""
import argparse
import json
import os
import sys
import time

CONFIGS = {
    "c1": dict(N=32, beta=(1, 1), K=512, desc="N=32 beta=1 K=512"),
    "c2": dict(N=200, beta=(7, 4), K=2048, desc="N=200 beta=7/4 K=2048"),
    "c3b1": dict(N=500, beta=(1, 1), K=6144, desc="N=500 beta=1 K=6144"),
    "c3b2": dict(N=500, beta=(2, 1), K=6144, desc="N=500 beta=2 K=6144"),
    "c3b32": dict(N=500, beta=(3, 2), K=6144, desc="N=500 beta=3/2 K=6144"),
    "c3b12": dict(N=500, beta=(1, 2), K=6144, desc="N=500 beta=1/2 K=6144"),
    "c5": dict(N=1500, beta=(3, 2), K=24576, desc="N=1500 beta=3/2 K=24576"),
}
PEAK_INT_MUL = 256 * 64 * 2.4e9       # one 32x32 multiply per lane per clock
HBM_PEAK = 8.0e12
HERE = os.path.dirname(os.path.abspath(__file__))
PROFILE_TAG = {"c2": "N200_beta7-4_K2048", "c3b1": "N500_beta1_K6144"}


def measured_traffic(cfg_name, kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary of this workload, or None when there is none or the kernel
    source has changed since the counters were taken."""
    import hashlib
    import re
    tag = PROFILE_TAG.get(cfg_name)
    if tag is None:
        return None, None
    path = os.path.join(HERE, "profiles", "%s_%s_secant.txt" % (kernel, tag))
    try:
        txt = open(path).read()
    except OSError:
        return None, None
    src = open(os.path.join(HERE, "paper_0902_0852_amd", "csrc", "hk_kernels.hip"), "rb").read()
    m = re.search(r"sha256 ([0-9a-f]{16})", txt)
    t = re.search(r"traffic_bytes_per_launch=(\d+)", txt)
    if not m or not t or m.group(1) != hashlib.sha256(src).hexdigest()[:16]:
        return None, os.path.relpath(path, HERE)
    return int(t.group(1)), os.path.relpath(path, HERE)


def log(msg):
    sys.stderr.write(msg + "\n")
    sys.stderr.flush()


def cpu_baseline(cfg, method, budget_s=20.0):
    """The oracle (test infrastructure) on the same workload, bounded: full
    verified lambda_1 runs (iteration + the two bracket factorisations) until
    the budget is spent; work = factorisations x the limb MACs of one."""
    import oracle
    from oracle.drivers import inverse_iteration, secant, verify
    from oracle.moments import moments
    N, beta, K = cfg["N"], cfg["beta"], cfg["K"]
    X = moments(N, beta, K)                 # matrix generation excluded, as in the paper
    macs0 = oracle.factor_from_moments(X, N, K, 0).limb_macs
    t0 = time.time()
    nfact, n = 0, 0
    while True:
        if method == "secant":
            lam, info = secant(N, beta, K, X=X)
        else:
            lam, info = inverse_iteration(N, beta, K, X=X)
        ok, _ = verify(N, beta, K, lam, X=X)
        nfact += info["factorizations"] + 2
        n += 1
        if time.time() - t0 > budget_s / 2 or n >= 12:
            break
    dt = time.time() - t0
    return {"value": nfact * macs0 / dt, "unit": "limb-MAC/s", "cores": oracle.max_threads(),
            "kind": "oracle",
            "sample": "%d verified lambda_1 runs (%s driver, %d factorisations) of %s, "
                      "moments excluded, %.1f s" % (n, method, nfact, cfg["desc"], dt),
            "lambda_per_s": n / dt}


def learned_gain(args):
    """Batched + learned form against the batched plain form on the same
    held-out instances: lambda_1 instances per second at 1e-40 agreement."""
    import torch
    import paper_0902_0852_amd as hk
    from paper_0902_0852_amd import learned
    from fractions import Fraction
    model = learned.load_model(args.model) if args.model else learned.load_model()
    single = args.config == "c5"
    if single:
        # one large instance: the plain form is inverse iteration from 0 at the
        # fixed precision plus the inertia bracket (the faster plain driver)
        cfg = CONFIGS["c5"]
        insts = [(cfg["N"], cfg["beta"])]
        plain = [(cfg["N"], cfg["beta"], cfg["K"])]
    else:
        insts = learned.sample_instances(args.instances, args.seed, args.n_lo, args.n_hi)
        plain = [(N, b, learned.plain_bits(N)) for N, b in insts]
        # warm-up on a small batch of the same kind (graph capture, code load)
        hk.eig_batched(plain[:2], digits=45)
        learned.smallest_eig_learned(model, plain[:2])
    torch.cuda.synchronize()
    t0 = time.time()
    if single:
        N, beta, K = plain[0]
        dec, rep = hk.smallest_eig(N, beta, K, method=hk.HK_INVERSE, digits=45, flags=hk.HK_FLAG_NO_WORK_COUNT)
        res_p = [(rep["status"], dec, rep["verified"], rep["factorizations"])]
        log("plain: %s in %.1f s (%d factorisations, %d solves)" % (dec, time.time() - t0, rep["factorizations"],
                                                                    rep["solves"]))
    else:
        res_p, rep_p = hk.eig_batched(plain, digits=45, panel=args.panel)
    torch.cuda.synchronize()
    t_plain = time.time() - t0
    t0 = time.time()
    res_l, rep_l, bits, lns = learned.smallest_eig_learned(model, plain, panel=args.panel)
    torch.cuda.synchronize()
    t_learned = time.time() - t0

    def val(dec):
        m, e = dec.split("e")
        return Fraction(m) * Fraction(10) ** int(e)
    agree = 0
    for (st, dec, ver, nf), r in zip(res_p, res_l):
        if st == 0 and r["status"] == 0:
            a, b = val(dec), val(r["lambda_dec"])
            agree += abs(a - b) <= Fraction(1, 10 ** 40) * abs(a)
    n = len(insts)
    out = {
        "metric": "lambda_1 instances/s at 1e-40 agreement, batched + learned precision vs batched plain "
                  "fixed precision",
        "value": n / t_learned, "unit": "instances/s", "n_gpus": 1, "higher_is_better": True,
        "data": "synthetic", "dtype": "int32 (method), float32 (network)",
        "config": {"workload": ("N=1500 beta=3/2, plain: inverse iteration + bracket at 24576 bits" if single else
                                "%d held-out instances, seed %d, N uniform in [%d, %d], beta = p/q, p, q in 1..8, "
                                "beta in [1/2, 3]; plain: batched Secant + bracket at 1024 + 20.48 (N - 50) bits" %
                                (n, args.seed, args.n_lo, args.n_hi))},
        "lambda_plain": res_p[0][1] if single else None,
        "lambda_learned": res_l[0]["lambda_dec"] if single else None,
        "plain_instances_per_s": n / t_plain, "speedup": t_plain / t_learned,
        "t_plain_s": t_plain, "t_learned_s": t_learned,
        "accepted_learned": sum(r["path"] == 1 for r in res_l), "fallback_plain": sum(r["path"] == 0 for r in res_l),
        "agree_1e-40": agree,
        "mean_bits_plain": sum(k for _, _, k in plain) / n, "mean_bits_proposed": sum(bits) / n,
        "mean_bits_used": sum(r["bits_used"] for r in res_l) / n,
        "factorizations_plain": sum(nf for _, _, _, nf in res_p),
        "factorizations_learned": sum(r["factorizations"] for r in res_l),
        "solves_learned": sum(r["solves"] for r in res_l),
        "panel": args.panel,
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c2", choices=sorted(CONFIGS))
    ap.add_argument("--method", default="secant", choices=["secant", "inverse"])
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--mode", default="plain", choices=["plain", "learned"],
                    help="learned: batched + learned form against the batched plain form")
    ap.add_argument("--model", default=None, help="network file (default: the package's trained one)")
    ap.add_argument("--instances", type=int, default=64)
    ap.add_argument("--seed", type=int, default=4242)
    ap.add_argument("--n-lo", type=int, default=50)
    ap.add_argument("--n-hi", type=int, default=400)
    ap.add_argument("--panel", type=int, default=0, help="panel width (0: tuned here / tuned or 4 in learned mode)")
    ap.add_argument("--lookahead", type=int, default=-1, choices=[-1, 0, 1, 2],
                    help="with --panel: look-ahead mode 0 none, 1 second stream, 2 one launch per column "
                         "(-1: chosen by size)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the method has no multi-GPU path "
              "(independent instances would shard one per GPU).", file=sys.stderr)
        sys.exit(2)
    if args.mode == "learned":
        learned_gain(args)
        return
    import torch
    import paper_0902_0852_amd as hk
    cfg = CONFIGS[args.config]
    N, beta, K = cfg["N"], cfg["beta"], cfg["K"]
    method = hk.HK_SECANT if args.method == "secant" else hk.HK_INVERSE
    ws = torch.empty(hk.workspace_bytes(N, beta, K), dtype=torch.uint8, device="cuda")
    # untimed: the panel width tuned for this shape (hk_autotune; the library
    # reads it back from the cache named by HK_TUNE_CACHE)
    import tempfile
    tune_path = os.path.join(tempfile.gettempdir(), "hk_tune_%d.txt" % os.getpid())
    os.environ["HK_TUNE_CACHE"] = tune_path
    if args.panel > 0:
        panel, la = args.panel, args.lookahead
        if la < 0:   # the mode the library picks for this size
            m = hk.Matrix(N, beta, K)
            m.set_panel(panel)
            la = m.info().lookahead
            del m
        log("panel width %d, look-ahead %d (given)" % (panel, la))
    else:
        panel, la = hk.autotune([(N, beta, K)], cache_path=tune_path)
        log("tuned panel width %d, look-ahead %d" % (panel, la))
    pflag = hk.HK_FLAG_PANEL(panel)
    pflag |= {0: hk.HK_FLAG_LOOKAHEAD_OFF, 1: hk.HK_FLAG_LOOKAHEAD_ON,
              2: hk.HK_FLAG_LOOKAHEAD_FUSED}.get(la, 0)
    # untimed: work count (deterministic) and warmup
    dec, rep = hk.smallest_eig(N, beta, K, method=method, digits=45, ws=ws, flags=pflag)
    macs_per_step = rep["limb_macs"]
    log("work per step: %.4e limb-MACs over %d factorisations; lambda_1 = %s"
        % (macs_per_step, rep["factorizations"], dec))
    for _ in range(max(0, args.warmup - 1)):
        hk.smallest_eig(N, beta, K, method=method, digits=45, ws=ws, flags=hk.HK_FLAG_NO_WORK_COUNT | pflag)
    torch.cuda.synchronize()
    t0 = time.time()
    for _ in range(args.steps):
        dec, r = hk.smallest_eig(N, beta, K, method=method, digits=45, ws=ws,
                                 flags=hk.HK_FLAG_NO_WORK_COUNT | pflag)
        assert r["verified"] == 1
    torch.cuda.synchronize()
    dt = time.time() - t0
    ms_step = 1e3 * dt / args.steps
    value = macs_per_step * args.steps / dt
    # the update kernel's own time: one more step in which every update
    # launch records its start and end on HIP events of the library's stream
    # (stream launches instead of the graph replay, the kernels are the same)
    _, r = hk.smallest_eig(N, beta, K, method=method, digits=45, ws=ws,
                           flags=hk.HK_FLAG_NO_WORK_COUNT | hk.HK_FLAG_TIME_UPDATES | pflag)
    torch.cuda.synchronize()
    upd_ms, upd_n = r["update_ms"], r["update_launches"]
    achieved = macs_per_step / (upd_ms * 1e-3) if upd_ms > 0 else 0.0
    kernel = "k_column" if la == 2 else "k_update"
    kdesc = ("k_column (one column: its rows' update by the previous column, finalisation and division; "
             "the update of the columns beyond)" if la == 2 else "k_update (trailing + in-panel update)")
    traffic, traffic_src = measured_traffic(args.config, kernel)
    out = {
        "metric": "multiprecision limb-MACs/s (whole job) and % int-mul peak of the update kernel; "
                  "lambda_min solves/s at 1e-40 rel",
        "value": value, "unit": "limb-MAC/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": {"workload": "lambda_1 of the Hankel moment matrix, %s, %s driver, verified "
                               "to 45 digits" % (cfg["desc"], args.method),
                   "N": N, "beta": "%d/%d" % beta, "prec_bits": K, "method": args.method,
                   "panel": panel, "lookahead": la},
        "lambda_solves_per_s": args.steps / dt,
        "lambda_1": dec,
        "roofline": {"bound": "alu", "kernel": kdesc,
                     "achieved": achieved / 1e12, "peak": PEAK_INT_MUL / 1e12,
                     "unit": "Tlimb-MAC/s", "frac": achieved / PEAK_INT_MUL,
                     "launches": upd_n,
                     "avg_launch_us": 1e3 * upd_ms / max(upd_n, 1),
                     "limb_macs_per_launch": macs_per_step / max(upd_n, 1),
                     "share_of_step": upd_ms / ms_step,
                     "traffic": traffic, "traffic_unit": "bytes per launch (HBM, rocprofv3 FETCH_SIZE + "
                                                          "WRITE_SIZE, copy-calibrated)",
                     "traffic_source": traffic_src},
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(cfg, args.method)
    try:
        os.remove(tune_path)
    except OSError:
        pass
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
