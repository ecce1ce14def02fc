"""Benchmark: smallest eigenvalue of the Hankel moment matrix on one MI355X.

One step = one pass of the whole hot path over the workload's synthetic
instances: for each, moments (Gamma at the working precision) -> LDL^T
factorisations (expansion, panel, trailing update) -> the eigenvalue
iteration -> the inertia bracket at 45 digits, i.e. one verified lambda_1
per instance.  The default workload is N = 500, K = 6144 fractional bits,
beta = 1/2, 1, 3/2 and 2 (four separate runs, one step covers all four).

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

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--config c3]
"""
import argparse
import json
import os
import sys
import time

CONFIGS = {
    "c1": dict(runs=[(32, (1, 1), 512)], desc="N=32 beta=1 K=512"),
    "c2": dict(runs=[(200, (7, 4), 2048)], desc="N=200 beta=7/4 K=2048"),
    "c3": dict(runs=[(500, (1, 2), 6144), (500, (1, 1), 6144), (500, (3, 2), 6144), (500, (2, 1), 6144)],
               desc="N=500 K=6144, beta = 1/2, 1, 3/2 and 2 (four runs)", cpu_run=3),
    "c3b1": dict(runs=[(500, (1, 1), 6144)], desc="N=500 beta=1 K=6144"),
    "c3b2": dict(runs=[(500, (2, 1), 6144)], desc="N=500 beta=2 K=6144"),
    "c3b32": dict(runs=[(500, (3, 2), 6144)], desc="N=500 beta=3/2 K=6144"),
    "c3b12": dict(runs=[(500, (1, 2), 6144)], desc="N=500 beta=1/2 K=6144"),
    "c5": dict(runs=[(1500, (3, 2), 24576)], desc="N=1500 beta=3/2 K=24576"),
}
PEAK_INT_MUL = 256 * 64 * 2.4e9       # one 32x32 multiply per lane per clock
PEAK_INT8_OPS = 5.0e15                 # dense int8 matrix-core peak
HBM_PEAK = 8.0e12
HERE = os.path.dirname(os.path.abspath(__file__))
PROFILE_TAG = {"c2": "N200_beta7-4_K2048_secant", "c3b1": "N500_beta1_K6144_secant", "c3": "N500_K6144_4beta"}


def profile_figures(cfg_name, kernel):
    """Per-launch figures of `kernel` from the committed rocprofv3 counter
    summary of this workload (HBM bytes; 64-bit integer VALU instructions),
    each None when there is no summary or the kernel source has changed
    since the counters were taken; and the summary's path."""
    import hashlib
    import re
    tag = PROFILE_TAG.get(cfg_name)
    if tag is None:
        return {}, None
    path = os.path.join(HERE, "profiles", "%s_%s.txt" % (kernel, tag))
    try:
        txt = open(path).read()
    except OSError:
        return {}, None
    src = open(os.path.join(HERE, "paper_0902_0852_amd", "csrc", "hk_kernels.hip"), "rb").read()
    m = re.search(r"sha256 ([0-9a-f]{16})", txt)
    if not m or m.group(1) != hashlib.sha256(src).hexdigest()[:16]:
        return {}, os.path.relpath(path, HERE)
    out = {}
    for key in ("traffic_bytes_per_launch", "valu_int64_per_launch"):
        t = re.search(key + r"=([0-9.eE+]+)", txt)
        if t:
            out[key] = float(t.group(1))
    return out, os.path.relpath(path, HERE)


def measured_traffic(cfg_name, kernel):
    """HBM bytes per launch of `kernel` from the committed profile (None when
    there is none or it is stale), and the profile's path."""
    fig, path = profile_figures(cfg_name, kernel)
    t = fig.get("traffic_bytes_per_launch")
    return (int(t) if t is not None else None), path


def log(msg):
    sys.stderr.write(msg + "\n")
    sys.stderr.flush()


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(cfg, method, budget_s=20.0):
    """The oracle (test infrastructure) on the same workload, bounded.  For
    a single small run: whole verified lambda_1 runs (iteration + the two
    bracket factorisations) until the budget is spent, work = factorisations
    x the limb MACs of one.  For N >= 500: one whole factorisation at x = 0
    of the configuration's sample run (about 10 s on 16 host threads at
    N = 500, K = 6144); the rate is the same quantity, limb MACs per
    second."""
    import oracle
    from oracle.drivers import inverse_iteration, secant, verify
    from oracle.moments import moments
    N, beta, K = cfg["runs"][cfg.get("cpu_run", 0)]
    X = moments(N, beta, K)                 # matrix generation excluded, as in the paper
    info = {"cores": oracle.max_threads(), "kind": "oracle", "cpu": cpu_model(), "nproc": os.cpu_count()}
    if N >= 500:
        t0 = time.time()
        f = oracle.factor_from_moments(X, N, K, 0)
        dt = time.time() - t0
        info.update({"value": f.limb_macs / dt, "unit": "limb-MAC/s",
                     "sample": "one whole factorisation at x = 0 of N=%d beta=%d/%d K=%d "
                               "(%.3e limb-MACs), moments excluded, %.1f s"
                               % (N, beta[0], beta[1], K, f.limb_macs, dt)})
        return info
    macs0 = oracle.factor_from_moments(X, N, K, 0).limb_macs
    t0 = time.time()
    nfact, n = 0, 0
    while True:
        if method == "secant":
            lam, inf = secant(N, beta, K, X=X)
        else:
            lam, inf = inverse_iteration(N, beta, K, X=X)
        ok, _ = verify(N, beta, K, lam, X=X)
        nfact += inf["factorizations"] + 2
        n += 1
        if time.time() - t0 > budget_s / 2 or n >= 12:
            break
    dt = time.time() - t0
    info.update({"value": nfact * macs0 / dt, "unit": "limb-MAC/s",
                 "sample": "%d verified lambda_1 runs (%s driver, %d factorisations) of N=%d beta=%d/%d K=%d, "
                           "moments excluded, %.1f s" % (n, method, nfact, N, beta[0], beta[1], K, dt),
                 "lambda_per_s": n / dt})
    return info


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
        N5, beta5, K5 = CONFIGS["c5"]["runs"][0]
        insts = [(N5, beta5)]
        plain = [(N5, beta5, K5)]
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


def peak_rates(args):
    """Measured issue rates of the VALU multiply instructions (hk_mul_rate)
    against the nominal one operation per lane per clock on 256 CUs at
    2.4 GHz; the update kernel multiplies with v_mad_i64_i32."""
    import paper_0902_0852_amd as hk
    kinds = [("v_mad_i64_i32", hk.HK_RATE_MAD_I64_I32), ("v_mad_u64_u32", hk.HK_RATE_MAD_U64_U32),
             ("v_mad_u32_u24", hk.HK_RATE_MAD_U32_U24), ("v_fma_f64", hk.HK_RATE_FMA_F64)]
    out = {"metric": "measured issue rate (VALU: lane operations/s; matrix cores: int8 multiply-adds/s)",
           "unit": "ops/s", "n_gpus": 1, "nominal_per_s": PEAK_INT_MUL, "rates": {}}
    for name, k in kinds:
        rate, clk = hk.mul_rate(k)
        out["rates"][name] = {"per_s": rate, "of_nominal": rate / PEAK_INT_MUL, "clock_hz": clk,
                              "per_lane_per_clock": rate / (256 * 64 * clk) if clk > 0 else None}
        log("%-14s %.4e ops/s = %.3f of nominal, clock %.3f GHz" % (name, rate, rate / PEAK_INT_MUL, clk / 1e9))
    rate, clk = hk.mul_rate(hk.HK_RATE_MFMA_I8)
    out["rates"]["v_mfma_i32_32x32x32_i8"] = {"per_s": rate, "unit": "int8 multiply-adds/s",
                                              "of_dense_peak": 2 * rate / PEAK_INT8_OPS, "clock_hz": clk,
                                              "limb_macs_per_s": rate / 16 / (32 / 29) ** 2}
    log("%-14s %.4e MAC/s = %.3f of the 5.0 POP/s dense peak, clock %.3f GHz; %.4e limb-MAC/s of 29-bit digits"
        % ("mfma_i8", rate, 2 * rate / PEAK_INT8_OPS, clk / 1e9, rate / 16 / (32 / 29) ** 2))
    print(json.dumps(out), flush=True)


# the paper's table of smallest eigenvalues ('Numerical results'), the rows
# beyond the GPU tests: (N, column of beta, precision K, driver)
TABLE_BETAS = [(1, 3), (1, 2), (1, 1), (7, 4)]
TABLE_RUNS = {
    1000: [(0, 8192), (1, 6144), (2, 6144), (3, 8192)],
    1500: [(0, 10240), (1, 8192), (2, 8192), (3, 10240)],
}


def lambda_table(args):
    """lambda_1 of rows of the paper's table on the GPU (inverse iteration
    from 0, or the Secant iteration where the solve vectors do not fit, and
    the 45-digit inertia bracket), each compared with the printed five
    digits; one JSON line per run."""
    from fractions import Fraction
    os.environ.setdefault("HK_TRACE", "1")   # the driver reports each factorisation and solve
    import paper_0902_0852_amd as hk
    gold = json.load(open(os.path.join(HERE, "tests", "golden", "paper_lambda_table.json")))
    for N in [int(x) for x in args.rows.split(",")]:
        for col, K in TABLE_RUNS[N]:
            if args.cols and col not in [int(c) for c in args.cols.split(",")]:
                continue
            beta = TABLE_BETAS[col]
            log("table: N=%d beta=%d/%d K=%d" % (N, beta[0], beta[1], K))
            t0 = time.time()
            method = "inverse"
            try:
                dec, rep = hk.smallest_eig(N, beta, K, method=hk.HK_INVERSE, digits=45,
                                           flags=hk.HK_FLAG_NO_WORK_COUNT)
            except hk.HKError as e:
                # the solve sweeps' vectors too wide for one workgroup's LDS:
                # the Secant iteration needs factorisations only
                if e.status != 1 or "LDS" not in str(e):
                    raise
                log("  %s; Secant instead" % e)
                method = "secant"
                t0 = time.time()
                dec, rep = hk.smallest_eig(N, beta, K, method=hk.HK_SECANT, digits=45,
                                           flags=hk.HK_FLAG_NO_WORK_COUNT)
            dt = time.time() - t0
            m, e = (gold["rows"][str(N)][col].split("e") + ["0"])[:2]
            ref = Fraction(m) * Fraction(10) ** int(e)
            lam = rep["lambda"]
            rel = abs(lam - ref) / ref
            print(json.dumps({"N": N, "beta": "%d/%d" % beta, "K": K, "method": method, "lambda_1": dec, "paper": gold["rows"][str(N)][col],
                              "rel_diff_vs_paper": float(rel), "within_print": bool(rel <= Fraction(51, 10 ** 6)),
                              "verified": rep["verified"], "factorizations": rep["factorizations"],
                              "solves": rep["solves"], "seconds": dt}), flush=True)


def roofline_record(hk, engine, macs_bulk, bulk_ms, bulk_n, macs_per_step, upd_ms, upd_n, ms_step, fig,
                    traffic, traffic_src, kernel):
    """The roofline record of the kernel that carries the bulk of the update
    work.  On the matrix cores (k_update_mma) the algorithmic work is priced
    as int8 matrix operations: one 32-bit limb-MAC is 16 int8 multiply-adds
    (32 ops), against the dense int8 peak (5.0 POP/s); on the vector units
    (k_update, k_column) against one 32-bit multiply per lane per clock."""
    achieved = macs_bulk / (bulk_ms * 1e-3) if bulk_ms > 0 else 0.0
    avg_s = 1e-3 * bulk_ms / max(bulk_n, 1)
    valu64 = fig.get("valu_int64_per_launch")
    all_rate = macs_per_step / (upd_ms * 1e-3) if upd_ms else 0.0
    rec = {"launches": bulk_n, "avg_launch_us": 1e3 * bulk_ms / max(bulk_n, 1),
           "limb_macs_per_launch": macs_bulk / max(bulk_n, 1),
           "work_share": macs_bulk / macs_per_step if macs_per_step else None,
           "time_share_of_step": bulk_ms / ms_step,
           "traffic": traffic, "traffic_unit": "bytes per launch (HBM, rocprofv3 FETCH_SIZE + WRITE_SIZE, "
                                              "copy-calibrated)",
           "traffic_source": traffic_src,
           "limb_mac_rate_T": achieved / 1e12}
    if engine == 1:
        rec.update({"bound": "mfma", "kernel": "k_update_mma (the bulk of the trailing update on the matrix "
                                               "cores: int8 byte-plane products, v_mfma_i32_32x32x32_i8)",
                    "achieved": 32 * achieved / 1e12, "peak": PEAK_INT8_OPS / 1e12, "unit": "TOP/s",
                    "op_basis": "int8 ops of the algorithmic 32-bit limb-MACs (32 per limb-MAC)",
                    "frac": 32 * achieved / PEAK_INT8_OPS,
                    "all_update_launches": {"launches": upd_n, "ms_per_step": upd_ms,
                                            "achieved": 32 * all_rate / 1e12, "frac": 32 * all_rate / PEAK_INT8_OPS}})
    else:
        rec.update({"bound": "alu", "kernel": kernel,
                    "achieved": achieved / 1e12, "peak": PEAK_INT_MUL / 1e12, "unit": "Tlimb-MAC/s",
                    "frac": achieved / PEAK_INT_MUL,
                    "executed_int64_valu_frac": valu64 * 64 / avg_s / PEAK_INT_MUL if valu64 and avg_s > 0 else None,
                    "all_update_launches": {"launches": upd_n, "ms_per_step": upd_ms,
                                            "achieved": all_rate / 1e12, "frac": all_rate / PEAK_INT_MUL}})
    return rec


def plain_batched(args, cfg, hk, torch):
    """The workload's runs as one batch per step (hk_eig_batched: the Secant
    iterations of all runs in lockstep, every factorisation launch covering
    all of them, then the inertia bracket for all).  The algorithmic work
    and lambda_1 come from one untimed run of each instance alone
    (hk_smallest_eig with the same schedule): the batch must reproduce every
    lambda_1 digit for digit with the same number of factorisations."""
    import tempfile
    runs = cfg["runs"]
    if args.method != "secant":
        raise SystemExit("the batched driver runs the Secant iteration")
    tune_path = os.path.join(tempfile.gettempdir(), "hk_tune_%d.txt" % os.getpid())
    os.environ["HK_TUNE_CACHE"] = tune_path
    # batches: the runs dealt round-robin after sorting by work (widest first)
    nsplit = max(1, min(args.split, len(runs)))
    order = sorted(range(len(runs)), key=lambda i: -hk.workspace_bytes(*runs[i]))
    groups = [[order[k] for k in range(g, len(runs), nsplit)] for g in range(nsplit)]
    if args.panel > 0:
        panel, la, group = args.panel, args.lookahead, args.group or 4
    else:
        panel, la, group = hk.autotune([runs[i] for i in groups[0]], cache_path=tune_path)
        group = args.group or group
    la_flag = {0: hk.HK_FLAG_LOOKAHEAD_OFF, 1: hk.HK_FLAG_LOOKAHEAD_ON, 2: hk.HK_FLAG_LOOKAHEAD_FUSED}.get(la, 0)
    bflags = la_flag | hk.HK_FLAG_GROUP(group)
    log("batch of %d runs: panel width %d, look-ahead %d, %d update items per workgroup (%s)"
        % (len(runs), panel, la, group, "given" if args.panel > 0 else "tuned"))
    wsg = [torch.empty(hk.batch_workspace_bytes([runs[i] for i in g], paired=not args.unpaired), dtype=torch.uint8, device="cuda")
           for g in groups]
    streams = [torch.cuda.current_stream()] + [torch.cuda.Stream() for _ in groups[1:]]
    from concurrent.futures import ThreadPoolExecutor
    pool = ThreadPoolExecutor(max_workers=len(groups)) if len(groups) > 1 else None
    # untimed reference: each run alone, with its work count
    wss = torch.empty(max(hk.workspace_bytes(N, beta, K) for N, beta, K in runs), dtype=torch.uint8,
                      device="cuda")
    single = []
    for N, beta, K in runs:
        dec, r = hk.smallest_eig(N, beta, K, method=hk.HK_SECANT, digits=45, ws=wss,
                                 flags=hk.HK_FLAG_PANEL(panel) | bflags)
        assert r["verified"] == 1
        single.append((dec, r))
    del wss
    macs_per_step = sum(r["limb_macs"] for _, r in single)
    macs_bulk = sum(r["limb_macs_bulk"] for _, r in single)
    lams = [dec for dec, _ in single]

    def one_batch(gi, extra):
        g = groups[gi]
        res, d = hk.eig_batched([runs[i] for i in g], digits=45, panel=panel, ws=wsg[gi], stream=streams[gi],
                                method=hk.HK_SECANT, flags=bflags | extra)
        for (st, dec, ver, nf), i in zip(res, g):
            dec1, r1 = single[i]
            assert st == 0 and ver == 1, (st, dec)
            assert dec == dec1 and nf == r1["factorizations"], (dec, dec1, nf, r1["factorizations"])
        return d

    def one_step(extra):
        if pool is None:
            return one_batch(0, extra)
        ds = list(pool.map(lambda gi: one_batch(gi, extra), range(len(groups))))
        d = dict(ds[0])
        for k in ("update_launches", "update_ms", "bulk_launches", "bulk_ms"):
            d[k] = sum(x[k] for x in ds)
        return d
    log("work per step: %.4e limb-MACs over %d factorisations; lambda_1 = %s"
        % (macs_per_step, sum(r["factorizations"] for _, r in single), ", ".join(lams)))
    for _ in range(max(1, args.warmup)):
        one_step(0)
    torch.cuda.synchronize()
    t0 = time.time()
    for _ in range(args.steps):
        one_step(0)
    torch.cuda.synchronize()
    dt = time.time() - t0
    ms_step = 1e3 * dt / args.steps
    value = macs_per_step * args.steps / dt
    # one more step with every update launch timed on HIP events of the
    # stream it runs on (launched one by one instead of the graph replay)
    d = one_step(hk.HK_FLAG_TIME_UPDATES)
    torch.cuda.synchronize()
    engine = d["update_engine"]
    kernel = "k_update_mma" if engine == 1 else "k_update"
    traffic, traffic_src = measured_traffic(args.config, kernel)
    fig, _ = profile_figures(args.config, kernel)
    rec = roofline_record(hk, engine, macs_bulk, d["bulk_ms"], d["bulk_launches"], macs_per_step,
                          d["update_ms"], d["update_launches"], ms_step, fig, traffic, traffic_src,
                          "k_update (the bulk of the trailing update on the vector units)")
    out = {
        "metric": "multiprecision limb-MACs/s (whole job) and % int-mul peak of the update kernel; "
                  "lambda_min solves/s at 1e-40 rel",
        "value": value, "unit": "limb-MAC/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": {"workload": "lambda_1 of the Hankel moment matrix, %s, Secant driver, all runs of a step "
                               "as one batch, verified to 45 digits" % cfg["desc"],
                   "N": [N for N, _, _ in runs], "beta": ["%d/%d" % b for _, b, _ in runs],
                   "prec_bits": [K for _, _, K in runs], "method": "secant", "driver": "batched",
                   "concurrent_batches": [[i for i in g] for g in groups],
                   "paired_factorisations": not args.unpaired,
                   "panel": panel, "lookahead": la, "update_group": group,
                   "update_engine": "matrix cores" if engine == 1 else "vector units"},
        "lambda_solves_per_s": len(runs) * args.steps / dt,
        "lambda_1": lams,
        "roofline": rec,
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(cfg, args.method)
    try:
        os.remove(tune_path)
    except OSError:
        pass
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c3", choices=sorted(CONFIGS))
    ap.add_argument("--method", default="secant", choices=["secant", "inverse"])
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--mode", default="plain", choices=["plain", "learned", "peak", "table"],
                    help="learned: batched + learned form against the batched plain form; "
                         "peak: measured issue rates of the multiply instructions; "
                         "table: rows of the paper's lambda table (--rows, --cols)")
    ap.add_argument("--rows", default="1000", help="table mode: N rows, comma separated (1000, 1500)")
    ap.add_argument("--cols", default="", help="table mode: beta columns 0..3 (1/3, 1/2, 1, 7/4); default all")
    ap.add_argument("--model", default=None, help="network file (default: the package's trained one)")
    ap.add_argument("--instances", type=int, default=64)
    ap.add_argument("--seed", type=int, default=4242)
    ap.add_argument("--n-lo", type=int, default=50)
    ap.add_argument("--n-hi", type=int, default=400)
    ap.add_argument("--panel", type=int, default=0, help="panel width (0: tuned here / tuned or 4 in learned mode)")
    ap.add_argument("--group", type=int, default=0, choices=[0, 1, 2, 4],
                    help="update items per workgroup (0: tuned, else 4)")
    ap.add_argument("--driver", default="", choices=["", "single", "batched"],
                    help="single: the runs one after another (hk_smallest_eig); batched: all runs of a "
                         "step as one batch (hk_eig_batched, lockstep Secant); default batched when the "
                         "workload has several runs")
    ap.add_argument("--split", type=int, default=1,
                    help="batched driver: the runs as this many batches launched concurrently, one host thread "
                         "and one stream each")
    ap.add_argument("--unpaired", action="store_true",
                    help="batched driver: the batch workspace without the second copy of every run, so "
                         "the Secant's start points and the bracket's ends are factored one at a time")
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
    if args.mode == "peak":
        peak_rates(args)
        return
    if args.mode == "table":
        lambda_table(args)
        return
    import torch
    import paper_0902_0852_amd as hk
    cfg = CONFIGS[args.config]
    runs = cfg["runs"]
    method = hk.HK_SECANT if args.method == "secant" else hk.HK_INVERSE
    if args.driver == "batched" or (args.driver == "" and len(runs) > 1):
        plain_batched(args, cfg, hk, torch)
        return
    ws = torch.empty(max(hk.workspace_bytes(N, beta, K) for N, beta, K in runs), dtype=torch.uint8, device="cuda")
    # untimed: the schedule tuned for each shape (hk_autotune; the library
    # reads it back from the cache named by HK_TUNE_CACHE)
    import tempfile
    tune_path = os.path.join(tempfile.gettempdir(), "hk_tune_%d.txt" % os.getpid())
    os.environ["HK_TUNE_CACHE"] = tune_path
    flags, scheds = [], []
    for N, beta, K in runs:
        group = args.group
        if args.panel > 0:
            panel, la = args.panel, args.lookahead
            if la < 0:   # the mode the library picks for this size
                m = hk.Matrix(N, beta, K, ws=ws)
                m.set_panel(panel)
                la = m.info().lookahead
                del m
        else:
            panel, la, g = hk.autotune([(N, beta, K)], cache_path=tune_path)
            group = group or g
        pflag = hk.HK_FLAG_PANEL(panel) | (hk.HK_FLAG_GROUP(group) if group else 0)
        pflag |= {0: hk.HK_FLAG_LOOKAHEAD_OFF, 1: hk.HK_FLAG_LOOKAHEAD_ON,
                  2: hk.HK_FLAG_LOOKAHEAD_FUSED}.get(la, 0)
        flags.append(pflag)
        scheds.append((panel, la, group or 4))
        log("N=%d beta=%d/%d K=%d: panel width %d, look-ahead %d, %d update items per workgroup (%s)"
            % (N, beta[0], beta[1], K, panel, la, group or 4, "given" if args.panel > 0 else "tuned"))

    def one_step(extra):
        out = []
        for (N, beta, K), fl in zip(runs, flags):
            dec, r = hk.smallest_eig(N, beta, K, method=method, digits=45, ws=ws, flags=fl | extra)
            assert r["verified"] == 1
            out.append((dec, r))
        return out
    # untimed: work count (deterministic) and warmup
    res = one_step(0)
    macs_per_step = sum(r["limb_macs"] for _, r in res)
    lams = [dec for dec, _ in res]
    log("work per step: %.4e limb-MACs over %d factorisations; lambda_1 = %s"
        % (macs_per_step, sum(r["factorizations"] for _, r in res), ", ".join(lams)))
    for _ in range(max(0, args.warmup - 1)):
        one_step(hk.HK_FLAG_NO_WORK_COUNT)
    torch.cuda.synchronize()
    t0 = time.time()
    for _ in range(args.steps):
        one_step(hk.HK_FLAG_NO_WORK_COUNT)
    torch.cuda.synchronize()
    dt = time.time() - t0
    ms_step = 1e3 * dt / args.steps
    value = macs_per_step * args.steps / dt
    # the update kernel's own time: one more step in which every update
    # launch records its start and end on HIP events of the library's stream
    # (stream launches instead of the graph replay, the kernels are the same)
    res_t = one_step(hk.HK_FLAG_NO_WORK_COUNT | hk.HK_FLAG_TIME_UPDATES)
    torch.cuda.synchronize()
    upd_ms = sum(r["update_ms"] for _, r in res_t)
    upd_n = sum(r["update_launches"] for _, r in res_t)
    bulk_ms = sum(r["bulk_ms"] for _, r in res_t)
    bulk_n = sum(r["bulk_launches"] for _, r in res_t)
    macs_bulk = sum(r["limb_macs_bulk"] for _, r in res)
    fused = all(la == 2 for _, la, _ in scheds)
    kernel = "k_column" if fused else "k_update"
    kdesc = ("k_column (one column: its rows' update by the previous column, finalisation and division; "
             "the update of the columns beyond)" if fused else
             "k_update (the bulk of the trailing update: each panel's update of the columns beyond the next "
             "panel under look-ahead, or its whole trailing update without)")
    engine = 0 if fused else res_t[0][1]["update_engine"]
    if engine == 1:
        kernel = "k_update_mma"
    traffic, traffic_src = measured_traffic(args.config, kernel)
    fig, _ = profile_figures(args.config, kernel)
    rec = roofline_record(hk, engine, macs_bulk, bulk_ms, bulk_n, macs_per_step, upd_ms, upd_n, ms_step, fig,
                          traffic, traffic_src, kdesc)
    out = {
        "metric": "multiprecision limb-MACs/s (whole job) and % int-mul peak of the update kernel; "
                  "lambda_min solves/s at 1e-40 rel",
        "value": value, "unit": "limb-MAC/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": {"workload": "lambda_1 of the Hankel moment matrix, %s, %s driver, verified "
                               "to 45 digits" % (cfg["desc"], args.method),
                   "N": [N for N, _, _ in runs], "beta": ["%d/%d" % b for _, b, _ in runs],
                   "prec_bits": [K for _, _, K in runs], "method": args.method,
                   "panel": [p for p, _, _ in scheds], "lookahead": [la for _, la, _ in scheds],
                   "update_group": [g for _, _, g in scheds]},
        "lambda_solves_per_s": len(runs) * args.steps / dt,
        "lambda_1": lams,
        "roofline": rec,
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
