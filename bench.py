"""Benchmark: CP-ALS time-to-fit and MTTKRP TFLOP/s, split-BF16 vs FP64, on one MI355X.

Workload (default): the mixed-precision configuration -- THC input with
N = 800 orbitals, R_thc = 4000, R_cp = 4000, from the seeded generator
(synthetic stand-in for the paper's water clusters).

Protocol
  1. Reference (untimed): plain FP64 CP-ALS for --ref-sweeps sweeps with the
     stopping rule off; f_ref = its best fit, target f* = f_ref (1 + 1e-4).
  2. Warm-up (untimed): --warmup mixed runs to the target.
  3. Timed: --steps runs of the mixed-precision path, each from cpd_init
     (inputs already in HBM) to the end of the first sweep whose fit --
     evaluated in FP64 -- is <= f*.  value = median seconds per run (null
     if any run missed the target), with the spread.  Three timed FP64 runs
     to the same target give the FP64 time-to-fit (median).
     Untimed: one split-BF16 run with the fit evaluated every sweep gives
     the per-sweep fit error |f_mixed - f_fp64| / f_fp64 against the
     reference trajectory.
  4. Kernel times (hipEvents on the plan's stream) of the projection, core
     product, back-projection, Gram and solve at this shape give MTTKRP
     TFLOP/s for both precisions and the roofline of the dominant kernel.
  5. CPU baseline: the matrix-free NumPy oracle on the host, a bounded
     sample of sweeps (all threads, and one sweep on one thread),
     extrapolated to the FP64 sweep count.

Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

MFMA_PEAK = {"bf16": 2.5e15, "f64": 78.6e12, "f32": 157.3e12}
HBM_PEAK = 8.0e12


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def mttkrp_flops(n, r_thc, r_cp):
    return 4.0 * r_thc * r_cp * sum(n) + 4.0 * r_thc * r_thc * r_cp


def measured_traffic(kernel, profile="chol_fwd_flow_traffic_n800_r4000.md"):
    """HBM bytes per launch of `kernel` from a committed PMC summary, or
    None once the kernel's source has changed since the counters were taken."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", profile)
    try:
        text = open(path).read()
    except OSError:
        return None
    m = re.search(r"kernel=(\S+) traffic_bytes_per_launch=(\d+) source=(\S+) sha256=([0-9a-f]+)", text)
    if not m or m.group(1) != kernel:
        return None
    src = os.path.join(ROOT, m.group(3))
    try:
        digest = hashlib.sha256(open(src, "rb").read()).hexdigest()
    except OSError:
        return None
    return float(m.group(2)) if digest == m.group(4) else None


def run_to_target(make, target, max_sweeps, chunk=1):
    """Wall time (s) from plan creation to the sweep that reaches target,
    plus the sweep count, whether the target was reached, the last evaluated
    fit and whether the precision guard moved the run to FP64 products."""
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    cpd = make()
    sweeps, reached, last = 0, False, None
    while sweeps < max_sweeps:
        fits = cpd.sweep(chunk)
        if not fits:
            break
        sweeps += len(fits)
        evaluated = [f for f in fits if f >= 0]
        if evaluated:
            last = evaluated[-1]
            if last <= target:
                reached = True
                break
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    st = cpd.stats()
    cpd.close()
    return t, sweeps, reached, last, int(st["fp64_path"])


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def spread(xs):
    a = np.asarray(xs, dtype=np.float64)
    return {"median": float(np.median(a)), "min": float(a.min()), "max": float(a.max()),
            "p25": float(np.percentile(a, 25)), "p75": float(np.percentile(a, 75)), "n": int(a.size)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=800)
    ap.add_argument("--r-thc", type=int, default=4000)
    ap.add_argument("--r-cp", type=int, default=4000)
    ap.add_argument("--ref-sweeps", type=int, default=200)
    ap.add_argument("--max-sweeps", type=int, default=400)
    ap.add_argument("--fit-every", type=int, default=4)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--cpu-sweeps", type=int, default=3)
    ap.add_argument("--cpu-sweeps-1t", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--init", choices=("normal", "uniform"), default="normal",
                    help="initial factors: N(0,1)/sqrt(n) (default) or the paper's U[-1,1]")
    ap.add_argument("--workload", choices=("mixed", "lt", "warmstart", "exchange", "tied", "df", "combined",
                                           "kernels"),
                    default="mixed",
                    help="mixed: the headline time-to-fit line (default); lt: the batched "
                         "Laplace-transform CPDs; warmstart: train and evaluate the learned warm start; "
                         "exchange: the robust CPD+THC LT-MP2 exchange energy of the batched systems; "
                         "tied: the particle-tied CPD (symmetric ALS) against the four-factor one, FP64; "
                         "df: DF-based against THC-based CP-ALS, FP64, growing n; combined: the 48 "
                         "Laplace CPDs in split BF16 from the learned warm start, each to its FP64 "
                         "reference fit, against FP64 from the random start; kernels: only the "
                         "per-kernel timing hook of both precisions at the headline shape (a short run for "
                         "hardware counters)")
    ap.add_argument("--lt-sweeps", type=int, default=40)
    ap.add_argument("--lt-precisions", default="mixed,fp32,fp64",
                    help="lt workload: the precisions of the batched sweeps (comma-separated)")
    ap.add_argument("--lt-batched-only", action="store_true",
                    help="lt workload: only the batched sweeps (no one-by-one runs, no runs to convergence); "
                         "short enough for hardware counters")
    ap.add_argument("--accuracy-sweeps", type=int, default=100,
                    help="exchange workload: CP-ALS sweep cap for the accuracy comparison (0: skip)")
    ap.add_argument("--ws-train", type=int, default=2000)
    ap.add_argument("--ws-heldout", type=int, default=200)
    ap.add_argument("--ws-heldout-large", type=int, default=200)
    ap.add_argument("--ws-budget", type=int, default=200)
    ap.add_argument("--comb-train-sets", type=int, default=4,
                    help="combined workload: training Laplace batches (3 systems x 16 points each)")
    ap.add_argument("--comb-ref-sweeps", type=int, default=300)
    ap.add_argument("--comb-cap", type=int, default=600)
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="run one plain device-to-device copy of this size first (for scaling HBM counters)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: there is no multi-GPU path "
              "(the design notes describe how it would shard).", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration_mib > 0:
        import torch
        nb = args.copy_calibration_mib << 20
        src = torch.ones(nb // 8, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] copy calibration: {nb} bytes read, {nb} bytes written")
        del src, dst
    if args.workload == "lt":
        return bench_lt(args)
    if args.workload == "warmstart":
        return bench_warmstart(args)
    if args.workload == "exchange":
        return bench_exchange(args)
    if args.workload == "tied":
        return bench_tied(args)
    if args.workload == "df":
        return bench_df(args)
    if args.workload == "combined":
        return bench_combined(args)
    if args.workload == "kernels":
        return bench_kernels(args)

    import torch
    from paper_2502_17683_amd import CPD
    from synth import make_thc, init_factors, init_factors_uniform

    N, Rt, Rc = args.n, args.r_thc, args.r_cp
    dev = torch.device("cuda:0")
    log(f"[bench] generating THC input N={N} R_thc={Rt} R_cp={Rc} seed={args.seed}")
    X, Z = make_thc(N, Rt, args.seed)
    init = (init_factors_uniform if args.init == "uniform" else init_factors)([N] * 4, Rc, args.seed + 1000)
    Xd = torch.as_tensor(X, device=dev)
    Zd = torch.as_tensor(Z, device=dev)
    Id = [torch.as_tensor(f, device=dev) for f in init]

    def make(prec, tol=0.0, fit_every=1):
        return CPD(Xd, Zd, Rc, Id, precision=prec, tol=tol, fit_floor=0.0, fit_every=fit_every)

    # 1. FP64 reference trajectory
    log(f"[bench] FP64 reference: {args.ref_sweeps} sweeps")
    ref = make("fp64")
    ref_fits = ref.sweep(args.ref_sweeps)
    ref.close()
    f_ref = float(min(ref_fits))
    target = f_ref * (1.0 + 1e-4)
    log(f"[bench] f_ref={f_ref:.8f} target={target:.8f} (first fit {ref_fits[0]:.6f})")

    # 2./3. time-to-fit
    mk_mixed = lambda: make("mixed", fit_every=args.fit_every)
    for w in range(args.warmup):
        t, s, ok, last, p64 = run_to_target(mk_mixed, target, args.max_sweeps, args.fit_every)
        log(f"[bench] warmup {w}: mixed {t:.3f}s sweeps={s} reached={ok} last_fit={last} fp64_path={p64}")
    times, sweeps_m, reached_m, last_m, path_m = [], [], [], [], []
    for k in range(args.steps):
        t, s, ok, last, p64 = run_to_target(mk_mixed, target, args.max_sweeps, args.fit_every)
        times.append(t)
        sweeps_m.append(s)
        reached_m.append(ok)
        last_m.append(last)
        path_m.append(p64)
        log(f"[bench] step {k}: mixed {t:.3f}s sweeps={s} reached={ok} last_fit={last} fp64_path={p64}")
    t64s = []
    for k in range(3):
        t64, s64, ok64, last64, _ = run_to_target(lambda: make("fp64"), target, args.max_sweeps, 1)
        t64s.append(t64)
        log(f"[bench] fp64 run {k}: {t64:.3f}s sweeps={s64} reached={ok64} last_fit={last64}")
    t64 = float(np.median(t64s))

    # per-sweep fit error of split BF16 against the FP64 reference trajectory
    # (same start; the split run evaluates its fit in FP64 every sweep)
    em = make("mixed", fit_every=1)
    mfits = em.sweep(args.ref_sweeps)
    em_path = int(em.stats()["fp64_path"])
    em.close()
    nerr = min(len(mfits), len(ref_fits))
    err = np.abs(np.array(mfits[:nerr]) - np.array(ref_fits[:nerr])) / np.array(ref_fits[:nerr])
    fit_err = {"per_sweep": [float(e) for e in err],
               "max_first_10": float(err[:10].max()), "max_first_50": float(err[:50].max()),
               "max_all": float(err.max()), "final": float(err[-1]),
               "final_fit_mixed": float(mfits[nerr - 1]), "final_fit_fp64": float(ref_fits[nerr - 1]),
               "fp64_path": em_path}
    log(f"[bench] per-sweep |f_mixed - f_fp64| / f_fp64: first 10 <= {fit_err['max_first_10']:.2e}, "
        f"first 50 <= {fit_err['max_first_50']:.2e}, all {nerr} <= {fit_err['max_all']:.2e}, "
        f"final {fit_err['final']:.2e}")

    # 4. kernel times
    kt = {}
    for prec in ("mixed", "fp64"):
        c = make(prec)
        kt[prec] = c.kernel_times(reps=5)
        c.close()
        log(f"[bench] kernel ms ({prec}): {kt[prec]}")
    fl_core = 2.0 * Rt * Rt * Rc
    def mttkrp_ms(k):
        return 4 * k["projection"] + 2 * k["core"] + 4 * k["backprojection"]
    mtt = mttkrp_flops([N] * 4, Rt, Rc)
    tflops = {p: mtt / (mttkrp_ms(kt[p]) * 1e-3) / 1e12 for p in kt}
    core_ms = kt["mixed"]["core"]
    core_achieved = fl_core / (core_ms * 1e-3)
    # what the matrix cores execute for it: three BF16 passes over the
    # 256 x 256 tile grid (rows and columns padded to a multiple of 256)
    pad = lambda x: (x + 255) // 256 * 256
    core_executed = 3.0 * 2.0 * pad(Rc) * pad(Rt) * Rt / (core_ms * 1e-3)
    # dominant kernel of the mixed sweep: the dataflow Cholesky factorisation
    # fused with the forward solve (one launch per mode update, after a flag
    # reset of ~5 us that stays in the timing; FP64 matrix cores): R^3 / 3
    # flops plus the forward triangular solve of n rows, n R^2
    fl_factor_fwd = Rc ** 3 / 3.0 + 1.0 * N * Rc * Rc
    launches = 1
    per_launch_ms = kt["mixed"]["factor_fwd"] - kt["mixed"]["form_v"]
    fac_achieved = fl_factor_fwd / (per_launch_ms * 1e-3)
    sweep_ms = {p: 4 * (k["projection"] + k["backprojection"] + k["gram"] + k["solve"]) + 2 * k["core"]
                for p, k in kt.items()}

    # 5. CPU oracle baseline
    cpu = None
    if not args.no_cpu:
        from oracle import matfree
        import multiprocessing
        from threadpoolctl import threadpool_limits
        cores = int(os.environ.get("OMP_NUM_THREADS", multiprocessing.cpu_count()))
        log(f"[bench] CPU oracle: {args.cpu_sweeps} sweeps on {cores} threads, "
            f"{args.cpu_sweeps_1t} on one thread ({cpu_model()})")
        st = matfree.MatFreeCPALS([X] * 4, Z, init)
        with threadpool_limits(cores):
            t0 = time.perf_counter()
            for _ in range(args.cpu_sweeps):
                st.sweep()
            dt = (time.perf_counter() - t0) / args.cpu_sweeps
        dt1 = None
        if args.cpu_sweeps_1t > 0:
            with threadpool_limits(1):
                t0 = time.perf_counter()
                for _ in range(args.cpu_sweeps_1t):
                    st.sweep()
                dt1 = (time.perf_counter() - t0) / args.cpu_sweeps_1t
        cpu = {"value": dt * s64, "unit": "s", "cores": cores, "kind": "oracle",
               "sample": f"{args.cpu_sweeps} matrix-free FP64 NumPy sweeps at N={N}, R_thc={Rt}, "
                         f"R_cp={Rc} ({dt:.2f} s/sweep, set-up excluded), extrapolated to the "
                         f"{s64} sweeps the FP64 GPU run needed",
               "cpu_model": cpu_model(), "s_per_sweep": dt, "s_per_sweep_1thread": dt1,
               "sweeps_1thread": args.cpu_sweeps_1t}

    value = float(np.median(times)) if all(reached_m) else None
    out = {
        "metric": "CP-ALS time-to-fit 1e-4 (s) and MTTKRP TFLOP/s, mixed vs FP64, 1 MI355X",
        "value": value,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": value * 1e3 if value is not None else None,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16-split(fp32 acc)+f64",
        "data": "synthetic",
        "config": {"workload": f"mixed-precision THC CP-ALS, N={N}, R_thc={Rt}, R_cp={Rc}, "
                               f"seed {args.seed}, target fit = FP64 best over "
                               f"{args.ref_sweeps} sweeps x (1+1e-4)",
                   "n": N, "r_thc": Rt, "r_cp": Rc, "fit_every": args.fit_every, "init": args.init},
        "time_to_fit_s": {"mixed": spread(times), "fp64": spread(t64s)},
        "fp64_time_to_fit_s": t64,
        "speedup_vs_fp64": t64 / value if value else None,
        "sweeps_to_fit": {"mixed": sweeps_m, "fp64": s64},
        "reached": {"mixed": reached_m, "fp64": ok64},
        "fp64_path_timed_runs": path_m,
        "fit_error_vs_fp64": fit_err,
        "f_ref": f_ref, "target_fit": target,
        "mttkrp_tflops": tflops,
        "kernel_ms": kt,
        "roofline": {"bound": "mfma", "kernel": "chol_fwd_flow_kernel<double> (dataflow Cholesky "
                                                  "factorisation fused with the forward solve, FP64)",
                     "achieved": fac_achieved / 1e12, "peak": MFMA_PEAK["f64"] / 1e12,
                     "unit": "TFLOP/s", "frac": fac_achieved / MFMA_PEAK["f64"],
                     # the counters were taken at N=800, R_cp=4000 only
                     "traffic": (measured_traffic("chol_fwd_flow_kernel<double>")
                                 if (N, Rc) == (800, 4000) else None),
                     "avg_launch_us": per_launch_ms * 1e3, "launches_per_mode": launches},
        "roofline_core_product": {"bound": "mfma", "kernel": "pair split + gemm_split_dma_kernel (core product, "
                                                            "split BF16, useful flops)",
                                  "achieved": core_achieved / 1e12, "peak": MFMA_PEAK["bf16"] / 1e12,
                                  "unit": "TFLOP/s", "frac": core_achieved / MFMA_PEAK["bf16"],
                                  "executed": core_executed / 1e12,
                                  "executed_frac": core_executed / MFMA_PEAK["bf16"],
                                  "avg_launch_us": core_ms * 1e3},
        "sweep_ms_from_kernels": sweep_ms,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def sweep_flops(n, r_thc, r_cp):
    """Useful flops of one sweep: MTTKRP, Gram SYRKs, Cholesky, triangular solves."""
    return (mttkrp_flops(n, r_thc, r_cp) + r_cp * r_cp * sum(n) + 4.0 / 3.0 * r_cp ** 3
            + 2.0 * r_cp * r_cp * sum(n))


def bench_lt(args):
    """48 CPDs (3 systems x 16 Laplace points) of uneven size as one grouped
    sweep; throughput against the same CPDs run one after another, and the
    time for all of them to converge (per-problem stopping rule)."""
    import torch
    from paper_2502_17683_amd import CPD, CPDBatch, lt_batch_problems
    from synth import make_lt_system, init_factors, lt_points, LT_SYSTEMS

    systems = [make_lt_system(o, v, i) for i, (o, v) in enumerate(LT_SYSTEMS)]
    problems, meta = lt_batch_problems(systems, lt_points(),
                                       init_fn=lambda dims, r, idx: init_factors(dims, r, 1000 + idx))
    shapes = [([int(x.shape[0]) for x in p["X"]], int(p["Z"].shape[0]), p["r_cp"]) for p in problems]
    useful = sum(sweep_flops(*sh) for sh in shapes)
    mtt = sum(mttkrp_flops(*sh) for sh in shapes)
    K = args.lt_sweeps
    res = {}
    from paper_2502_17683_amd import CpdError
    precisions = [x for x in args.lt_precisions.split(",") if x]
    if not args.lt_batched_only and not {"mixed", "fp64"} <= set(precisions):
        raise SystemExit("--lt-precisions must include mixed and fp64 unless --lt-batched-only is given")
    for prec in precisions:
        b = CPDBatch(problems, precision=prec, tol=0.0, fit_floor=0.0, autotune=True,
                     fit_every=args.fit_every)
        try:
            b.sweep(3)
        except CpdError as e:
            # all-FP32 (Cholesky included) cannot factor the normal matrices of
            # the large-t problems, whose condition estimates reach ~1e12
            res[prec] = {"error": str(e)}
            b.close()
            log(f"[bench-lt] batched {prec}: {e}")
            continue
        torch.cuda.synchronize()
        # asynchronous sweeps (one graph launch each, the damped retry inside
        # the graph), then the default synchronised ones (the fused solve,
        # a host check per sweep, replay on a failed pivot)
        t0 = time.perf_counter()
        b.sweep(K, sync=False)
        torch.cuda.synchronize()
        ms_async = (time.perf_counter() - t0) * 1e3 / K
        t0 = time.perf_counter()
        b.sweep(K)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / K
        res[prec] = {"ms_per_batched_sweep": ms, "ms_per_batched_sweep_async": ms_async, "sweeps_per_s": 1e3 / ms,
                     "useful_tflops": useful / (ms * 1e-3) / 1e12}
        if prec == "mixed":
            res[prec]["autotune"] = b.autotune_log()
            res[prec]["promoted_to_fp64"] = sum(b.stats(i)["fp64_path"] for i in range(len(problems)))
        b.close()
        log(f"[bench-lt] batched {prec}: {ms:.3f} ms/sweep (asynchronous sweeps {ms_async:.3f})")
    if args.lt_batched_only:
        print(json.dumps({"metric": "batched LT CP-ALS sweep time (ms), 1 MI355X",
                          "value": res.get("mixed", {}).get("ms_per_batched_sweep"), "unit": "ms", "n_gpus": 1,
                          "steps": K, "higher_is_better": False, "data": "synthetic",
                          "config": {"workload": "48 LT CPDs, batched sweeps only", "fit_every": args.fit_every},
                          "per_precision": res}), flush=True)
        return
    # the same 48 CPDs one after another (one plan each, graph-replayed sweeps)
    for prec in ("mixed", "fp64"):
        plans = [CPD(p["X"], p["Z"], p["r_cp"], p["init"], precision=prec, tol=0.0, fit_floor=0.0,
                     fit_every=args.fit_every) for p in problems]
        for c in plans:
            c.sweep(3)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for c in plans:
            c.sweep(K, sync=False)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / K
        res[prec]["sequential_ms_per_sweep"] = ms
        res[prec]["batched_speedup_vs_sequential"] = ms / res[prec]["ms_per_batched_sweep"]
        for c in plans:
            c.close()
        log(f"[bench-lt] sequential {prec}: {ms:.3f} ms per sweep of all 48")
    # time to converge every CPD (tol 1e-4), batched, mixed vs FP64
    conv = {}
    finals = {}
    for prec in ("mixed", "fp64"):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b = CPDBatch(problems, precision=prec, tol=1e-4, fit_floor=1e-7, fit_every=args.fit_every)
        fits = b.sweep(args.max_sweeps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        _, done, sw = b.states()
        finals[prec] = [f[-1] for f in fits]
        conv[prec] = {"seconds": dt, "all_converged": bool(all(done)), "sweeps_max": int(max(sw)),
                      "sweeps_total": int(sum(sw))}
        b.close()
        log(f"[bench-lt] converge {prec}: {dt:.3f}s max sweeps {max(sw)}")
    rel = [abs(a - b) / b for a, b in zip(finals["mixed"], finals["fp64"]) if b > 0]
    out = {
        "metric": "batched LT CP-ALS sweep time (ms) and time to converge all CPDs (s), 1 MI355X",
        "value": res["mixed"]["ms_per_batched_sweep"], "unit": "ms", "n_gpus": 1, "steps": K,
        "higher_is_better": False, "data": "synthetic",
        "dtype": "bf16-split(fp32 acc)+f64",
        "config": {"workload": "48 LT CPDs: (o,v) in (20,100),(40,200),(80,400) x 16 Laplace points "
                               "0.01-20, R_thc=4(o+v), R_cp=2(o+v)", "fit_every": args.fit_every,
                   "useful_gflop_per_batched_sweep": useful / 1e9, "mttkrp_gflop": mtt / 1e9},
        "per_precision": res,
        "converge_tol_1e-4": conv,
        "final_fit_rel_diff_mixed_vs_fp64": {"max": max(rel), "median": float(np.median(rel))},
        "speedup_converge_mixed_vs_fp64": conv["fp64"]["seconds"] / conv["mixed"]["seconds"],
    }
    print(json.dumps(out), flush=True)


def exchange_flops(o, v, r_thc, r_cp, n_points):
    """Useful flops of one exchange call: the four projections, the Z
    product and the three double-term overlaps, over all points."""
    L = n_points * r_cp
    return 2.0 * r_thc * L * (2 * o + 2 * v) + 2.0 * r_thc * r_thc * L + 2.0 * r_cp * L * (2 * o + v)


def bench_exchange(args):
    """Robust CPD+THC LT-MP2 exchange energy (k_single, k_double and E_K at
    16 Laplace points) of the three systems of the batched workload.  value:
    summed milliseconds per call of the three systems, inputs resident in
    HBM.  Roofline: the Z product Y = Z (W2 o W3) of the largest system
    (the Hadamard product formed beforehand, as in the library call),
    timed with hipEvents around the same library product on the stream it
    runs on.  CPU baseline: the oracle on the largest system."""
    import ctypes
    import multiprocessing
    import torch
    from paper_2502_17683_amd import (lt_exchange, lt_exchange_workspace_bytes, lt_mp2, lt_mp2_workspace_bytes,
                                      CPD, _lib)
    from synth import make_lt_system, init_factors, lt_quadrature, LT_SYSTEMS

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    ts, w = lt_quadrature()
    npt = len(ts)
    per_system, total_ms, total_flops = [], 0.0, 0.0
    largest = None
    for si, (o, v) in enumerate(LT_SYSTEMS):
        Xo, Xv, Z, eo, ev = make_lt_system(o, v, si)
        r_thc, r_cp = Z.shape[0], 2 * (o + v)
        F = init_factors([o, v, o, v], r_cp, 1000 + 16 * si)
        d = [torch.as_tensor(a, device=dev) for a in (Xo, Xv, Z, eo, ev)]
        Fd = [torch.as_tensor(f, device=dev) for f in F]
        lam = torch.ones(r_cp, dtype=torch.float64, device=dev)
        ws = torch.empty(lt_exchange_workspace_bytes(o, v, r_thc, r_cp, npt), dtype=torch.uint8, device=dev)
        for _ in range(args.warmup + 1):
            lt_exchange(*d, ts, w, Fd, lam, workspace=ws)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.steps):
            k1, k2, ek = lt_exchange(*d, ts, w, Fd, lam, workspace=ws)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.steps
        fl = exchange_flops(o, v, r_thc, r_cp, npt)
        total_ms += ms
        total_flops += fl
        del ws
        # the THC LT-MP2 terms of the same system: Coulomb alone, then with
        # the THC exchange (the dense (ia|jb) route the CPD avoids)
        mp2_ms = {}
        for with_k in (False, True):
            wsm = torch.empty(lt_mp2_workspace_bytes(o, v, r_thc, npt, with_k, True), dtype=torch.uint8,
                              device=dev)
            for _ in range(args.warmup + 1):
                lt_mp2(*d, ts, w, thc_exchange=with_k, z_symmetric=True, workspace=wsm)
            torch.cuda.synchronize()
            reps = max(1, args.steps // 2) if with_k else args.steps
            e0.record(stream)
            for _ in range(reps):
                _, _, en = lt_mp2(*d, ts, w, thc_exchange=with_k, z_symmetric=True, workspace=wsm)
            e1.record(stream)
            torch.cuda.synchronize()
            mp2_ms[with_k] = e0.elapsed_time(e1) / reps
            del wsm
        thc_k_ms = mp2_ms[True] - mp2_ms[False]
        per_system.append({"o": o, "v": v, "r_thc": r_thc, "r_cp": r_cp, "ms": ms,
                           "useful_tflops": fl / (ms * 1e-3) / 1e12, "e_k": float(ek.cpu()[0]),
                           "coulomb_ms": mp2_ms[False], "thc_exchange_ms": thc_k_ms,
                           "robust_vs_thc_exchange_speedup": thc_k_ms / ms})
        log(f"[bench-exchange] ({o},{v}) R_thc={r_thc} R_cp={r_cp}: robust exchange {ms:.3f} ms/call "
            f"{fl / (ms * 1e-3) / 1e12:.1f} TF/s; THC Coulomb {mp2_ms[False]:.3f} ms; THC exchange "
            f"{thc_k_ms:.3f} ms ({thc_k_ms / ms:.1f}x the robust one)")
        largest = (Xo, Xv, Z, eo, ev, F, d, o, v, r_thc, r_cp)

    # the Z product of the largest system (Y = Z S2, S2 = W2 o W3 formed
    # beforehand) through the same library product
    Xo, Xv, Z, eo, ev, F, d, o, v, r_thc, r_cp = largest
    L = npt * r_cp
    lib = _lib.load()
    g = torch.Generator(device="cpu").manual_seed(5)
    B1 = torch.randn(r_thc, L, dtype=torch.float64, generator=g).to(dev)
    C = torch.empty(r_thc, L, dtype=torch.float64, device=dev)
    vp = ctypes.c_void_p
    sp = vp(stream.cuda_stream)

    def zprod():
        _lib.check(lib.cpd_test_gemm(0, r_thc, L, r_thc, vp(d[2].data_ptr()), r_thc, 0, vp(B1.data_ptr()),
                                     None, L, 0, vp(C.data_ptr()), L, sp), "cpd_test_gemm")
    zprod()
    torch.cuda.synchronize()
    reps = 10
    e0.record(stream)
    for _ in range(reps):
        zprod()
    e1.record(stream)
    torch.cuda.synchronize()
    z_ms = e0.elapsed_time(e1) / reps
    z_flops = 2.0 * r_thc * r_thc * L
    z_achieved = z_flops / (z_ms * 1e-3) / 1e12
    del B1, C

    # accuracy (the paper's comparison): a CPD of each bare tensor by FP64
    # CP-ALS (stopping rule 1e-4 or --accuracy-sweeps), then the THC LT-MP2
    # exchange energy against the robust and the single-CPD ones
    accuracy = []
    batch_facs = None
    if args.accuracy_sweeps > 0:
        # the batched per-point CPDs (one per system and Laplace point, of the
        # scaled tensors), as the batched workload fits them, in FP64
        from paper_2502_17683_amd import CPDBatch, lt_batch_problems
        systems = [make_lt_system(o, v, si) for si, (o, v) in enumerate(LT_SYSTEMS)]
        problems, _ = lt_batch_problems(systems, ts,
                                        init_fn=lambda dims, r, idx: init_factors(dims, r, 1000 + idx))
        b = CPDBatch(problems, precision="fp64", tol=1e-4, fit_floor=1e-7)
        b.sweep(args.accuracy_sweeps)
        batch_facs = [b.factors(i) for i in range(len(problems))]
        b.close()
        del problems
    for si, (o, v) in enumerate(LT_SYSTEMS if args.accuracy_sweeps > 0 else ()):
        Xo, Xv, Z, eo, ev = make_lt_system(o, v, si)
        r_thc, r_cp = Z.shape[0], 2 * (o + v)
        d = [torch.as_tensor(a, device=dev) for a in (Xo, Xv, Z, eo, ev)]
        c = CPD([d[0], d[1], d[0], d[1]], d[2], r_cp, init_factors([o, v, o, v], r_cp, 1000 + 16 * si),
                precision="fp64", tol=1e-4, fit_floor=1e-7)
        fits = c.sweep(args.accuracy_sweeps)
        Fd, lam = c.factors()
        c.close()
        k1, k2, ek = lt_exchange(*d, ts, w, Fd, lam)
        _, _, en = lt_mp2(*d, ts, w, thc_exchange=True, z_symmetric=True)
        e_j, e_thc = float(en[0]), float(en[1])
        e_rob = float(ek[0])
        e_single = -float(np.sum(w * k1.cpu().numpy()))
        mine = batch_facs[si * npt:(si + 1) * npt]
        _, _, ekp = lt_exchange(*d, ts, w, Fd, lam, E=[f for f, _ in mine], lam_e=[lk for _, lk in mine])
        e_rob_pp = float(ekp[0])
        accuracy.append({"o": o, "v": v, "cpd_sweeps": len(fits), "cpd_fit": float(fits[-1]),
                         "E_J": e_j, "E_K_thc": e_thc, "E_K_robust": e_rob, "E_K_single": e_single,
                         "E_K_robust_batched_cpds": e_rob_pp,
                         "rel_err_robust": (e_rob - e_thc) / abs(e_thc),
                         "rel_err_single": (e_single - e_thc) / abs(e_thc),
                         "rel_err_robust_batched_cpds": (e_rob_pp - e_thc) / abs(e_thc),
                         "rel_err_total_robust": (e_rob - e_thc) / abs(e_j + e_thc)})
        log(f"[bench-exchange] accuracy ({o},{v}): CPD fit {fits[-1]:.3e} after {len(fits)} sweeps; "
            f"E_K THC {e_thc:.8e} robust err {(e_rob - e_thc) / abs(e_thc):.2e} single err "
            f"{(e_single - e_thc) / abs(e_thc):.2e} robust with the batched CPDs "
            f"{(e_rob_pp - e_thc) / abs(e_thc):.2e}")

    cpu = None
    if not args.no_cpu:
        sys.path.insert(0, ROOT)
        from oracle import exchange as ox
        cores = int(os.environ.get("OMP_NUM_THREADS", multiprocessing.cpu_count()))
        t0 = time.perf_counter()
        ox.exchange_terms(Xo, Xv, Z, F, np.ones(r_cp), eo, ev, ts)
        dt = time.perf_counter() - t0
        cpu = {"value": dt * 1e3, "unit": "ms", "cores": cores, "kind": "oracle",
               "sample": f"one full call of the largest system ({o},{v}), 16 points"}
        log(f"[bench-exchange] CPU oracle ({o},{v}): {dt * 1e3:.1f} ms on {cores} threads")

    out = {
        "metric": "robust CPD+THC LT-MP2 exchange energy, time per call summed over the three systems (ms), "
                  "1 MI355X",
        "value": total_ms, "unit": "ms", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "higher_is_better": False, "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "exchange energy of the systems (o,v) in (20,100),(40,200),(80,400); "
                               "R_thc=4(o+v), R_cp=2(o+v), 16 Laplace points 0.01-20 with log-trapezoid "
                               "weights; CPD = seeded factors (the cost does not depend on their values)"},
        "useful_tflops": total_flops / (total_ms * 1e-3) / 1e12,
        "per_system": per_system,
        "accuracy_vs_thc_exchange": accuracy,
        "roofline": {"bound": "mfma", "kernel": "gemm_dma_kernel<false,false,false>: FP64 Z product Y = Z (W2 o W3), largest system",
                     "achieved": z_achieved, "peak": MFMA_PEAK["f64"] / 1e12, "unit": "TFLOP/s",
                     "frac": z_achieved * 1e12 / MFMA_PEAK["f64"],
                     "traffic": measured_traffic("gemm_dma_kernel<false,false,false>",
                                                 "exchange_zproduct_traffic_lt80x400.md"),
                     "avg_launch_us": z_ms * 1e3,
                     "shape": [r_thc, L, r_thc]},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def bench_tied(args):
    """Particle-tied CPD (F1 = F0, F3 = F2, symmetric ALS) against the
    four-factor CPD at the headline shape, FP64 (the tied model has no split
    BF16 path): time per sweep and the fit after --ref-sweeps sweeps, both
    from the same initial factors (modes 0 and 2 of the usual draw)."""
    import torch
    from paper_2502_17683_amd import CPD
    from synth import make_thc, init_factors, init_factors_uniform
    N, Rt, Rc = args.n, args.r_thc, args.r_cp
    dev = torch.device("cuda:0")
    X, Z = make_thc(N, Rt, args.seed)
    init = (init_factors_uniform if args.init == "uniform" else init_factors)([N] * 4, Rc, args.seed + 1000)
    Xd, Zd = torch.as_tensor(X, device=dev), torch.as_tensor(Z, device=dev)
    Id = [torch.as_tensor(f, device=dev) for f in init]
    tied_init = [Id[0], Id[0], Id[2], Id[2]]
    out = {}
    for name, tie, ini in (("four_factor", False, tied_init), ("tied", True, tied_init)):
        c = CPD(Xd, Zd, Rc, ini, precision="fp64", tol=0.0, fit_floor=0.0, tied=tie)
        c.sweep(2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        c.sweep(args.steps * 4, sync=False)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / (args.steps * 4)
        c.close()
        c = CPD(Xd, Zd, Rc, ini, precision="fp64", tol=0.0, fit_floor=0.0, tied=tie)
        fits = c.sweep(args.ref_sweeps)
        c.close()
        out[name] = {"ms_per_sweep": ms, "fit_after": fits[-1], "sweeps": len(fits),
                     "best_fit": min(fits), "fit_at_10": fits[min(9, len(fits) - 1)]}
        log(f"[bench-tied] {name}: {ms:.2f} ms/sweep, fit after {len(fits)} sweeps {fits[-1]:.6f}")
    line = {
        "metric": "particle-tied vs four-factor CP-ALS, FP64, time per sweep (ms) and fit after a fixed sweep count",
        "value": out["tied"]["ms_per_sweep"], "unit": "ms", "n_gpus": 1, "higher_is_better": False,
        "data": "synthetic", "dtype": "f64",
        "config": {"workload": f"THC CP-ALS N={N}, R_thc={Rt}, R_cp={Rc}, seed {args.seed}, init {args.init}, "
                               f"{args.ref_sweeps} sweeps"},
        "per_model": out,
        "sweep_time_ratio_tied_vs_four_factor": out["tied"]["ms_per_sweep"] / out["four_factor"]["ms_per_sweep"],
    }
    print(json.dumps(line), flush=True)


def bench_df(args):
    """CP-ALS on the DF loss (eq. df_loss, run through the exact THC form with
    R_thc = n^2) against CP-ALS on the THC loss (eq. lossF, R_thc = 4n), FP64,
    n = 50, 100, 200, R_cp = 2n, n_aux = 3n.  The DF tensor is the THC
    stand-in with its core truncated to n_aux eigenpairs, so the two losses
    describe nearly the same tensor.  Per sweep: O(n^4 R_cp) against
    O(n^3 R_cp)."""
    import torch
    from paper_2502_17683_amd import CPD, df_to_thc
    from synth import make_thc, make_df, init_factors
    dev = torch.device("cuda:0")
    rows = []
    for n in (50, 100, 200):
        r_cp, naux = 2 * n, 3 * n
        X, Z = make_thc(n, 4 * n, args.seed)
        B = make_df(n, naux, args.seed)
        init = [torch.as_tensor(f, device=dev) for f in init_factors([n] * 4, r_cp, args.seed + 1000)]
        Bd = torch.as_tensor(B, device=dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        X0, X1, Zd, nrm = df_to_thc(Bd, n)
        torch.cuda.synchronize()
        conv_ms = (time.perf_counter() - t0) * 1e3
        res = {"n": n, "r_cp": r_cp, "n_aux": naux, "df_to_thc_ms": conv_ms}
        for name, Xs, Zs, nr in (("df", [X0, X1, X0, X1], Zd, nrm),
                                 ("thc", torch.as_tensor(X, device=dev), torch.as_tensor(Z, device=dev), None)):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            c = CPD(Xs, Zs, r_cp, init, precision="fp64", tol=0.0, fit_floor=0.0, norm2=nr)
            torch.cuda.synchronize()
            init_ms = (time.perf_counter() - t0) * 1e3
            c.sweep(2)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            c.sweep(10, sync=False)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3 / 10
            fits = c.sweep(20)
            c.close()
            res[name] = {"r_thc": int(Zs.shape[0]), "ms_per_sweep": ms, "fit_after_32": fits[-1], "init_ms": init_ms}
        res["df_vs_thc_sweep_time"] = res["df"]["ms_per_sweep"] / res["thc"]["ms_per_sweep"]
        rows.append(res)
        log(f"[bench-df] n={n}: DF (R_thc={n * n}) {res['df']['ms_per_sweep']:.2f} ms/sweep, THC (R_thc={4 * n}) "
            f"{res['thc']['ms_per_sweep']:.2f} ms/sweep ({res['df_vs_thc_sweep_time']:.1f}x); fits "
            f"{res['df']['fit_after_32']:.4f} / {res['thc']['fit_after_32']:.4f}")
        del X0, X1, Zd, Bd, nrm
        torch.cuda.empty_cache()
    line = {
        "metric": "CP-ALS sweep time (ms), DF loss vs THC loss, FP64, 1 MI355X",
        "value": rows[-1]["df_vs_thc_sweep_time"], "unit": "ratio", "n_gpus": 1, "higher_is_better": False,
        "data": "synthetic", "dtype": "f64",
        "config": {"workload": "n = 50, 100, 200; R_cp = 2n; DF: n_aux = 3n, R_thc = n^2 (exact THC form); "
                               "THC: R_thc = 4n"},
        "per_n": rows,
    }
    print(json.dumps(line), flush=True)


def bench_warmstart(args):
    """Train the warm-start network on converged CPDs (N=100, R_thc=500,
    R_cp=400) and compare sweeps and wall time to the random start's best
    fit on held-out seeds at N=100 and N=400."""
    import torch
    from paper_2502_17683_amd import CPD, CPDBatch, WarmStartMLP, training_set, ws_init
    from synth import make_thc, init_factors, mlp_init_params, minibatch_order

    dev = torch.device("cuda:0")
    N, Rt, Rc = 100, 500, 400
    t0 = time.perf_counter()
    train = []
    for k in range(args.ws_train):
        X, Z = make_thc(N, Rt, 10000 + k)
        train.append({"X": X, "Z": Z, "r_cp": Rc, "init": init_factors([N] * 4, Rc, 11000 + k)})
    t_gen = time.perf_counter() - t0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    parts = []
    for a in range(0, len(train), 256):
        parts.append(training_set(train[a:a + 256], sweeps=300, tol=1e-4, chunk=64))
        torch.cuda.synchronize()
        log(f"[bench-ws] labelled {min(a + 256, len(train))}/{len(train)} training CPDs "
            f"({time.perf_counter() - t0:.1f}s)")
    data = tuple(torch.cat([q[i] for q in parts]) for i in range(4))
    del parts
    torch.cuda.synchronize()
    t_label = time.perf_counter() - t0
    del train
    net = WarmStartMLP(mlp_init_params(7))
    order = minibatch_order(int(data[0].shape[0]), 3)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    losses = net.train(data, order, batch_rows=8192, lr=2e-3, epochs=20)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    packed = net.pack()
    log(f"[bench-ws] generated {args.ws_train} inputs in {t_gen:.1f}s, labelled in {t_label:.1f}s, "
        f"trained {len(losses)} steps in {t_train:.2f}s, loss {losses[0]:.3f} -> {losses[-1]:.3f}")

    def evaluate(n, r_thc, r_cp, seeds, budget, chunk):
        """Held-out problems in batches of `chunk`: the FP64 random start's
        best fit over `budget` sweeps x (1 + 1e-4) is each problem's target
        (untimed reference); then the random, learned and heuristic starts
        each run as one FP64 batch whose problems stop on the device at their
        targets (timed, warm-start inference included).  Returns per kind
        the sweeps each problem needed (None: missed within the budget) and
        the summed wall time."""
        seeds = list(seeds)
        sweeps = {k: [] for k in ("random", "learned", "heuristic")}
        secs = {k: 0.0 for k in sweeps}
        for a in range(0, len(seeds), chunk):
            part = seeds[a:a + chunk]
            base = []
            for seed in part:
                X, Z = make_thc(n, r_thc, seed)
                rnd = init_factors([n] * 4, r_cp, seed + 1000)
                base.append({"X": torch.as_tensor(X, device=dev), "Z": torch.as_tensor(Z, device=dev),
                             "r_cp": r_cp, "init": [torch.as_tensor(f, device=dev) for f in rnd]})
            ref = CPDBatch(base, precision="fp64", tol=0.0, fit_floor=0.0)
            rf = ref.sweep(budget)
            ref.close()
            targets = [min(f) * (1.0 + 1e-4) for f in rf]
            for kind in sweeps:
                torch.cuda.synchronize()
                t = time.perf_counter()
                probs = base
                if kind != "random":
                    probs = [dict(b, init=ws_init(b["X"], b["Z"], r_cp, packed=packed if kind == "learned" else None,
                                                  noise=b["init"])[0]) for b in base]
                bt = CPDBatch(probs, precision="fp64", tol=0.0, fit_floor=0.0, fit_targets=targets)
                bt.sweep(budget)
                last, _, sw = bt.states()
                bt.close()
                torch.cuda.synchronize()
                secs[kind] += time.perf_counter() - t
                sweeps[kind] += [int(sw[i]) if last[i] <= targets[i] else None for i in range(len(part))]
            log(f"[bench-ws] N={n}: {a + len(part)}/{len(seeds)} held-out problems; median sweeps so far " +
                ", ".join(f"{k} {np.median([x if x is not None else budget + 1 for x in v]):.1f}"
                          for k, v in sweeps.items()))
            del base
        return sweeps, secs

    def summary(res, budget):
        sweeps, secs = res
        out = {}
        for kind, v in sweeps.items():
            sw = [x if x is not None else budget + 1 for x in v]
            out[kind] = {"median_sweeps": float(np.median(sw)), "mean_sweeps": float(np.mean(sw)),
                         "reached": int(sum(x is not None for x in v)), "of": len(v),
                         "wall_s_total": secs[kind], "wall_s_per_cpd": secs[kind] / max(len(v), 1)}
        out["speedup_wall_learned_vs_random"] = secs["random"] / secs["learned"]
        out["speedup_wall_learned_vs_heuristic"] = secs["heuristic"] / secs["learned"]
        out["learned_fewer_or_equal_sweeps_than_heuristic"] = int(sum(
            (l if l is not None else budget + 1) <= (h if h is not None else budget + 1)
            for l, h in zip(sweeps["learned"], sweeps["heuristic"])))
        return out

    small = evaluate(N, Rt, Rc, range(20000, 20000 + args.ws_heldout), args.ws_budget, 100)
    large = evaluate(400, 2000, 1600, range(20000, 20000 + args.ws_heldout_large), args.ws_budget, 16)
    out = {
        "metric": "warm-start sweeps and wall time to the random start's best fit x (1+1e-4), 1 MI355X",
        "value": summary(small, args.ws_budget)["learned"]["wall_s_per_cpd"], "unit": "s", "n_gpus": 1,
        "higher_is_better": False, "data": "synthetic", "dtype": "f64 CP-ALS, f32 train / bf16 infer",
        "config": {"workload": f"train {args.ws_train} converged CPDs N=100 R_thc=500 R_cp=400 "
                               f"(seeds 10000+), held-out {args.ws_heldout} at N=100 and "
                               f"{args.ws_heldout_large} at N=400 R_thc=2000 R_cp=1600 (seeds 20000+), "
                               f"budget {args.ws_budget} sweeps, blend sigma 0.25"},
        "train": {"rows": int(data[0].shape[0]), "steps": len(losses), "seconds": t_train,
                  "label_seconds": t_label, "loss_first": float(losses[0]), "loss_last": float(losses[-1])},
        "heldout_n100": summary(small, args.ws_budget),
        "heldout_n400": summary(large, args.ws_budget),
    }
    print(json.dumps(out), flush=True)


def bench_kernels(args):
    """Per-kernel times of the sweep's kernel families (cpd_kernel_times:
    one warm-up and --steps repetitions each) for split BF16 and FP64 at the
    headline shape; no time-to-fit runs.  Short enough to run under
    hardware-counter collection."""
    import torch
    from paper_2502_17683_amd import CPD
    from synth import make_thc, init_factors
    N, Rt, Rc = args.n, args.r_thc, args.r_cp
    dev = torch.device("cuda:0")
    X, Z = make_thc(N, Rt, args.seed)
    init = init_factors([N] * 4, Rc, args.seed + 1000)
    Xd, Zd = torch.as_tensor(X, device=dev), torch.as_tensor(Z, device=dev)
    Id = [torch.as_tensor(f, device=dev) for f in init]
    kt = {}
    for prec in ("mixed", "fp64"):
        c = CPD(Xd, Zd, Rc, Id, precision=prec, tol=0.0, fit_floor=0.0)
        kt[prec] = c.kernel_times(reps=max(args.steps, 1))
        c.close()
        log(f"[bench-kernels] {prec}: {kt[prec]}")
    out = {"metric": "per-kernel time (ms) of the sweep's kernel families, 1 MI355X", "value": None, "unit": "ms",
           "n_gpus": 1, "steps": args.steps, "higher_is_better": False, "data": "synthetic",
           "config": {"workload": f"THC CP-ALS kernel families, N={N}, R_thc={Rt}, R_cp={Rc}"},
           "kernel_ms": kt}
    print(json.dumps(out), flush=True)


def bench_combined(args):
    """The three forms together on the batched Laplace workload (48 CPDs:
    (o,v) = (20,100), (40,200), (80,400) x 16 points): split BF16, started
    from the learned warm start, each CPD run until its fit reaches its own
    FP64 reference fit x (1 + 1e-4) (the plain FP64 batch from the random
    start, best fit over --comb-ref-sweeps sweeps), against that FP64 batch
    from the random start run to the same targets.  Each problem stops on
    the device once it reaches its target (cpd_desc.fit_target).  The
    network is trained on converged CPDs of other Laplace systems of the
    same sizes (system seeds 100+), generated by the library itself; the
    warm start's inference is inside the timed region.  A warm-started CPD
    that has not reached its target after --comb-cap sweeps falls back to
    the plain method (FP64 from the random start), also timed.  Also reported: the
    two forms alone (split BF16 from the random start, FP64 from the
    warm start)."""
    import torch
    from paper_2502_17683_amd import CPDBatch, WarmStartMLP, lt_batch_problems, training_set, ws_init
    from synth import make_lt_system, init_factors, lt_points, LT_SYSTEMS, mlp_init_params, minibatch_order

    ts = lt_points()
    rnd_init = lambda dims, r, idx: init_factors(dims, r, 1000 + idx)
    systems = [make_lt_system(o, v, i) for i, (o, v) in enumerate(LT_SYSTEMS)]
    problems, meta = lt_batch_problems(systems, ts, init_fn=rnd_init)
    P = len(problems)
    log(f"[bench-comb] FP64 reference: {P} CPDs x {args.comb_ref_sweeps} sweeps")
    ref = CPDBatch(problems, precision="fp64", tol=0.0, fit_floor=0.0)
    ref_fits = ref.sweep(args.comb_ref_sweeps)
    ref.close()
    f_ref = [min(f for f in fs if f >= 0) for fs in ref_fits]
    # a reference fit at the matrix-free cancellation floor (~1e-7, where the
    # residual is a difference of O(1) terms) is met by reaching that floor
    floor = 1e-7
    targets = [max(f * (1.0 + 1e-4), floor) for f in f_ref]
    log(f"[bench-comb] reference fits {min(f_ref):.3e} .. {max(f_ref):.3e}, "
        f"{sum(f <= floor for f in f_ref)} at the floor")

    # training data: converged CPDs of other systems of the same sizes
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    feats = []
    for k in range(args.comb_train_sets):
        tsys = [make_lt_system(o, v, 100 + 3 * k + i) for i, (o, v) in enumerate(LT_SYSTEMS)]
        tprob, _ = lt_batch_problems(tsys, ts, init_fn=lambda dims, r, idx, k=k: init_factors(dims, r,
                                                                                          5000 + 64 * k + idx))
        feats.append(training_set(tprob, sweeps=400, tol=1e-4, chunk=len(tprob)))
    data = tuple(torch.cat([f[i] for f in feats]) for i in range(4))
    torch.cuda.synchronize()
    t_label = time.perf_counter() - t0
    net = WarmStartMLP(mlp_init_params(7))
    order = minibatch_order(int(data[0].shape[0]), 3)
    t0 = time.perf_counter()
    losses = net.train(data, order, batch_rows=8192, lr=2e-3, epochs=40)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    packed = net.pack()
    log(f"[bench-comb] labelled {args.comb_train_sets * P} CPDs in {t_label:.1f}s, trained {len(losses)} steps "
        f"in {t_train:.2f}s, loss {losses[0]:.3f} -> {losses[-1]:.3f}")

    def run(prec, warm, fit_every, fallback=False):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        probs, sources = problems, None
        if warm:
            probs, sources = [], []
            for pr in problems:
                init, src = ws_init(pr["X"], pr["Z"], pr["r_cp"], packed=packed, noise=pr["init"])
                probs.append(dict(pr, init=init))
                sources.append(src)
        b = CPDBatch(probs, precision=prec, tol=0.0, fit_floor=0.0, fit_every=fit_every, fit_targets=targets)
        b.sweep(args.comb_cap)
        last, done, sw = b.states()
        promoted = sum(b.stats(i)["fp64_path"] for i in range(P)) if prec == "mixed" else 0
        b.close()
        reached = [bool(last[i] <= targets[i]) for i in range(P)]
        t_first = time.perf_counter() - t0
        redo = [i for i in range(P) if not reached[i]] if fallback else []
        if redo:
            # the fallback of the warm start: a CPD that missed its target
            # within the cap is rerun by the plain method (FP64, random start)
            fb = CPDBatch([problems[i] for i in redo], precision="fp64", tol=0.0, fit_floor=0.0,
                          fit_targets=[targets[i] for i in redo])
            fb.sweep(args.comb_cap)
            flast, _, fsw = fb.states()
            fb.close()
            for j, i in enumerate(redo):
                last[i] = flast[j]
                sw[i] += fsw[j]
                reached[i] = bool(flast[j] <= targets[i])
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        gap = [(last[i] - f_ref[i]) / max(f_ref[i], floor) for i in range(P)]
        res = {"seconds": dt, "seconds_before_fallback": t_first, "fallback_reruns": redo,
               "reached": int(sum(reached)), "of": P, "sweeps": [int(x) for x in sw],
               "sweeps_max": int(max(sw)), "sweeps_total": int(sum(sw)), "fit_gap_vs_fp64_ref": gap,
               "fit_gap_max": float(max(gap)), "not_reached": [i for i in range(P) if not reached[i]]}
        if prec == "mixed":
            res["promoted_to_fp64"] = int(promoted)
        if sources is not None:
            res["init_source"] = {s: sources.count(s) for s in set(sources)}
        log(f"[bench-comb] {prec} {'warm' if warm else 'random'}: {dt:.3f}s, reached {sum(reached)}/{P}, "
            f"max sweeps {max(sw)}, total sweeps {sum(sw)}, max gap {max(gap):.2e}")
        return res

    run("fp64", False, 1)  # warm-up of the plan set-up paths
    base = run("fp64", False, 1)
    comb = run("mixed", True, args.fit_every, fallback=True)
    mixed_rnd = run("mixed", False, args.fit_every)
    fp64_warm = run("fp64", True, 1, fallback=True)
    ok = comb["reached"] == P
    out = {
        "metric": "batched LT CP-ALS wall time to every CPD's FP64 reference fit x (1+1e-4) (s), "
                  "split BF16 + learned warm start vs FP64 from random start, 1 MI355X",
        "value": comb["seconds"] if ok else None, "unit": "s", "n_gpus": 1, "steps": 1,
        "higher_is_better": False, "data": "synthetic", "dtype": "bf16-split(fp32 acc)+f64",
        "config": {"workload": "48 LT CPDs: (o,v) in (20,100),(40,200),(80,400) x 16 Laplace points 0.01-20, "
                               "R_thc=4(o+v), R_cp=2(o+v); targets = max(FP64 random-start best fit over "
                               f"{args.comb_ref_sweeps} sweeps x (1+1e-4), 1e-7); cap {args.comb_cap} sweeps",
                   "fit_every": args.fit_every, "train_sets": args.comb_train_sets},
        "speedup_vs_fp64_random": base["seconds"] / comb["seconds"],
        "all_reached": ok,
        "combined": comb, "fp64_random": base, "mixed_random": mixed_rnd, "fp64_warm": fp64_warm,
        "train": {"rows": int(data[0].shape[0]), "steps": len(losses), "seconds": t_train,
                  "label_seconds": t_label, "loss_first": float(losses[0]), "loss_last": float(losses[-1])},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
