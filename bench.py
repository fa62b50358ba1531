"""Benchmark of the MI355X rAPDHG hot path.

Workload: the large sparse random QP (n = 1e6 variables, m = 5e5 rows: 2.5e5
equality + 2.5e5 '>=' rows; A with 10 N(0,1) nonzeros per row; Q = S + S' with
S holding 5 N(0,1) off-diagonal nonzeros per row plus a diagonal making Q
diagonally dominant; c ~ N(0,1); x >= 0; b feasible from x0 ~ U(0,1)), FP64
CSR, seeded synthetic data standing in for the paper's large random-QP class.

One step = one qp_solve of ITERS iterations (eps = 0, so it never stops
early): ITERS x (dual kernel + primal kernel), a KKT evaluation of z and z-bar
every 64 iterations, the device-side restart / primal-weight / step-size
decision and restart application.  value = iterations per second over the K
timed steps.  Inputs are resident in HBM (copied at qp_create) before timing.

Also reported: hipEvent durations of the dual and primal phases recorded over
the timed region (settings.profile = 16: direct launches, events around both
phases of every 16th iteration on the library's stream), the roofline of the
dominant (primal) kernel from its algorithmic bytes, wall time to relKKT 1e-4
and 1e-6, and the CPU oracle's iteration rate on a bounded sample.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--iters ITERS]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "rAPDHG iters/s + time-to-1e-6 KKT; SpMV HBM GB/s % peak; warm vs cold"
HBM_PEAK_GBS = 8000.0  # MI355X published HBM3E bandwidth
# random FP64 gathers per second from a vector slice held in one XCD's L2, measured with a
# standalone probe kernel (column index + value streamed, one gather per entry)
GATHER_CEILING = 210e9


PROFILE_MD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles",
                          "panels_large_random_qp.md")
KERNEL_SRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2311_07710_amd",
                          "csrc", "qp_kernels.hip")


def measured_traffic():
    """HBM bytes per primal-phase launch from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE
    summary (scaled by the copy-kernel calibration), or None when the kernel source has
    changed since those counters were taken."""
    import hashlib
    try:
        text = open(PROFILE_MD).read()
        fields = dict(line[2:].split(": ", 1) for line in text.splitlines()
                      if line.startswith("- ") and ": " in line)
        sha = hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()
        if fields.get("kernel_source_sha256") != sha:
            return None
        return float(fields["traffic_primal_phase_bytes"])
    except (OSError, KeyError, ValueError):
        return None


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--iters", type=int, default=1024)
    ap.add_argument("--no-tol", action="store_true", help="skip the time-to-tolerance solves")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--graph", action="store_true",
                    help="time with graph replay instead of per-phase hipEvents")
    ap.add_argument("--profile-every", type=int, default=16,
                    help="time the phases of every k-th iteration with hipEvents")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched MPC section")
    ap.add_argument("--no-classes", action="store_true",
                    help="skip the seven synthetic classes at medium size")
    ap.add_argument("--no-ablation", action="store_true",
                    help="skip the Sec. 5 momentum/restart ablation")
    ap.add_argument("--no-warmstart", action="store_true",
                    help="skip the learned warm-start section")
    ap.add_argument("--ws-count", type=int, default=20000,
                    help="portfolio-family instances for the warm-start section")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one 256 MiB device-to-device copy first (a known-size reference "
                         "for rocprofv3 FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}): the solver has no "
              "multi-GPU path.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2311_07710_amd as qpa
    import qpgen

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.calibrate_copy:
        src = torch.empty(32 << 20, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log("[bench] calibration copy: 256 MiB read + 256 MiB written")
        del src, dst
    # measured streaming bandwidth: a plain 1 GiB device-to-device copy (read + write)
    src = torch.empty(128 << 20, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    copy_gbs = 0.0
    for _ in range(5):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        e1.synchronize()
        copy_gbs = max(copy_gbs, 2 * src.numel() * 8 / (e0.elapsed_time(e1) * 1e-3) / 1e9)
    del src, dst
    log(f"[bench] device copy (1 GiB read + 1 GiB written): {copy_gbs:.0f} GB/s")
    t = time.time()
    qp = qpgen.large_random_qp()
    log(f"[bench] generated n={qp.n} m={qp.m} nnzA={qp.a_nnz} nnzQ={qp.q_nnz} "
        f"in {time.time() - t:.1f}s")

    t = time.time()
    profile = 0 if args.graph else max(1, args.profile_every)
    settings = qpa.Settings(eps=0.0, max_iter=args.iters, profile=profile, use_graph=1)
    solver = qpa.Solver(qp, settings)
    create_s = time.time() - t
    nA, nQ = solver.norms()
    log(f"[bench] qp_create {create_s:.2f}s (incl. power iteration) ||A||={nA:.6g} ||Q||={nQ:.6g}")

    for w in range(args.warmup):
        solver.solve()
        log(f"[bench] warmup {w + 1}/{args.warmup} done")

    dual_ms = primal_ms = 0.0
    dual_n = primal_n = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters = 0
    for k in range(args.steps):
        _, _, r = solver.solve()
        iters += r["iterations"]
        if profile:
            p = solver.profile()
            dual_ms += p["dual_ms"]
            primal_ms += p["primal_ms"]
            dual_n += p["dual_launches"]
            primal_n += p["primal_launches"]
            dual_bytes, primal_bytes = p["dual_bytes"], p["primal_bytes"]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    log(f"[bench] timed {args.steps} steps x {args.iters} iterations in {elapsed:.3f}s")
    value = iters / elapsed
    ms_per_step = 1000.0 * elapsed / args.steps

    # the same solves replayed as hipGraphs without phase timing: with the KKT evaluation
    # every 64 iterations, and with one evaluation per step (the cost of the checks)
    replay = {}
    for ce in (64, args.iters):
        with qpa.Solver(qp, qpa.Settings(eps=0.0, max_iter=args.iters, check_every=ce,
                                         norm_A=nA, norm_Q=nQ)) as s4:
            s4.solve()
            torch.cuda.synchronize()
            t = time.perf_counter()
            n_it = sum(s4.solve()[2]["iterations"] for _ in range(3))
            torch.cuda.synchronize()
            replay[f"check_every_{ce}"] = n_it / (time.perf_counter() - t)
    log("[bench] graph replay: " + ", ".join(f"{k} {v:.0f} it/s" for k, v in replay.items()))

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "large sparse random QP, n=1e6, m=5e5 (half EQ, half GE), A 10 nnz/row, "
                        "Q diag-dominant ~11 nnz/row, x>=0, FP64 CSR (seed 2)",
            "n": qp.n, "m": qp.m, "nnz_A": qp.a_nnz, "nnz_Q": qp.q_nnz,
            "iters_per_step": args.iters, "check_every": 64,
            "timing": "graph replay" if args.graph else
                      f"direct launches; both phases of every {profile}th iteration timed with hipEvents",
        },
        "create_s": create_s,
        "iters_per_s_graph_replay": replay,
    }
    if profile and primal_n:
        d_avg = dual_ms / dual_n
        p_avg = primal_ms / primal_n
        p_gbs = primal_bytes / (p_avg * 1e-3) / 1e9
        d_gbs = dual_bytes / (d_avg * 1e-3) / 1e9
        # the phase's random FP64 gathers (one per nonzero of P) against the rate measured
        # for gathers that stay in one XCD's L2 (a standalone probe, 210 G/s)
        gathers_ps = (qp.q_nnz + qp.a_nnz) / (p_avg * 1e-3)
        out["roofline"] = {"bound": "hbm",
                           "kernel": "primal phase (k_panel_spmv<1> + k_primal_combine)",
                           "achieved": p_gbs,
                           "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": p_gbs / HBM_PEAK_GBS,
                           "traffic": measured_traffic(), "avg_us": 1000.0 * p_avg,
                           "algorithmic_bytes_per_launch": primal_bytes,
                           "copy_GBps": copy_gbs, "frac_of_copy": p_gbs / copy_gbs,
                           "gathers_per_s": gathers_ps,
                           "gather_ceiling_per_s": GATHER_CEILING,
                           "frac_of_gather_ceiling": gathers_ps / GATHER_CEILING}
        out["kernels"] = {
            "k_dual": {"avg_us": 1000.0 * d_avg, "bytes": dual_bytes, "GB/s": d_gbs,
                       "frac": d_gbs / HBM_PEAK_GBS, "launches": dual_n},
            "k_primal": {"avg_us": 1000.0 * p_avg, "bytes": primal_bytes, "GB/s": p_gbs,
                         "frac": p_gbs / HBM_PEAK_GBS, "launches": primal_n},
            "iteration_frac": (dual_bytes + primal_bytes) / ((d_avg + p_avg) * 1e-3) / 1e9
                              / HBM_PEAK_GBS,
        }
        log(f"[bench] k_dual {1000 * d_avg:.1f}us {d_gbs:.0f} GB/s | k_primal {1000 * p_avg:.1f}us "
            f"{p_gbs:.0f} GB/s")

    if not args.no_tol:
        tt = {}
        for eps in (1e-4, 1e-6):
            with qpa.Solver(qp, qpa.Settings(eps=eps, norm_A=nA, norm_Q=nQ, max_iter=200000,
                                             time_limit_s=120.0)) as s2:
                t = time.perf_counter()
                _, _, r = s2.solve()
                dt = time.perf_counter() - t
            tt[f"{eps:g}"] = {"seconds": dt, "iterations": r["iterations"],
                              "restarts": r["restarts"], "rel_kkt": r["rel_kkt"],
                              "status": r["status"]}
            log(f"[bench] to relKKT {eps:g}: {dt:.3f}s, {r['iterations']} iterations, "
                f"status {r['status']}, relKKT {r['rel_kkt']:.3e}")
        # the Sec. 6 configuration: Sec. 5 preprocessing before the iteration
        t = time.time()
        with qpa.Solver(qp, qpa.Settings(eps=1e-6, precondition=1, max_iter=200000,
                                         time_limit_s=120.0)) as s3:
            pre_create = time.time() - t
            t = time.perf_counter()
            _, _, r = s3.solve()
            dt = time.perf_counter() - t
        tt["1e-06 preconditioned"] = {"seconds": dt, "iterations": r["iterations"],
                                      "restarts": r["restarts"], "rel_kkt": r["rel_kkt"],
                                      "status": r["status"], "create_s": pre_create}
        log(f"[bench] to relKKT 1e-06 with Sec. 5 preprocessing: {dt:.3f}s, "
            f"{r['iterations']} iterations, status {r['status']} (create {pre_create:.2f}s)")
        out["time_to_tolerance"] = tt

    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(qp, log)

    solver.close()
    if not args.no_batch:
        out["batched_mpc"] = bench_batch(log)
    if not args.no_classes:
        out["classes"] = bench_classes(log)
    if not args.no_classes:
        out["infeasibility"] = bench_infeasibility(log)
    if not args.no_ablation:
        out["ablation"] = bench_ablation(log)
    if not args.no_warmstart:
        out["warm_start"] = bench_warmstart(log, args.ws_count)
    print(json.dumps(out), flush=True)


def cpu_baseline(qp, log):
    """The oracle (plain FP64 C, sequential sums in the paper's order) on the host: 1024
    rAPDHG iterations of the same instance (KKT evaluation every 64) with its threaded mode
    on the host's CPU share (row ranges split over OpenMP threads; every sum keeps its
    order, so the result is bitwise the one-thread one), and a one-thread run beside it."""
    import platform
    import subprocess
    import oracle
    ncpu = os.cpu_count() or 1
    share = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else ncpu
    threads = max(1, min(16, share))
    model = platform.processor() or ""
    try:
        for line in subprocess.run(["lscpu"], capture_output=True, text=True).stdout.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
    except OSError:
        pass
    onA, _ = oracle.norm_A(qp, 40, 1e-7)
    onQ, _ = oracle.norm_Q(qp, 40, 1e-7)
    rates = {}
    for th, n_it in ((threads, 1024), (1, 256)):
        oracle.set_threads(th)
        t = time.perf_counter()
        _, _, ro, _ = oracle.solve(qp, oracle.OracleSettings(eps=0.0, max_iter=n_it, norm_A=onA,
                                                             norm_Q=onQ))
        rates[th] = ro["iterations"] / (time.perf_counter() - t)
        log(f"[bench] cpu oracle {th} thread(s): {rates[th]:.2f} iters/s ({n_it} iterations)")
    # time to relKKT 1e-6 on all cores (the same solve the GPU's time_to_tolerance times)
    oracle.set_threads(threads)
    t = time.perf_counter()
    _, _, rt, _ = oracle.solve(qp, oracle.OracleSettings(eps=1e-6, norm_A=onA, norm_Q=onQ))
    tt = time.perf_counter() - t
    log(f"[bench] cpu oracle {threads} threads to relKKT 1e-6: {tt:.1f}s, "
        f"{rt['iterations']} iterations")
    oracle.set_threads(1)
    return {"value": rates[threads], "unit": "iters/s", "cores": threads, "kind": "oracle",
            "time_to_1e-6_s": tt, "time_to_1e-6_iterations": rt["iterations"],
            "sample": f"1024 rAPDHG iterations (KKT evaluated every 64) of the same full-size "
                      f"instance, C oracle on {threads} OpenMP threads (sums in fixed order)",
            "value_1_thread": rates[1], "sample_1_thread": "256 iterations, one thread",
            "host": {"nproc": ncpu, "cpu_share": share, "model": model}}


def bench_batch(log):
    """4096 MPC-style QPs (uneven sizes) to relKKT 1e-6 in one persistent launch per size
    class, against looping single-instance solves over a sample."""
    import numpy as np
    import paper_2311_07710_amd as qpa
    import qpgen
    t = time.time()
    batch = qpgen.mpc_batch(seed=4, count=4096)
    log(f"[bench] MPC batch generated in {time.time() - t:.1f}s "
        f"(sum n={batch.var_off[-1]}, sum m={batch.row_off[-1]})")
    import torch
    n_i = np.diff(batch.var_off)
    m_i = np.diff(batch.row_off)
    a_nnz = np.diff(batch.a_rowptr[batch.row_off].astype(np.int64))
    q_nnz = np.diff(batch.q_rowptr[batch.var_off].astype(np.int64))
    # bytes one iteration of instance i reads besides its LDS-resident iterates: the rows
    # of A and of P = [Q | -A'] (8 B value + 4 B column per nonzero, 4 B row pointers), and
    # c, l, u (24 B per variable), b and the row type (9 B per row).  The leading slices of
    # the rows come from the team's LDS cache where it has room, so as memory traffic this
    # is an upper bound.
    it_bytes = 12.0 * (2 * a_nnz + q_nnz) + 4.0 * (n_i + m_i + 2) + 24.0 * n_i + 9.0 * m_i
    # memory-side ceiling for this access pattern: a device copy of a buffer that the L2s
    # and the 256 MB MALL hold (64 MiB read + 64 MiB written, repeated)
    src = torch.empty(8 << 20, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(50):
        dst.copy_(src)
    torch.cuda.synchronize()
    mall_gbs = 50 * 2 * src.numel() * 8 / (time.perf_counter() - t) / 1e9
    del src, dst
    out = {"workload": "4096 MPC QPs, T~U{10..100}, n_x~U{4..12}, n_u~U{2..4}, FP64, eps 1e-6"}
    for pre in (1, 0):
        t = time.time()
        bs = qpa.BatchSolver(batch, qpa.Settings(eps=1e-6, precondition=pre))
        create_s = time.time() - t
        t = time.perf_counter()
        threads = bs.autotune(sample=128, iters=256)
        tune_s = time.perf_counter() - t
        # three solves; the one with the median time is reported (a solve's makespan
        # moves by a few percent with where the slowest instance's team starts)
        runs = []
        for _ in range(3):
            t = time.perf_counter()
            _, _, res = bs.solve()
            runs.append((time.perf_counter() - t, res))
        dts = [r[0] for r in runs]
        dt, res = sorted(runs, key=lambda r: r[0])[1]
        its = np.array([r["iterations"] for r in res], dtype=float)
        end = np.array([r["end_s"] for r in res])
        start = np.array([r["start_s"] for r in res])
        ok = int(sum(r["status"] == 0 for r in res))
        if pre:
            gA, gQ = bs.norms()
        bs.close()
        slow = int(np.argmax(its))
        moved = float(np.sum(its * it_bytes))
        row = {"instances_per_s": batch.count / dt, "seconds": dt, "seconds_runs": dts,
               "optimal": ok,
               "iterations_mean": float(its.mean()), "iterations_max": int(its.max()),
               "completion_s": {"p50": float(np.percentile(end, 50)),
                                "p99": float(np.percentile(end, 99)), "max": float(end.max())},
               "slowest": {"instance": slow, "iterations": int(its[slow]),
                           "n_plus_m": int(n_i[slow] + m_i[slow]), "start_s": float(start[slow]),
                           "end_s": float(end[slow]),
                           "us_per_iteration": 1e6 * float(end[slow] - start[slow]) / its[slow]},
               "threads_per_class": threads, "autotune_s": tune_s, "create_s": create_s,
               "memory_bytes_moved": moved, "GBps": moved / dt / 1e9}
        key = "preprocessed" if pre else "not_preprocessed"
        out[key] = row
        log(f"[bench] batched ({key}): {batch.count} instances in {dt:.3f}s "
            f"(median of {', '.join(f'{d:.3f}' for d in dts)}s) "
            f"({batch.count / dt:.0f}/s), {ok} optimal, threads {threads}; completion p50 "
            f"{row['completion_s']['p50']:.3f}s p99 {row['completion_s']['p99']:.3f}s max "
            f"{row['completion_s']['max']:.3f}s; slowest instance {slow}: {int(its[slow])} "
            f"iterations from {start[slow]:.3f}s to {end[slow]:.3f}s; "
            f"{row['GBps']:.0f} GB/s of matrix and data streams")
    pre = out["preprocessed"]
    sample = list(range(0, batch.count, 256))
    t = time.perf_counter()
    for i in sample:
        with qpa.Solver(batch.instance(i), qpa.Settings(eps=1e-6, norm_A=gA[i], norm_Q=gQ[i],
                                                         precondition=1)) as s:
            s.solve()
    st = time.perf_counter() - t
    log(f"[bench] looping qp_solve over {len(sample)} instances: {st:.2f}s "
        f"({len(sample) / st:.1f}/s)")
    out.update({"instances_per_s": pre["instances_per_s"], "seconds": pre["seconds"],
                "single_loop_instances_per_s": len(sample) / st,
                "single_loop_sample": len(sample),
                "speedup_vs_single_loop": pre["instances_per_s"] / (len(sample) / st),
                "roofline": {"bound": "latency",
                             "note": "each instance's iteration is a chain of dependent loads "
                                     "and barriers on one workgroup; the makespan is the "
                                     "slowest instance's iterations times its per-iteration "
                                     "latency; achieved counts every matrix and data byte an "
                                     "iteration reads, also those served by the LDS matrix "
                                     "cache, so as memory traffic it is an upper bound",
                             "achieved": pre["GBps"], "peak": mall_gbs, "unit": "GB/s",
                             "peak_kind": "measured device copy of a 64 MiB buffer (L2/MALL "
                                          "resident), read + write",
                             "frac": pre["GBps"] / mall_gbs}})
    return out


def bench_ablation(log):
    """Sec. 5's comparison of PDHG, accelerated PDHG, restarted PDHG and rAPDHG (Tables
    1-2): solved counts and shifted geometric means of iterations (shift 10, unsolved =
    the 200000-iteration limit) to relKKT 1e-3 and 1e-6, with the Sec. 5 preprocessing,
    zero starts, the halving restart for the restarted methods, and the tuned
    fixed-frequency leg (rAPDHG restarted every K in {10, 100, 1000}, the best K per
    instance).  Every method is measured at the average, as Algorithm 1 outputs it.  The
    Sec. 6 adaptive rule is run beside them for context.  Workload: a synthetic stand-in
    for a mixed test set, 24 small instances of each of the seven classes of the paper's
    synthetic set; each method is one batched launch per tolerance."""
    import math
    import numpy as np
    import paper_2311_07710_amd as qpa
    import qpgen
    per = 24
    insts = qpgen.ablation_set(per)
    batch = qpgen.concat_batch(insts)
    cap = 200000
    runs = (("rAPDHG (Sec. 5 halving restart)", 1, 2, 100),
            ("accelerated PDHG (no restart)", 1, 3, 100),
            ("restarted PDHG (Sec. 5 halving restart)", 0, 2, 100),
            ("PDHG (no restart)", 0, 3, 100),
            ("rAPDHG fixed frequency K=10", 1, 1, 10),
            ("rAPDHG fixed frequency K=100", 1, 1, 100),
            ("rAPDHG fixed frequency K=1000", 1, 1, 1000),
            ("rAPDHG (Sec. 6 adaptive restart)", 1, 0, 100),
            ("restarted PDHG (Sec. 6 adaptive restart)", 0, 0, 100))
    norms = None
    out = {"workload": f"{batch.count} QPs: {per} each of {', '.join(qpgen.ABLATION_CLASSES)} "
                       f"(small synthetic instances), Sec. 5 preprocessing, zero start, "
                       f"iteration limit {cap}", "methods": {}}

    def summary(its):
        return {"solved": int(np.sum(its < cap)),
                "sgm10_iterations": math.exp(np.mean(np.log(its + 10.0))) - 10.0,
                "per_class_sgm10": {c: math.exp(np.mean(np.log(its[k * per:(k + 1) * per] + 10.0)))
                                    - 10.0 for k, c in enumerate(qpgen.ABLATION_CLASSES)}}

    for eps in (1e-3, 1e-6):
        fixed = []
        for name, mom, mode, K in runs:
            bs = qpa.BatchSolver(batch, qpa.Settings(eps=eps, momentum=mom, restart_mode=mode,
                                                     fixed_K=K, max_iter=cap, precondition=1))
            if norms is None:
                norms = bs.norms()
            else:
                bs.set_norms(*norms)
            t = time.perf_counter()
            _, _, res = bs.solve()
            dt = time.perf_counter() - t
            bs.close()
            its = np.array([r["iterations"] if r["status"] == 0 else cap for r in res], float)
            row = summary(its)
            row["seconds"] = dt
            if mode == 1:
                fixed.append(its)
            out["methods"].setdefault(name, {})[f"{eps:g}"] = row
            log(f"[bench] ablation eps {eps:g}: {name}: solved {row['solved']}/{batch.count}, "
                f"SGM10 {row['sgm10_iterations']:.0f} iterations, {dt:.2f}s")
        best = np.minimum.reduce(fixed)
        row = summary(best)
        out["methods"].setdefault("rAPDHG tuned fixed frequency (best K per instance)",
                                  {})[f"{eps:g}"] = row
        log(f"[bench] ablation eps {eps:g}: rAPDHG tuned fixed frequency: solved "
            f"{row['solved']}/{batch.count}, SGM10 {row['sgm10_iterations']:.0f} iterations")
    return out


def bench_classes(log):
    """The seven synthetic classes of the paper's large-scale set at medium size (about
    1-4 M nonzeros each), plus the full-size factor-model portfolio QP (5e5 assets, 1000
    factors), preconditioned (Sec. 5), solved to relKKT 1e-6 one instance at a time:
    iterations, seconds and iterations per second."""
    import numpy as np
    import paper_2311_07710_amd as qpa
    import qpgen
    makers = {
        "random_qp": lambda: qpgen.large_random_qp(seed=12, n=150_000, m=75_000),
        "eq_qp": lambda: qpgen.eq_qp(seed=13, n=200_000),
        "control": lambda: qpgen.mpc_qp(np.random.default_rng(14), 2000, 20, 10,
                                        name="control_T2000_nx20_nu10"),
        "portfolio": lambda: qpgen.portfolio_qp(seed=15, n_assets=200_000, k=1000),
        "portfolio_full_size": lambda: qpgen.portfolio_qp(),   # 5e5 assets, 1000 factors
        "huber": lambda: qpgen.huber_qp(seed=16, n_features=10_000, m_samples=100_000,
                                        density=0.003),
        "lasso": lambda: qpgen.lasso_qp(seed=17, n_features=10_000, m_samples=100_000,
                                        density=0.003),
        "svm": lambda: qpgen.svm_qp(seed=18, n_features=10_000, m_samples=100_000,
                                    density=0.003),
    }
    out = {}
    for name, make in makers.items():
        t = time.time()
        qp = make()
        gen_s = time.time() - t
        t = time.time()
        with qpa.Solver(qp, qpa.Settings(eps=1e-6, precondition=1, time_limit_s=60.0)) as s:
            create_s = time.time() - t
            t = time.perf_counter()
            _, _, r = s.solve()
            dt = time.perf_counter() - t
        nnz = int(qp.q_nnz + qp.a_nnz)
        out[name] = {"n": int(qp.n), "m": int(qp.m), "nnz": nnz, "status": r["status"],
                     "iterations": r["iterations"], "rel_kkt": r["rel_kkt"], "seconds": dt,
                     "iters_per_s": r["iterations"] / dt if dt > 0 else None,
                     "create_s": create_s}
        log(f"[bench] class {name}: n={qp.n} m={qp.m} nnz={nnz} (gen {gen_s:.1f}s, create "
            f"{create_s:.2f}s): status {r['status']}, {r['iterations']} iterations in {dt:.3f}s "
            f"({r['iterations'] / dt:.0f} it/s), relKKT {r['rel_kkt']:.2e}")
    return out


def bench_infeasibility(log):
    """Infeasibility certificates on the random-QP class at medium size (n = 1.5e5,
    m = 7.5e4): a primal-infeasible variant (a contradictory row pair) and an unbounded
    one (a ray of descent along x_0), preprocessed, detection on."""
    import qpgen
    import paper_2311_07710_amd as qpa
    base = qpgen.large_random_qp(seed=12, n=150_000, m=75_000)
    out = {}
    for name, qp in (("primal_infeasible", qpgen.with_contradictory_rows(base, 1)),
                     ("unbounded", qpgen.with_unbounded_ray(base))):
        with qpa.Solver(qp, qpa.Settings(eps=1e-6, precondition=1, detect_infeasibility=1,
                                         max_iter=200000, time_limit_s=60.0)) as s:
            t = time.perf_counter()
            _, _, r = s.solve()
            dt = time.perf_counter() - t
        out[name] = {"status": r["status"], "iterations": r["iterations"], "seconds": dt}
        log(f"[bench] {name}: status {r['status']} after {r['iterations']} iterations "
            f"({dt:.3f}s)")
    return out


def bench_warmstart(log, count):
    """Learned warm start on the portfolio family (n_assets 5000, k 100): labels from
    batched cold solves at 1e-8, MLP 10001-512-512-5202 trained by the library's BF16
    kernels on 80 %, warm vs cold to relKKT 1e-6 on the held-out 20 %."""
    import numpy as np
    import paper_2311_07710_amd as qpa
    from paper_2311_07710_amd import warmstart as ws
    import qpgen
    t = time.time()
    fam = qpgen.portfolio_family(seed=5, count=count)
    ntr = int(0.8 * count)
    tr, te = np.arange(ntr), np.arange(ntr, count)
    log(f"[bench] portfolio family generated in {time.time() - t:.1f}s")
    nA, nQ = ws.family_norms(fam)
    s8 = qpa.Settings(eps=1e-8, norm_A=nA, norm_Q=nQ)
    s6 = qpa.Settings(eps=1e-6, norm_A=nA, norm_Q=nQ)
    X, Y, res, t_lab = ws.solve_family(fam, tr, s8, chunk=2048,
                                       log=lambda msg: log(f"[bench] labels: {msg}"))
    omega = np.array([r["omega"] for r in res])
    log(f"[bench] {ntr} label solves (1e-8) in {t_lab:.1f}s")
    t = time.perf_counter()
    epochs = 60
    model = ws.train(ws.features(fam, tr), ws.targets(X, Y, omega), fam.base.n, fam.base.m,
                     hidden=(512, 512), epochs=epochs, batch=256, lr=3e-4, seed=0,
                     log=lambda msg: log(f"[bench] train: {msg}"))
    train_s = time.perf_counter() - t
    # GEMM work of training: forward 2*in*out per layer and sample, backward twice that
    sizes = model.mlp.sizes
    steps = epochs * (ntr // 256)
    gemm_flops = 3.0 * 2.0 * sum(a * b for a, b in zip(sizes[:-1], sizes[1:])) * 256 * steps
    log(f"[bench] MLP trained in {train_s:.1f}s ({gemm_flops / train_s / 1e12:.2f} TFLOP/s of "
        f"BF16 GEMM work incl. host loop), loss {model.history[0]:.4f} -> "
        f"{model.history[-1]:.4f}")
    t = time.perf_counter()
    x0, y0, w0 = model.predict(ws.features(fam, te))
    pred_s = time.perf_counter() - t
    _, _, cold, t_cold = ws.solve_family(fam, te, s6, log=lambda msg: log(f"[bench] cold: {msg}"))
    _, _, warm, t_warm = ws.solve_family(fam, te, s6, x0=x0, y0=y0, omega0=w0,
                                         log=lambda msg: log(f"[bench] warm: {msg}"))
    # what the network adds over constant priors taken from the training labels: the mean
    # solution with the geometric-mean primal weight, and the primal weight alone
    # (predicted, or the training geometric mean) from a zero start
    nt = te.size
    gm = np.full(nt, float(np.exp(np.log(omega).mean())))
    xm, ym = np.tile(X.mean(axis=0), (nt, 1)), np.tile(Y.mean(axis=0), (nt, 1))
    rows = {}
    for name, kw in (("mean_solution_start", dict(x0=xm, y0=ym, omega0=gm)),
                     ("predicted_omega_only", dict(omega0=w0)),
                     ("mean_omega_only", dict(omega0=gm))):
        _, _, rs, t_r = ws.solve_family(fam, te, s6, **kw)
        its = np.array([r["iterations"] for r in rs], dtype=float)
        rows[name] = {"iterations_mean": its.mean(), "seconds": t_r,
                      "optimal": int(sum(r["status"] == 0 for r in rs))}
        log(f"[bench] held-out {name}: {its.mean():.0f} it / {t_r:.2f}s")
    ci = np.array([r["iterations"] for r in cold], dtype=float)
    wi = np.array([r["iterations"] for r in warm], dtype=float)
    kept = int(sum(r["used_warm_start"] for r in warm))
    okw = int(sum(r["status"] == 0 for r in warm))
    log(f"[bench] held-out {te.size}: cold {ci.mean():.0f} it / {t_cold:.2f}s, warm "
        f"{wi.mean():.0f} it / {t_warm:.2f}s (+{pred_s:.2f}s inference), kept {kept}")
    return {"workload": f"portfolio family n_assets=5000 k=100, {count} instances "
                        f"({ntr} train / {te.size} held out), eps 1e-6",
            "cold_iterations_mean": ci.mean(), "warm_iterations_mean": wi.mean(),
            "cold_seconds": t_cold, "warm_seconds": t_warm, "inference_seconds": pred_s,
            "constant_priors": rows,
            "warm_kept": kept, "warm_optimal": okw, "held_out": int(te.size),
            "label_solve_seconds": t_lab, "train_seconds": train_s,
            "loss_first_epoch": model.history[0], "loss_last_epoch": model.history[-1],
            "mlp_train_gemm_tflops": gemm_flops / train_s / 1e12,
            "mlp_bf16_peak_tflops": 2500.0}


if __name__ == "__main__":
    main()
