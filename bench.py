"""Benchmark: whole iterative-sketching solves on one MI355X.

A step is one complete solve (sparse-sign sketch of A, Householder QR of the sketch, sketch-and-
solve start and q refinement passes) of the synthetic problem m = 2,000,000, n = 500, d = 10,000,
zeta = 8, q = 40, kappa = 1e10, ||r|| = 1e-6, with A and b already resident in HBM.  It prints one
JSON line: solves/s, the fused pass's achieved HBM bandwidth against the 8 TB/s peak (per-launch
kernel time from HIP events on the launch stream, around the pass launches of the first and the
last timed solve), and the CPU oracle (Householder least squares in
TSQR form, on every host thread and on one) timed on a bounded sample of the same A and b.  The line
also carries a bounded sub-record ("large") of the largest workload: m = 4,000,000, n = 2000
(A = 64 GB), d = 40,000, q = 40, one warm-up and --large-steps timed FP64 solves.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline] [--large-steps 2]

Other workloads (one JSON line each):
    --workload mixed_m1e6_n1000   mixed precision (FP32 sketch/QR/R-solves, FP64 pass/update) against
                                  the FP64 solver on m = 1,000,000, n = 1000, d = 20,000 for
                                  kappa in {1e2, 1e6, 1e12} x ||r|| in {1e-12, 1e-3, 1}: time and
                                  forward error with the Section 3.3 stopping rule (equal forward
                                  error: both stop at their accuracy floor) and at q = 40
    --workload ls_large_m4e6_n2000  m = 4,000,000, n = 2000 (A is 64 GB), d = 40,000, q = 40, FP64
                                  and mixed
    --workload served_512         512 FP64 problems (m log-uniform on [2e4, 2e5], n in {32, 64, 128,
                                  256}, kappa log-uniform on [1e2, 1e12], ||r|| = 1e-6, d = 20 n, q = 40)
                                  through the served stream, arriving Poisson at 200/s and all at
                                  once (saturation), against ls_solve one request at a time; then
                                  the same with mixed precision (served and ls_solve)
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
WORKLOADS = {
    "ls_fp64_m2e6_n500": dict(m=2_000_000, n=500, d=10_000, zeta=8, q=40, kappa=1e10, beta=1e-6),
    # smaller shape for quick checks on the box
    "ls_fp64_m2e5_n500": dict(m=200_000, n=500, d=10_000, zeta=8, q=40, kappa=1e10, beta=1e-6),
    "mixed_m1e6_n1000": dict(m=1_000_000, n=1000, d=20_000, zeta=8, q=40, kappas=(1e2, 1e6, 1e12),
                             betas=(1e-12, 1e-3, 1.0), qmax=200),
    "ls_large_m4e6_n2000": dict(m=4_000_000, n=2000, d=40_000, zeta=8, q=40, kappa=1e10, beta=1e-6),
    "served_512": dict(count=512, rate=200.0, m_lo=20_000, m_hi=200_000, ns=(32, 64, 128, 256),
                       kappa_lo=1e2, kappa_hi=1e12, beta=1e-6, q=40, zeta=8),
}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_pass_ls_fp64_m2e6_n500_traffic.json")


def pass_bytes(m: int, n: int) -> int:
    """Algorithmic bytes of one fused pass: A (m x n) and b (m) read once, in FP64."""
    return 8 * m * n + 8 * m


def source_digest() -> str:
    p = os.path.join(ROOT, "paper_2311_04362_amd", "csrc", "pass.hip")
    return hashlib.sha256(open(p, "rb").read()).hexdigest()[:16]


def measured_traffic():
    """HBM bytes per pass launch from the committed rocprofv3 counter summary, if it was taken on
    the current pass kernel source; else None."""
    try:
        rec = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    if rec.get("pass_hip_sha256_16") != source_digest():
        return None
    return rec.get("bytes_per_launch")


def host_cpu():
    """(threads this process may use, nproc, CPU model from lscpu)."""
    import subprocess
    model = "unknown"
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
                break
    except (OSError, subprocess.SubprocessError):
        pass
    return len(os.sched_getaffinity(0)), os.cpu_count(), model


def median_time(fn, reps: int = 3) -> float:
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        fn()
        ts.append(time.perf_counter() - t0)
    return sorted(ts)[len(ts) // 2]


def cpu_baseline(w: dict, Ah, bh, copy_s: float, rows_all: int, rows_one: int):
    """The oracle timed on the host's cores on a bounded sample of the workload itself.

    Primary: Householder least squares in TSQR form (the oracle's backward-stable solver) on the
    first rows of the benchmark's own A and b (copied from the GPU beforehand; the copy is timed
    apart), on every host thread this process may use and on one, median of 3 runs each.  Its work
    (2 m n^2 flops) is linear in m for m >> n, so a sample of r rows scales by m / r.
    Second: the oracle's Algorithm 2 (sketch, Householder QR of the sketch, one refinement pass on
    the sample, scaled like the GPU solve: (m / r)(t_sketch + q t_pass) + t_qr), one thread."""
    import oracle

    m, n, d, q = w["m"], w["n"], w["d"], w["q"]
    threads, nproc, model = host_cpu()
    A1, b1 = Ah[:rows_all], bh[:rows_all]
    A2, b2 = Ah[:rows_one], bh[:rows_one]
    t_all = median_time(lambda: oracle.tsqr_lstsq(A1, b1, block_rows=8192, threads=threads))
    t_one = median_time(lambda: oracle.tsqr_lstsq(A2, b2, block_rows=8192, threads=1))
    s_all = t_all * m / rows_all
    s_one = t_one * m / rows_one
    # second baseline: Algorithm 2 on the oracle, one thread
    t0 = time.perf_counter()
    B, Sb = oracle.sketch(A1, b1, n, d, w["zeta"], 0)
    t1 = time.perf_counter()
    x0, R, _, _ = oracle.householder_lstsq(B, Sb)
    t2 = time.perf_counter()
    c, _ = oracle.residual_gradient(A1, b1, x0)
    oracle.solve_r(R, oracle.solve_rt(R, c))
    t3 = time.perf_counter()
    s_alg2 = (m / rows_all) * ((t1 - t0) + q * (t3 - t2)) + (t2 - t1)
    return {"value": 1.0 / s_all, "unit": "solves/s", "cores": threads, "kind": "oracle",
            "sample": (f"Householder least squares (TSQR form, 8192-row blocks) on the first {rows_all} "
                       f"of {m} rows of the benchmark's A and b, {threads} threads, median of 3: "
                       f"{t_all:.2f} s, scaled by m/rows to {s_all:.1f} s/solve"),
            "cpu_model": model, "nproc": nproc,
            "single_thread": {"value": 1.0 / s_one, "unit": "solves/s", "cores": 1,
                              "sample": f"the same on the first {rows_one} rows, 1 thread, median of 3: "
                                        f"{t_one:.2f} s, scaled to {s_one:.1f} s/solve"},
            "host_copy_s": copy_s,
            "algorithm2_oracle": {"value": 1.0 / s_alg2, "unit": "solves/s", "cores": 1,
                                  "sample": (f"the oracle's Algorithm 2 (sketch + 1 refinement pass) on "
                                             f"{rows_all} rows scaled by m/rows, plus Householder QR of "
                                             f"the {d}x{n} sketch; t_sketch={t1 - t0:.2f}s "
                                             f"t_qr={t2 - t1:.2f}s t_pass={t3 - t2:.3f}s")}}


def bench_large_record(args, ls):
    """A bounded run of the largest workload (m = 4e6, n = 2000, A = 64 GB): `steps` timed FP64
    solves after one warm-up, with the fused pass's bandwidth from HIP events and the forward error."""
    import torch

    from synth import ProblemSpec, make_problem_gpu

    w = WORKLOADS["ls_large_m4e6_n2000"]
    m, n, d, q = w["m"], w["n"], w["d"], w["q"]
    spec = ProblemSpec(m=m, n=n, kappa=w["kappa"], beta=w["beta"], d=d, q=q, zeta=w["zeta"], seed=0)
    t_gen = time.perf_counter()
    p = make_problem_gpu(spec)
    print(f"[bench] generated ls_large_m4e6_n2000 on GPU in {time.perf_counter() - t_gen:.1f}s",
          file=sys.stderr, flush=True)
    A, b = p.A[:, :n], p.b
    x = torch.empty(n, dtype=torch.float64, device="cuda")
    ctx = ls.Context(0)
    ctx.set_option(ls.OPT_SEED, spec.sketch_seed)
    ctx.set_option(ls.OPT_ZETA, w["zeta"])
    ctx.set_option(ls.OPT_QR_PANEL, args.qr_panel)
    ctx.solve(A, b, d, q, x)
    torch.cuda.synchronize()
    if args.verbose:
        print("[bench] large: warm-up solve done", file=sys.stderr, flush=True)
    ctx.set_option(ls.OPT_PROFILE, 1)
    ctx.profile(reset=True)
    t0 = time.perf_counter()
    for k in range(args.large_steps):
        ctx.solve(A, b, d, q, x)
        if args.verbose:
            torch.cuda.synchronize()
            print(f"[bench] large: timed solve {k} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / args.large_steps
    pass_ms, launches = ctx.profile(reset=True)
    per_launch = pass_ms / max(launches, 1)
    gbs = pass_bytes(m, n) / (per_launch * 1e-3) / 1e9
    fe = float(torch.linalg.norm(x - p.x_true).item())
    del A, b, x, p
    ctx.close()
    release_device()
    out = {"workload": "ls_large_m4e6_n2000", "m": m, "n": n, "d": d, "zeta": w["zeta"], "q": q,
           "kappa": w["kappa"], "residual_norm": w["beta"], "dtype": "f64",
           "steps": args.large_steps, "warmup": 1, "ms_per_step": 1e3 * t, "solves_per_s": 1.0 / t,
           "pass_avg_launch_ms": per_launch, "pass_GBps": gbs, "pass_frac_of_8TBps": gbs / HBM_PEAK_GBS,
           "forward_error": fe}
    print(f"[bench] large: {out}", file=sys.stderr, flush=True)
    return out


def release_device():
    """Wait for the device and return torch's cached blocks to HIP, so that no device memory,
    event or stream work is still held when the interpreter (and a profiler's exit hooks) tear
    down the runtime."""
    import gc

    import torch
    gc.collect()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def timed_solves(ctx, A, b, d, q, x, reps):
    """Seconds per ls_solve (mean of reps after one warm-up) and the solve info of the last."""
    import torch
    ctx.solve(A, b, d, q, x)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        ctx.solve(A, b, d, q, x)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps, ctx.solve_info()


def bench_mixed(args, w):
    """Mixed precision against FP64 on the nine (kappa, ||r||) cases of the m = 1e6, n = 1000 shape."""
    import torch

    from paper_2311_04362_amd import ls
    from synth import ProblemSpec, make_problem_gpu

    m, n, d, q = w["m"], w["n"], w["d"], w["q"]
    ctx = ls.Context(0)
    ctx.set_option(ls.OPT_ZETA, w["zeta"])
    ctx.set_option(ls.OPT_QR_PANEL, args.qr_panel)
    x = torch.empty(n, dtype=torch.float64, device="cuda")
    cases, speedups_stop, speedups_q = [], [], []
    kappas = [float(v) for v in args.kappas.split(",")] if args.kappas else list(w["kappas"])
    betas = [float(v) for v in args.betas.split(",")] if args.betas else list(w["betas"])
    precs = [(0, "fp64"), (1, "mixed")]
    precs = [pn for pn in precs if pn[1] in args.precisions.split(",")]
    modes = [md for md in ((1, w["qmax"], "stop"), (0, q, "q40")) if md[2] in args.modes.split(",")]
    for kappa in kappas:
        for beta in betas:
            spec = ProblemSpec(m=m, n=n, kappa=kappa, beta=beta, d=d, q=q, zeta=w["zeta"], seed=0)
            p = make_problem_gpu(spec)
            A, b = p.A[:, :n], p.b
            ctx.set_option(ls.OPT_SEED, spec.sketch_seed)
            row = {"kappa": kappa, "residual_norm": beta}
            for stop, qq, tag in modes:
                ctx.set_option(ls.OPT_STOP, stop)
                for prec, name in precs:
                    ctx.set_option(ls.OPT_PRECISION, prec)
                    t, info = timed_solves(ctx, A, b, d, qq, x, args.steps)
                    fe = float(torch.linalg.norm(x - p.x_true).item())
                    row[f"{tag}_{name}"] = {"ms": 1e3 * t, "steps": info[1], "forward_error": fe,
                                            "precision_used": ["fp64", "mixed", "fell_back_condest",
                                                               "fell_back_growth"][info[4]],
                                            "condest": info[3]}
            ctx.set_option(ls.OPT_PRECISION, 0)
            ctx.set_option(ls.OPT_STOP, 0)
            for tag, acc in (("stop", speedups_stop), ("q40", speedups_q)):
                if f"{tag}_fp64" in row and f"{tag}_mixed" in row:
                    row[f"speedup_{tag}"] = row[f"{tag}_fp64"]["ms"] / row[f"{tag}_mixed"]["ms"]
                    acc.append(row[f"speedup_{tag}"])
            brief = {k: (v["ms"], v["precision_used"], v["forward_error"]) for k, v in row.items()
                     if isinstance(v, dict)}
            print(f"[bench] kappa={kappa:.0e} r={beta:.0e}: {brief}", file=sys.stderr, flush=True)
            cases.append(row)
            del p, A, b
            torch.cuda.empty_cache()
    def geomean(v):
        return math.exp(sum(math.log(t) for t in v) / len(v)) if v else None

    geo = geomean(speedups_stop)
    rec = {
        "metric": "mixed/FP64 speedup at equal fwd error",
        "value": geo,
        "unit": "x (geometric mean over the nine cases, both with the Section 3.3 stopping rule)",
        "n_gpus": 1, "steps": args.steps, "warmup": 1,
        "ms_per_step": (sum(c["stop_mixed"]["ms"] for c in cases) / len(cases)
                        if all("stop_mixed" in c for c in cases) else None),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "m": m, "n": n, "d": d, "zeta": w["zeta"],
                   "qmax_stop": w["qmax"], "q_fixed": q},
        "speedup_q40_geomean": geomean(speedups_q),
        "cases": cases,
    }
    ctx.close()
    release_device()
    print(json.dumps(rec), flush=True)


def bench_large(args, w):
    """One large problem (A = 64 GB) in FP64 and mixed precision."""
    import torch

    from paper_2311_04362_amd import ls
    from synth import ProblemSpec, make_problem_gpu

    m, n, d, q = w["m"], w["n"], w["d"], w["q"]
    spec = ProblemSpec(m=m, n=n, kappa=w["kappa"], beta=w["beta"], d=d, q=q, zeta=w["zeta"], seed=0)
    p = make_problem_gpu(spec)
    A, b = p.A[:, :n], p.b
    ctx = ls.Context(0)
    ctx.set_option(ls.OPT_ZETA, w["zeta"])
    ctx.set_option(ls.OPT_SEED, spec.sketch_seed)
    ctx.set_option(ls.OPT_QR_PANEL, args.qr_panel)
    x = torch.empty(n, dtype=torch.float64, device="cuda")
    out = {}
    for prec, name in ((0, "fp64"), (1, "mixed")):
        if name not in args.precisions.split(","):
            continue
        ctx.set_option(ls.OPT_PRECISION, prec)
        ctx.set_option(ls.OPT_PROFILE, 1)
        ctx.profile(reset=True)
        t, info = timed_solves(ctx, A, b, d, q, x, args.steps)
        pass_ms, launches = ctx.profile(reset=True)
        ctx.set_option(ls.OPT_PROFILE, 0)
        per_launch = pass_ms / max(launches, 1)
        out[name] = {"ms": 1e3 * t, "solves_per_s": 1.0 / t,
                     "forward_error": float(torch.linalg.norm(x - p.x_true).item()),
                     "precision_used": ["fp64", "mixed", "fell_back_condest", "fell_back_growth"][info[4]],
                     "pass_GBps": pass_bytes(m, n) / (per_launch * 1e-3) / 1e9}
        print(f"[bench] {name}: {out[name]}", file=sys.stderr, flush=True)
    ctx.set_option(ls.OPT_PRECISION, 0)
    main = out["fp64"] if "fp64" in out else out["mixed"]
    achieved = main["pass_GBps"]
    rec = {
        "metric": "solves/s + iteration-pass HBM GB/s; mixed/FP64 speedup at equal fwd error",
        "value": main["solves_per_s"], "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": 1, "ms_per_step": main["ms"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if "fp64" in out else "f32+f64", "data": "synthetic",
        "config": {"workload": args.workload, "m": m, "n": n, "d": d, "zeta": w["zeta"], "q": q,
                   "kappa": w["kappa"], "residual_norm": w["beta"]},
        "roofline": {"bound": "hbm", "kernel": "k_pass (fused A^T(b - A x) pass)", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None},
        **out,
        "mixed_speedup": (out["fp64"]["ms"] / out["mixed"]["ms"]) if len(out) == 2 else None,
    }
    del p, A, b, x
    ctx.close()
    release_device()
    print(json.dumps(rec), flush=True)


def served_problems(w, seed=2311):
    """The request stream: Poisson arrival times, shapes and conditioning from the master seed
    (synth.served_stream); problem k is built from problem seed 1000 + k."""
    from synth.problems import served_stream
    t, ms, ns, kap = served_stream(count=w["count"], rate=w["rate"], seed=seed)
    return [dict(m=int(ms[i]), n=int(ns[i]), kappa=float(kap[i]), d=20 * int(ns[i]), arrival=float(t[i]),
                 seed=1000 + i) for i in range(w["count"])]


def pct(v, q):
    v = sorted(v)
    return v[min(len(v) - 1, int(math.ceil(q / 100.0 * len(v))) - 1)]


def bench_served(args, w):
    """Served stream against ls_solve one request at a time, Poisson arrivals and saturation."""
    import threading

    import torch

    from paper_2311_04362_amd import ls
    from synth import ProblemSpec, make_problem_gpu

    reqs = served_problems(w)
    t_gen = time.perf_counter()
    probs = []
    for r in reqs:
        spec = ProblemSpec(m=r["m"], n=r["n"], kappa=r["kappa"], beta=w["beta"], d=r["d"], q=w["q"],
                           zeta=w["zeta"], seed=r["seed"])
        p = make_problem_gpu(spec)
        probs.append((spec, p.A[:, :r["n"]], p.b, p.x_true))
    torch.cuda.synchronize()
    resident = sum(8 * r["m"] * r["n"] + 8 * r["m"] for r in reqs)
    print(f"[bench] generated {len(reqs)} problems ({resident / 1e9:.1f} GB of A and b) in "
          f"{time.perf_counter() - t_gen:.1f}s", file=sys.stderr, flush=True)
    q = w["q"]

    names = ["fp64", "mixed", "fell_back_condest", "fell_back_growth"]

    def served(poisson: bool, precision: int = 0):
        srv = ls.Server(0, budget_bytes=200 << 30, max_active=len(reqs))
        srv.set_precision(precision)
        xs = [torch.empty(r["n"], dtype=torch.float64, device="cuda") for r in reqs]
        # warm-up: one small request compiles nothing but touches every code path once
        spec, A, b, _ = probs[0]
        t, _ = srv.submit(A, b, spec.d, q, spec.sketch_seed)
        srv.wait(t)
        tickets = [None] * len(reqs)
        t_start = time.perf_counter()

        def submitter():
            for i, (spec, A, b, _) in enumerate(probs):
                if poisson:
                    delay = t_start + reqs[i]["arrival"] - time.perf_counter()
                    if delay > 0:
                        time.sleep(delay)
                tickets[i] = srv.submit(A, b, spec.d, q, spec.sketch_seed, xs[i])[0]
        th = threading.Thread(target=submitter)
        th.start()
        th.join()
        status = [srv.wait(t) for t in tickets]
        t_end = time.perf_counter()
        lat, wait, setup, rounds = [], [], [], []
        for t in tickets:
            t0, t1, t2, t3 = srv.times(t)
            lat.append(t3 - t0)
            wait.append(t1 - t0)
            setup.append(t2 - t1)
            rounds.append(t3 - t2)
        used = [srv.precision(t) for t in tickets]
        stats = srv.stats()
        srv.close()
        out = {"seconds": t_end - t_start, "solves_per_s": len(reqs) / (t_end - t_start),
               "p50_ms": 1e3 * pct(lat, 50), "p99_ms": 1e3 * pct(lat, 99),
               "rounds": stats["rounds"], "failed": sum(1 for s_ in status if s_ != ls.LS_OK),
               "footprint_peak_GB": stats["footprint_peak"] / 1e9,
               # medians of the phases of a request: queued until admitted, set up, iterated
               "p50_phase_ms": {"queued": 1e3 * pct(wait, 50), "setup": 1e3 * pct(setup, 50),
                                "rounds": 1e3 * pct(rounds, 50)}}
        if precision:
            out["precision_used"] = {nm: sum(1 for u in used if u == k) for k, nm in enumerate(names)}
        return out, xs

    def baseline(poisson: bool, precision: int = 0):
        ctx = ls.Context(0)
        ctx.set_option(ls.OPT_ZETA, w["zeta"])
        ctx.set_option(ls.OPT_PRECISION, precision)
        used = []
        xs = []
        spec, A, b, _ = probs[0]
        ctx.set_option(ls.OPT_SEED, spec.sketch_seed)
        ctx.solve(A, b, spec.d, q)
        lat = []
        t_start = time.perf_counter()
        for i, (spec, A, b, _) in enumerate(probs):
            arrival = t_start + (reqs[i]["arrival"] if poisson else 0.0)
            delay = arrival - time.perf_counter()
            if delay > 0:
                time.sleep(delay)
            ctx.set_option(ls.OPT_SEED, spec.sketch_seed)
            xs.append(ctx.solve(A, b, spec.d, q))      # waits for the result
            lat.append(time.perf_counter() - arrival)
            used.append(ctx.solve_info()[4])
        t_end = time.perf_counter()
        ctx.close()
        out = {"seconds": t_end - t_start, "solves_per_s": len(reqs) / (t_end - t_start),
               "p50_ms": 1e3 * pct(lat, 50), "p99_ms": 1e3 * pct(lat, 99)}
        if precision:
            out["precision_used"] = {nm: sum(1 for u in used if u == k) for k, nm in enumerate(names)}
            out["per_request"] = [{"n": r["n"], "kappa": r["kappa"], "used": names[u]} for r, u in zip(reqs, used)]
        return out, xs

    # Arms (--served-arms picks some, e.g. one per profiled run): the served stream and ls_solve one
    # request at a time, FP64, then with mixed precision (ls_solve mixed gives the bits the served
    # mixed arm must return).
    arms = {
        "served_saturation": lambda: served(False),
        "served_poisson": lambda: served(True),
        "ls_solve_saturation": lambda: baseline(False),
        "ls_solve_poisson": lambda: baseline(True),
        "served_mixed_saturation": lambda: served(False, precision=1),
        "served_mixed_poisson": lambda: served(True, precision=1),
        "ls_solve_mixed_saturation": lambda: baseline(False, precision=1),
    }
    pick = set(args.served_arms.split(","))
    out, xs = {}, {}
    for name, run in arms.items():
        if "all" in pick or name in pick:
            out[name], xs[name] = run()
            shown = {k: v for k, v in out[name].items() if k != "per_request"}
            print(f"[bench] {name}: {shown}", file=sys.stderr, flush=True)

    def rate(a, b_):
        return out[a]["solves_per_s"] / out[b_]["solves_per_s"] if a in out and b_ in out else None

    def same(a, b_):
        return all(torch.equal(u, v) for u, v in zip(xs[a], xs[b_])) if a in xs and b_ in xs else None

    def fes(a):
        return [float(torch.linalg.norm(x - p[3]).item()) for x, p in zip(xs[a], probs)] if a in xs else None

    fe, fe_mixed = fes("served_saturation"), fes("ls_solve_mixed_saturation")
    sat = out.get("served_saturation")
    rec = {
        "metric": "served solves/s (saturation) with p50/p99 latency under Poisson arrivals",
        "value": sat["solves_per_s"] if sat else None, "unit": "solves/s", "n_gpus": 1,
        "steps": 1, "warmup": 1, "ms_per_step": 1e3 * sat["seconds"] if sat else None,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "requests": len(reqs), "rate_per_s": w["rate"],
                   "m": [w["m_lo"], w["m_hi"]], "n": list(w["ns"]), "kappa": [w["kappa_lo"], w["kappa_hi"]],
                   "residual_norm": w["beta"], "d": "20n", "q": q, "zeta": w["zeta"],
                   "resident_GB": resident / 1e9, "arms": sorted(out)},
        "speedup_saturation_vs_ls_solve": rate("served_saturation", "ls_solve_saturation"),
        "bitwise_equal_to_ls_solve": same("served_saturation", "ls_solve_saturation"),
        "forward_error_max": max(fe) if fe else None,
        "mixed_vs_fp64_served_speedup": rate("served_mixed_saturation", "served_saturation"),
        "served_mixed_bitwise_equal_to_ls_solve_mixed": same("served_mixed_saturation", "ls_solve_mixed_saturation"),
        "mixed_vs_fp64_ls_solve_speedup": rate("ls_solve_mixed_saturation", "ls_solve_saturation"),
        "forward_error_max_mixed": max(fe_mixed) if fe_mixed else None,
        "forward_error_mixed_over_fp64_max": (max(a / max(b_, 1e-300) for a, b_ in zip(fe_mixed, fe))
                                              if fe and fe_mixed else None),
        **out,
    }
    del probs, xs
    release_device()
    print(json.dumps(rec), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="ls_fp64_m2e6_n500", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-rows", type=int, default=400_000,
                    help="rows of the all-threads oracle sample (the one-thread sample is a quarter)")
    ap.add_argument("--large-steps", type=int, default=2,
                    help="timed solves of the m = 4e6, n = 2000 sub-record (0: skip it)")
    ap.add_argument("--precisions", default="fp64,mixed",
                    help="mixed and large workloads: which of fp64, mixed to run")
    ap.add_argument("--kappas", default="", help="mixed workload: kappas to run (default: all three)")
    ap.add_argument("--betas", default="", help="mixed workload: ||r|| values to run (default: all three)")
    ap.add_argument("--modes", default="stop,q40",
                    help="mixed workload: stop (Section 3.3 rule, q <= 200) and/or q40 (fixed q)")
    ap.add_argument("--qr-panel", type=int, default=0, choices=(0, 1),
                    help="LS_OPT_QR_PANEL: 0 cooperative panels, 1 one launch per column (same bits)")
    ap.add_argument("--served-arms", default="all",
                    help="served workload: comma list of arms to run (served_saturation, served_poisson, "
                         "ls_solve_saturation, ls_solve_poisson, served_mixed_saturation, "
                         "served_mixed_poisson, ls_solve_mixed_saturation), or all")
    ap.add_argument("--verbose", action="store_true", help="a progress line on stderr after every solve")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also time a plain elementwise copy kernel of 2 GiB (scale for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: the solver runs on one GPU; --gpus above 1 (or WORLD_SIZE > 1) is not supported",
              file=sys.stderr)
        sys.exit(2)

    w = WORKLOADS[args.workload]
    if args.workload.startswith("mixed_"):
        return bench_mixed(args, w)
    if args.workload.startswith("ls_large_"):
        return bench_large(args, w)
    if args.workload.startswith("served_"):
        return bench_served(args, w)

    import torch

    from paper_2311_04362_amd import ls
    from synth import ProblemSpec, make_problem_gpu

    m, n, d, q = w["m"], w["n"], w["d"], w["q"]
    spec = ProblemSpec(m=m, n=n, kappa=w["kappa"], beta=w["beta"], d=d, q=q, zeta=w["zeta"], seed=0)
    t_gen = time.perf_counter()
    p = make_problem_gpu(spec)
    t_gen = time.perf_counter() - t_gen
    print(f"[bench] generated {args.workload} on GPU in {t_gen:.1f}s", file=sys.stderr, flush=True)
    A = p.A[:, :n]
    b = p.b
    x = torch.empty(n, dtype=torch.float64, device="cuda")
    ctx = ls.Context(0)
    ctx.set_option(ls.OPT_SEED, spec.sketch_seed)
    ctx.set_option(ls.OPT_ZETA, w["zeta"])

    ctx.set_option(ls.OPT_QR_PANEL, args.qr_panel)

    def progress(what):
        if args.verbose:
            print(f"[bench] {what} done at {time.perf_counter() - t_start:.1f}s", file=sys.stderr, flush=True)

    t_start = time.perf_counter()
    for k in range(args.warmup):
        ctx.solve(A, b, d, q, x)
        progress(f"warm-up solve {k}")
    torch.cuda.synchronize()
    ctx.profile(reset=True)
    # The pass launches of the first and the last timed solve are bracketed by HIP events (about
    # 4 us per record); the solves between them run without, so the events barely weigh on value.
    profiled = sorted({0, args.steps - 1})
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        ctx.set_option(ls.OPT_PROFILE, 1 if k in profiled else 0)
        ctx.solve(A, b, d, q, x)
        progress(f"timed solve {k}")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    pass_ms, launches = ctx.profile(reset=True)
    ctx.set_option(ls.OPT_PROFILE, 0)

    fe = float(torch.linalg.norm(x - p.x_true).item())
    ms_per_step = 1e3 * (t1 - t0) / args.steps
    value = args.steps / (t1 - t0)
    per_launch_ms = pass_ms / max(launches, 1)
    nbytes = pass_bytes(m, n)
    achieved = nbytes / (per_launch_ms * 1e-3) / 1e9
    traffic = measured_traffic()
    rec = {
        "metric": "solves/s + iteration-pass HBM GB/s; mixed/FP64 speedup at equal fwd error",
        "value": value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "m": m, "n": n, "d": d, "zeta": w["zeta"], "q": q,
                   "kappa": w["kappa"], "residual_norm": w["beta"], "precision": "fp64"},
        "roofline": {"bound": "hbm", "kernel": "k_pass (fused A^T(b - A x) pass)",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "algorithmic_bytes_per_launch": nbytes, "avg_launch_ms": per_launch_ms,
                     "launches_timed": launches, "timed_solves_with_events": profiled},
        "forward_error": fe,
        "pass_share_of_step": (pass_ms / len(profiled)) / max(ms_per_step, 1e-9),
    }
    if args.calib_copy:
        src = torch.full((1 << 28,), 1.0, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.neg(src, out=dst)               # elementwise kernel: reads and writes 2 GiB each
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(5):
            torch.neg(src, out=dst)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 5
        moved = 2 * src.numel() * 8
        rec["copy_calibration"] = {"bytes_read_per_copy": src.numel() * 8,
                                   "bytes_written_per_copy": src.numel() * 8,
                                   "ms_per_copy": ms, "GB/s": moved / (ms * 1e-3) / 1e9}
        del src, dst
    # The CPU oracle's sample: the first rows of this very A and b, copied to the host.
    if not args.no_cpu_baseline:
        rows = min(args.cpu_sample_rows, m)
        t_copy = time.perf_counter()
        Ah = A[:rows].cpu().numpy()
        bh = b[:rows].cpu().numpy()
        t_copy = time.perf_counter() - t_copy
    # Release the problem, the context's workspace, events and pinned word before the next
    # workload and well before interpreter shutdown.
    del A, b, x, p
    ctx.close()
    release_device()
    if args.large_steps > 0:
        rec["large"] = bench_large_record(args, ls)
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle on a bounded sample", file=sys.stderr, flush=True)
        rec["cpu_baseline"] = cpu_baseline(w, Ah, bh, t_copy, rows, max(rows // 4, n + 1))
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
