"""Host-side pieces of bench.py (no GPU): the served stream's request draw and the CPU baseline's
oracle timing on a small sample."""
import math

import numpy as np

import bench
from synth import ProblemSpec, make_problem_cpu


def test_served_stream_matches_the_workload():
    w = bench.WORKLOADS["served_512"]
    reqs = bench.served_problems(w)
    assert len(reqs) == 512
    ms = np.array([r["m"] for r in reqs])
    ns = np.array([r["n"] for r in reqs])
    ks = np.array([r["kappa"] for r in reqs])
    t = np.array([r["arrival"] for r in reqs])
    assert ms.min() >= 20_000 and ms.max() < 200_000
    assert set(ns.tolist()) <= {32, 64, 128, 256} and len(set(ns.tolist())) == 4
    assert ks.min() >= 1e2 and ks.max() <= 1e12
    assert all(r["d"] == 20 * r["n"] for r in reqs)
    assert [r["seed"] for r in reqs] == list(range(1000, 1512))
    assert t[0] == 0.0 and np.all(np.diff(t) >= 0)
    # Poisson arrivals at 200/s: 511 gaps of mean 5 ms (about 4% standard error)
    assert abs(t[-1] / 511 - 0.005) < 0.0008
    # log-uniform m: the mean of ln m is the midpoint of [ln 2e4, ln 2e5]
    assert abs(np.log(ms).mean() - 0.5 * (math.log(2e4) + math.log(2e5))) < 0.1
    assert bench.served_problems(w) == reqs                     # seeded: the same stream every time


def test_cpu_baseline_on_a_small_sample():
    w = dict(bench.WORKLOADS["ls_fp64_m2e6_n500"])
    w.update(m=200_000, n=40, d=800)
    p = make_problem_cpu(ProblemSpec(m=8000, n=40, kappa=1e6, beta=1e-6, d=800, seed=0))
    A = np.ascontiguousarray(p.A[:, :40])
    rec = bench.cpu_baseline(w, A, p.b, 0.01, 8000, 2000)
    assert rec["kind"] == "oracle" and rec["unit"] == "solves/s" and rec["value"] > 0
    assert rec["cores"] >= 1 and rec["single_thread"]["cores"] == 1
    assert rec["algorithm2_oracle"]["value"] > 0 and "nproc" in rec and "cpu_model" in rec
