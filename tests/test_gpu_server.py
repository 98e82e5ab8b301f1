"""The served stream (ls_server_*): continuous batching of many resident solves.  Each result must be
bitwise the result of ls_solve on that problem alone, whatever else is resident, under any
admission budget; a failing problem fails alone."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_2311_04362_amd import ls  # noqa: E402
from synth import ProblemSpec, make_problem_cpu  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = ls.Context(0)
    yield c
    c.close()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


SHAPES = [(4000, 32, 1e2), (20011, 64, 1e6), (3001, 20, 1e10), (60000, 128, 1e3), (9000, 256, 1e8),
          (5000, 50, 1e4), (100003, 33, 1e12), (2500, 100, 1e2)]


def problems():
    out = []
    for i, (m, n, kappa) in enumerate(SHAPES):
        spec = ProblemSpec(m=m, n=n, kappa=kappa, beta=1e-6, d=20 * n, seed=40 + i)
        p = make_problem_cpu(spec)
        out.append((spec, dev(p.A)[:, :n], dev(p.b), p))
    return out


@pytest.fixture(scope="module")
def probs():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return problems()


def alone_results(ctx, probs, q):
    res = []
    for spec, A, b, _ in probs:
        ctx.set_option(ls.OPT_SEED, spec.sketch_seed)
        res.append(ctx.solve(A, b, spec.d, q).clone())
    return res


@pytest.mark.parametrize("q", [0, 1, 7, 40])
def test_served_equals_ls_solve_bitwise(ctx, probs, q):
    ref = alone_results(ctx, probs, q)
    srv = ls.Server(0, budget_bytes=64 << 30, max_active=64)
    try:
        tk = [srv.submit(A, b, spec.d, q, spec.sketch_seed) for spec, A, b, _ in probs]
        for (t, x), r in zip(tk, ref):
            assert srv.wait(t, 120.0) == ls.LS_OK
            assert torch.equal(x, r)
        st = srv.stats()
        assert st["finished"] == len(probs) and st["admitted"] == 0
        assert st["footprint"] == st["setup_workspace"] > 0     # only the setup lanes' workspaces remain
        if q > 1:
            assert st["rounds"] < q * len(probs)          # rounds were shared
    finally:
        srv.close()


@pytest.fixture(scope="module")
def mixed_cases(probs):
    """The problems above (kappa 1e2 to 1e12: the FP32 factor is taken, or refused by condest) and
    one with d = n, where the iteration diverges although the FP32 factor is well conditioned (the
    growth monitor fires)."""
    spec = ProblemSpec(m=2000, n=20, kappa=1e3, beta=1e-3, d=20, seed=0)
    p = make_problem_cpu(spec)
    return [(sp, A, b) for sp, A, b, _ in probs] + [(spec, dev(p.A)[:, :20], dev(p.b))]


def mixed_alone(ctx, cases, q):
    """ls_solve with LS_OPT_PRECISION = 1 on each problem alone: (x, precision used)."""
    out = []
    ctx.set_option(ls.OPT_PRECISION, 1)
    try:
        for spec, A, b in cases:
            ctx.set_option(ls.OPT_SEED, spec.sketch_seed)
            x = ctx.solve(A, b, spec.d, q).clone()
            out.append((x, ctx.solve_info()[4]))
    finally:
        ctx.set_option(ls.OPT_PRECISION, 0)
    return out


@pytest.mark.parametrize("q", [0, 7, 40])
def test_served_mixed_equals_ls_solve_bitwise(ctx, mixed_cases, q):
    ref = mixed_alone(ctx, mixed_cases, q)
    srv = ls.Server(0, budget_bytes=64 << 30, max_active=64)
    try:
        srv.set_precision(ls.PRECISION_MIXED)
        tk = [srv.submit(A, b, spec.d, q, spec.sketch_seed) for spec, A, b in mixed_cases]
        for (t, x), (xr, used) in zip(tk, ref):
            assert srv.wait(t, 120.0) == ls.LS_OK
            assert srv.precision(t) == used
            assert torch.equal(x, xr)
        if q == 40:                               # every outcome occurs
            assert {srv.precision(t) for t, _ in tk} == {
                ls.PRECISION_MIXED, ls.PRECISION_FELL_BACK_COND, ls.PRECISION_FELL_BACK_GROWTH}
        st = srv.stats()
        assert st["finished"] == len(mixed_cases) and st["admitted"] == 0
        assert st["footprint"] == st["setup_workspace"] > 0
    finally:
        srv.close()


def test_served_mixed_and_fp64_together(ctx, probs, mixed_cases):
    q = 12
    ref64 = alone_results(ctx, probs, q)
    refm = mixed_alone(ctx, mixed_cases[:len(probs)], q)
    srv = ls.Server(0)
    try:
        tk = []
        for k, (spec, A, b, _) in enumerate(probs):
            srv.set_precision(ls.PRECISION_MIXED if k % 2 else ls.PRECISION_FP64)
            tk.append(srv.submit(A, b, spec.d, q, spec.sketch_seed))
        for k, ((t, x), r64, (rm, used)) in enumerate(zip(tk, ref64, refm)):
            assert srv.wait(t, 120.0) == ls.LS_OK
            if k % 2:
                assert srv.precision(t) == used and torch.equal(x, rm)
            else:
                assert srv.precision(t) == ls.PRECISION_FP64 and torch.equal(x, r64)
    finally:
        srv.close()


def test_served_mixed_growth_requeue_one_slot(ctx, mixed_cases):
    """A request whose growth monitor fires is queued again, first, as an FP64 request: with one
    slot the next request is admitted only after it has finished in FP64."""
    cases = [mixed_cases[-1], mixed_cases[0], mixed_cases[-1]]
    ref = mixed_alone(ctx, cases, 30)
    assert [u for _, u in ref] == [ls.PRECISION_FELL_BACK_GROWTH, ls.PRECISION_MIXED, ls.PRECISION_FELL_BACK_GROWTH]
    srv = ls.Server(0, max_active=1)
    try:
        srv.set_precision(ls.PRECISION_MIXED)
        tk = [srv.submit(A, b, spec.d, 30, spec.sketch_seed) for spec, A, b in cases]
        for (t, x), (xr, used) in zip(tk, ref):
            assert srv.wait(t, 120.0) == ls.LS_OK
            assert srv.precision(t) == used and torch.equal(x, xr)
        times = [srv.times(t) for t, _ in tk]
        assert times[1][1] >= times[0][3] and times[2][1] >= times[1][3]
        assert srv.stats()["admitted"] == 0
    finally:
        srv.close()


def test_served_mixed_wide_rows_bitwise(ctx):
    """n = 600: ls_solve's FP32 solves read four floats per load above n = 512, the served solve
    one; the sums, and so the bits, are the same (FP64 and mixed requests)."""
    spec = ProblemSpec(m=30000, n=600, kappa=1e2, beta=1e-6, d=12000, seed=77)
    p = make_problem_cpu(spec)
    A, b = dev(p.A)[:, :600], dev(p.b)
    (xm, used), = mixed_alone(ctx, [(spec, A, b)], 9)
    assert used == ls.PRECISION_MIXED
    ctx.set_option(ls.OPT_SEED, spec.sketch_seed)
    x64 = ctx.solve(A, b, spec.d, 9).clone()
    srv = ls.Server(0)
    try:
        t64, y64 = srv.submit(A, b, spec.d, 9, spec.sketch_seed)
        srv.set_precision(ls.PRECISION_MIXED)
        tm, ym = srv.submit(A, b, spec.d, 9, spec.sketch_seed)
        assert srv.wait(t64, 120.0) == ls.LS_OK and srv.wait(tm, 120.0) == ls.LS_OK
        assert srv.precision(tm) == ls.PRECISION_MIXED
        assert torch.equal(y64, x64) and torch.equal(ym, xm)
    finally:
        srv.close()


def test_served_mixed_under_tight_budget(ctx, mixed_cases):
    """Mixed requests, growth fallbacks among them, under a budget that admits only a few problems
    at a time: every request still finishes with ls_solve's bits, and the footprint stays within
    the budget (a re-queued request gives its block back before it is admitted again)."""
    cases = [mixed_cases[-1], mixed_cases[0], mixed_cases[3], mixed_cases[-1], mixed_cases[5]]
    ref = mixed_alone(ctx, cases, 12)
    probe = ls.Server(0, budget_bytes=1 << 40, max_active=8)
    probe.set_precision(ls.PRECISION_MIXED)
    fps = [probe.footprint(spec.m, spec.n, spec.d) for spec, _, _ in cases]
    probe.close()
    budget = max(r + s_ for r, s_ in fps) + min(r for r, _ in fps)
    srv = ls.Server(0, budget_bytes=budget, max_active=8)
    try:
        srv.set_precision(ls.PRECISION_MIXED)
        tk = [srv.submit(A, b, spec.d, 12, spec.sketch_seed) for spec, A, b in cases]
        for (t, x), (xr, used) in zip(tk, ref):
            assert srv.wait(t, 120.0) == ls.LS_OK
            assert srv.precision(t) == used and torch.equal(x, xr)
        st = srv.stats()
        assert st["footprint_peak"] <= budget and st["admitted"] == 0 and st["finished"] == len(cases)
    finally:
        srv.close()


def test_served_alone_vs_mixed_bitwise(probs):
    spec, A, b, _ = probs[3]
    srv = ls.Server(0)
    try:
        t, x_alone = srv.submit(A, b, spec.d, 30, spec.sketch_seed)
        assert srv.wait(t, 120.0) == ls.LS_OK
        tickets = []
        for k, (sp, A2, b2, _) in enumerate(probs):       # the same problem amid the others, twice
            tickets.append(srv.submit(A2, b2, sp.d, 30 + k, sp.sketch_seed))
            if k == 2:
                tickets.append(srv.submit(A, b, spec.d, 30, spec.sketch_seed))
        tickets.append(srv.submit(A, b, spec.d, 30, spec.sketch_seed))
        for t2, _ in tickets:
            assert srv.wait(t2, 120.0) == ls.LS_OK
        assert torch.equal(tickets[3][1], x_alone)
        assert torch.equal(tickets[-1][1], x_alone)
    finally:
        srv.close()


def test_admission_budget_limits_footprint(ctx, probs):
    ref = alone_results(ctx, probs, 12)
    probe = ls.Server(-1)
    host_fp = [probe.footprint(spec.m, spec.n, spec.d) for spec, _, _, _ in probs]
    probe.close()
    srv = ls.Server(0, budget_bytes=1 << 40, max_active=8)
    fps = [srv.footprint(spec.m, spec.n, spec.d) for spec, _, _, _ in probs]
    srv.close()
    # the resident bytes count at least A and b; the setup workspace at least the sketch and its QR
    for (spec, _, _, _), (res, su), (hres, hsu) in zip(probs, fps, host_fp):
        assert res >= 8 * spec.m * spec.n + 8 * spec.m + 16 * spec.n ** 2
        assert su >= 8 * spec.d * (spec.n + 1) + 4 * 8 * spec.m and su == hsu
    # room for the largest problem with its setup, and the smallest besides: at most a few at a time
    budget = max(r + s for r, s in fps) + min(r for r, _ in fps)
    srv = ls.Server(0, budget_bytes=budget, max_active=8)
    try:
        tk = [srv.submit(A, b, spec.d, 12, spec.sketch_seed) for spec, A, b, _ in probs]
        for (t, x), r in zip(tk, ref):
            assert srv.wait(t, 120.0) == ls.LS_OK
            assert torch.equal(x, r)
        st = srv.stats()
        assert st["footprint_peak"] <= budget
        times = [srv.times(t) for t, _ in tk]
        assert all(t0 <= t1 <= t2 <= t3 for t0, t1, t2, t3 in times)
    finally:
        srv.close()


def test_max_active_one_serializes(ctx, probs):
    ref = alone_results(ctx, probs[:3], 5)
    srv = ls.Server(0, max_active=1)
    try:
        tk = [srv.submit(A, b, spec.d, 5, spec.sketch_seed) for spec, A, b, _ in probs[:3]]
        for (t, x), r in zip(tk, ref):
            assert srv.wait(t, 120.0) == ls.LS_OK
            assert torch.equal(x, r)
        times = [srv.times(t) for t, _ in tk]
        assert times[1][1] >= times[0][3] and times[2][1] >= times[1][3]   # admitted after the previous finished
    finally:
        srv.close()


def test_failing_problem_fails_alone(ctx, probs):
    spec, A, b, _ = probs[0]
    Abad = A.clone()
    Abad[:, 5] = 0.0                                        # rank deficient
    ctx.set_option(ls.OPT_SEED, probs[1][0].sketch_seed)
    ref = ctx.solve(probs[1][1], probs[1][2], probs[1][0].d, 10)
    srv = ls.Server(0)
    try:
        t_bad, _ = srv.submit(Abad, b, spec.d, 10, spec.sketch_seed)
        t_ok, x_ok = srv.submit(probs[1][1], probs[1][2], probs[1][0].d, 10, probs[1][0].sketch_seed)
        assert srv.wait(t_bad, 120.0) == ls.LS_ERR_RANK
        assert srv.wait(t_ok, 120.0) == ls.LS_OK
        assert torch.equal(x_ok, ref)
    finally:
        srv.close()


def test_served_accuracy_vs_oracle(probs):
    """Against the oracle's Algorithm 2 with the same S, d and q (q = 40 does not reach the accuracy
    floor on every shape: the contraction per step varies with the embedding)."""
    srv = ls.Server(0)
    try:
        tk = [srv.submit(A, b, spec.d, 40, spec.sketch_seed) for spec, A, b, _ in probs[:4]]
        for (t, x), (spec, _, _, p) in zip(tk, probs[:4]):
            assert srv.wait(t, 120.0) == ls.LS_OK
            xo = oracle.iterative_sketching(p.A, p.b, spec.n, spec.d, 40, seed=spec.sketch_seed)
            fe_h = np.linalg.norm(oracle.householder_lstsq(p.Aview, p.b)[0] - p.x_true)
            fe_o = np.linalg.norm(xo - p.x_true)
            assert np.linalg.norm(x.cpu().numpy() - xo) <= 1e-3 * fe_o + 10 * fe_h
    finally:
        srv.close()


def test_wait_timeout_and_many_submitters(probs):
    import threading
    srv = ls.Server(0)
    try:
        spec, A, b, _ = probs[6]
        t, _ = srv.submit(A, b, spec.d, 400, spec.sketch_seed)
        with pytest.raises(ls.LSError) as e:
            srv.wait(t, 0.0)
        assert e.value.status == ls.LS_ERR_TIMEOUT
        assert srv.wait(t, 120.0) == ls.LS_OK
        out = []

        def worker(k):
            sp, A2, b2, _ = probs[k]
            out.append(srv.submit(A2, b2, sp.d, 5, sp.sketch_seed))
        th = [threading.Thread(target=worker, args=(k,)) for k in range(len(probs))]
        for x in th:
            x.start()
        for x in th:
            x.join()
        for t2, _ in out:
            assert srv.wait(t2, 120.0) == ls.LS_OK
    finally:
        srv.close()
