"""GPU parity: every step of the hot path, through the C ABI, against the CPU oracle on the same
seeded inputs.  Integer and index work must be bit-exact; floating point must meet the bound
stated in each test (derived from the arithmetic, or from Wedin's theorem for whole solves)."""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_2311_04362_amd import ls  # noqa: E402
from synth import ProblemSpec, integer_problem, make_problem_cpu  # noqa: E402
from synth.problems import wedin_floor  # noqa: E402

pytestmark = pytest.mark.gpu
U = 2.0 ** -53


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = ls.Context(0)
    yield c
    c.close()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    return t.cpu().numpy()


def expected_csr(m, d, zeta, seed):
    rows, signs = oracle.sparse_sign(m, d, zeta, seed)
    j = np.repeat(np.arange(m, dtype=np.int64), zeta)
    r = rows.ravel().astype(np.int64)
    neg = (signs.ravel() < 0).astype(np.int64)
    order = np.lexsort((j, r))                   # by sketch row, then ascending j
    rowptr = np.zeros(d + 1, dtype=np.int64)
    rowptr[1:] = np.cumsum(np.bincount(r, minlength=d))
    cols = (j[order] | (neg[order] << 31)).astype(np.uint32).view(np.int32)
    return rowptr.astype(np.int32), cols


# ------------------------------------------------------------------------- (a1) embedding

@pytest.mark.parametrize("m,d,zeta,seed", [(1000, 1000, 8, 4), (4000, 1000, 8, 4), (50000, 16, 8, 7),
                                           (300, 8, 8, 1), (1000, 3, 1, 2), (2000, 100, 32, 9),
                                           (1, 5, 5, 0), (100000, 10000, 8, 123456789)])
def test_embedding_bit_exact(ctx, m, d, zeta, seed):
    rows, signs = ctx.sketch_embedding(m, d, zeta, seed)
    er, es = oracle.sparse_sign(m, d, zeta, seed)
    assert np.array_equal(host(rows), er)
    assert np.array_equal(host(signs), es)


# ------------------------------------------------------------------------------- (a2) CSR

@pytest.mark.parametrize("m,d,zeta,seed", [(4000, 1000, 8, 4), (1000, 3, 1, 2), (777, 50, 8, 3),
                                           (40000, 4, 2, 5),      # 20000-entry rows: global-memory sort
                                           (200000, 10000, 8, 11),
                                           (100000, 40960, 8, 6),  # largest d of the chunked CSR
                                           (100000, 40961, 8, 6),  # past it: atomic CSR
                                           (20000, 8192, 8, 7),    # 8192-column chunks
                                           (20000, 8191, 8, 7),    # 4096-column chunks
                                           (78173, 640, 8, 3),     # 512-column chunks, ragged last
                                           (200003, 5120, 8, 9),   # 4096-column chunks, ragged last
                                           (20000, 256, 8, 7),     # smallest d of the chunked CSR
                                           (20000, 255, 8, 7)])    # below it: atomic CSR
def test_csr_bit_exact(ctx, m, d, zeta, seed):
    rowptr, cols = ctx.sketch_csr(m, d, zeta, seed)
    erp, ec = expected_csr(m, d, zeta, seed)
    assert np.array_equal(host(rowptr), erp)
    assert np.array_equal(host(cols), ec)


# ----------------------------------------------------------------------------- (a3) sketch

@pytest.mark.parametrize("m,n,d", [(1, 1, 1), (100, 7, 20), (4000, 50, 1000), (3000, 64, 500),
                                   (3000, 65, 500), (5000, 200, 4000), (20000, 500, 10000),
                                   (4099, 513, 1000), (2000, 1000, 2000), (1500, 2048, 2048)])
def test_sketch_bit_exact(ctx, m, n, d):
    rng = np.random.default_rng(m + n + d)
    lda = n + 3
    A = np.zeros((m, lda))
    A[:, :n] = rng.standard_normal((m, n))
    b = rng.standard_normal(m)
    zeta = min(8, d)
    B, Sb = ctx.sketch(dev(A)[:, :n], dev(b), d, zeta, 77)
    eB, eSb = oracle.sketch(A[:, :n], b, n, d, zeta, 77)
    assert np.array_equal(host(B), eB)          # same terms, same order, same single scaling
    assert np.array_equal(host(Sb), eSb)


def test_sketch_integer_and_no_rhs(ctx):
    A, b, _ = integer_problem(3001, 33, seed=1)
    B, Sb = ctx.sketch(dev(A)[:, :33], None, 300, 8, 5)
    eB, _ = oracle.sketch(A[:, :33], b, 33, 300, 8, 5)
    assert Sb is None
    assert np.array_equal(host(B), eB)
    Bp = torch.zeros((300, 40), dtype=torch.float64, device="cuda")      # padded ldb
    ctx.sketch(dev(A)[:, :33], dev(b), 300, 8, 5, B=Bp[:, :33])
    assert np.array_equal(host(Bp)[:, :33], eB)
    assert np.all(host(Bp)[:, 33:] == 0)


# -------------------------------------------------------------------------- (a4, a5) QR + x0

def _check_qr(ctx, B, Sb, kappa_hint):
    d, n = B.shape
    R, x0 = ctx.qr_sketch(dev(B), dev(Sb))
    ctx.sync()
    R, x0 = host(R), host(x0)
    xo, Ro, _, res = oracle.householder_lstsq(B, Sb)
    nB = np.linalg.norm(B)
    assert np.all(np.tril(R, -1) == 0)
    # Backward stability: R^T R = (B + dB)^T (B + dB) with ||dB|| <= c u ||B||.
    G = B.T @ B
    assert np.linalg.norm(R.T @ R - G) <= 20 * n * U * nB ** 2
    # Same sign convention as the oracle (beta = -sign(alpha) sigma).
    assert np.array_equal(np.sign(np.diag(R)), np.sign(np.diag(Ro)))
    kap = np.linalg.cond(B)
    assert np.linalg.norm(R - Ro) <= 50 * n * U * kap * nB
    # Sketch-and-solve start: both within the Wedin floor of the small problem.
    tol = 100 * kap * U * (np.linalg.norm(xo) + kap * res / np.linalg.norm(B, 2))
    assert np.linalg.norm(x0 - xo) <= tol + 1e-300


@pytest.mark.parametrize("panel", [0, 1])     # cooperative panel, per-column launches
@pytest.mark.parametrize("d,n,kappa", [(1, 1, 1.0), (20, 1, 1.0), (100, 31, 1e2), (100, 32, 1e2),
                                       (200, 33, 1e2), (1000, 50, 1e3), (2000, 100, 1e6),
                                       (5000, 257, 1e2), (10000, 500, 1e4), (70000, 40, 1e3)])
def test_qr_sketch_vs_oracle(ctx, d, n, kappa, panel):
    rng = np.random.default_rng(d * 7 + n)
    Uq, _ = np.linalg.qr(rng.standard_normal((d, n)))
    Vq, _ = np.linalg.qr(rng.standard_normal((n, n)))
    sig = kappa ** (-np.arange(n) / max(n - 1, 1))
    B = (Uq * sig) @ Vq.T
    Sb = rng.standard_normal(d)
    ctx.set_option(ls.OPT_QR_PANEL, panel)
    try:
        _check_qr(ctx, B, Sb, kappa)
    finally:
        ctx.set_option(ls.OPT_QR_PANEL, 0)


# d = 8192 is the first d whose panels take 512-row work-groups (128 below).  d = 30000, n = 2010
# (d n >= 6e7) takes the look-ahead on the cooperative path (trailing updates split between two
# streams, panels alternating between two vector buffers; last panel 26 columns wide), against the
# per-column path on one stream.
# d = 33000, n = 300: the first eight panels have 65 work-groups (step-flag barrier), the last two
# 64 (arrival-counter barrier), in one factorization.
@pytest.mark.parametrize("d,n", [(3000, 70), (8191, 70), (8192, 70), (12001, 70), (30000, 2010), (33000, 300),
                                 (20003, 1500), (14999, 2000)])   # just above / below d n = 3e7
def test_qr_panel_paths_agree_bitwise(ctx, d, n):
    """Both panel implementations, with or without the look-ahead, do the same arithmetic in the
    same order."""
    rng = np.random.default_rng(3 + d)
    B, Sb = dev(rng.standard_normal((d, n))), dev(rng.standard_normal(d))
    R0, x0 = ctx.qr_sketch(B, Sb)
    ctx.set_option(ls.OPT_QR_PANEL, 1)
    R1, x1 = ctx.qr_sketch(B, Sb)
    ctx.set_option(ls.OPT_QR_PANEL, 0)
    assert torch.equal(R0, R1) and torch.equal(x0, x1)


def test_qr_of_real_sketch_ill_conditioned(ctx):
    p = make_problem_cpu(ProblemSpec(m=4000, n=50, kappa=1e10, beta=1e-6, d=1000))
    B, Sb = oracle.sketch(p.A, p.b, 50, 1000, 8, p.spec.sketch_seed)
    R, x0 = ctx.qr_sketch(dev(B), dev(Sb))
    ctx.sync()
    R = host(R)
    nB = np.linalg.norm(B)
    assert np.linalg.norm(R.T @ R - B.T @ B) <= 20 * 50 * U * nB ** 2
    xo = oracle.householder_lstsq(B, Sb)[0]
    # x0 error is dominated by the sketch-and-solve error (Fact 2.3); GPU and oracle agree to
    # the Wedin floor of the sketched problem.
    assert np.linalg.norm(host(x0) - xo) <= 10 * wedin_floor(1e10, 1e-6)


def test_qr_rank_deficient_flags(ctx):
    B = np.random.default_rng(0).standard_normal((200, 10))
    B[:, 4] = 0.0
    ctx.qr_sketch(dev(B), dev(np.ones(200)))
    with pytest.raises(ls.LSError) as e:
        ctx.sync()
    assert e.value.status == ls.LS_ERR_RANK
    ctx.sync()                                   # status cleared


# -------------------------------------------------------------------- (a6, a7) fused pass

NS = [1, 5, 8, 9, 16, 17, 32, 33, 50, 64, 65, 128, 129, 256, 257, 500, 512, 513, 1000, 1024, 1025,
      2000, 2048]


@pytest.mark.parametrize("n", NS)
def test_gradient_integer_exact(ctx, n):
    m = 3001 if n > 500 else 20011
    A, b, x = integer_problem(m, n, seed=n, lda=n + 1)
    c, rr = ctx.gradient(dev(A)[:, :n], dev(b), dev(x))
    ec, err = oracle.residual_gradient(A[:, :n], b, x)
    assert np.array_equal(host(c), ec)
    assert host(rr)[0] == err


@pytest.mark.parametrize("n", NS)
@pytest.mark.parametrize("m", [1, 3, 4099, 100003])
def test_gradient_float_bound(ctx, n, m):
    if m * n > 60_000_000:          # keep the oracle's work bounded: the largest odd m that fits
        m = (60_000_000 // n) | 1
    rng = np.random.default_rng(n * 31 + m)
    A = rng.standard_normal((m, n))
    x = rng.standard_normal(n)
    b = A @ x + 1e-3 * rng.standard_normal(m)
    c, rr = ctx.gradient(dev(A), dev(b), dev(x))
    ec, err = oracle.residual_gradient(A, b, x)
    aA = np.abs(A)
    r = b - A @ x
    # |c_hat - c| <= gamma_{n+1} |A|^T (|b| + |A||x|) + gamma_m |A|^T |r| for each side (Higham 3.5)
    bound = (n + 2) * U * (aA.T @ (np.abs(b) + aA @ np.abs(x))) + (m + 1) * U * (aA.T @ np.abs(r))
    assert np.all(np.abs(host(c) - ec) <= 2 * bound)
    # each r_i is within e_i = gamma_{n+1} (|b_i| + |A_i| |x|) on either side
    e = (n + 2) * U * (np.abs(b) + aA @ np.abs(x))
    rr_bound = 2 * (2 * np.abs(r) @ e + e @ e) + 2 * (m + 1) * U * (r @ r)
    assert abs(host(rr)[0] - err) <= rr_bound


# ---------------------------------------------------------------- (a8, a9) solves, update

@pytest.mark.parametrize("n", [1, 2, 63, 64, 65, 200, 500, 1000, 2000])
def test_precond_solve_integer_exact(ctx, n):
    rng = np.random.default_rng(n)
    R = np.triu(rng.integers(-1, 2, size=(n, n)).astype(float), 1) + np.eye(n)
    R = R * (np.abs(np.arange(n)[:, None] - np.arange(n)[None, :]) < 3)   # banded: small integers
    xt = rng.integers(-3, 4, size=n).astype(float)
    c = R.T @ (R @ xt)
    d = ctx.precond_solve(dev(R), dev(c))
    assert np.array_equal(host(d), xt)


@pytest.mark.parametrize("n,kappa", [(50, 1e2), (500, 1e2), (2000, 1e2), (300, 1e8)])
def test_precond_solve_vs_oracle(ctx, n, kappa):
    rng = np.random.default_rng(n)
    Q, _ = np.linalg.qr(rng.standard_normal((2 * n, n)))
    R = np.linalg.qr((Q * kappa ** (-np.arange(n) / (n - 1))) @ np.linalg.qr(rng.standard_normal((n, n)))[0],
                     mode="r")
    c = rng.standard_normal(n)
    d = host(ctx.precond_solve(dev(R), dev(c)))
    eo = oracle.solve_r(R, oracle.solve_rt(R, c))
    # each substitution is backward stable: (R + dR) x = y, |dR| <= gamma_n |R| (Higham Thm 8.5),
    # so forward errors are within cond(R)^2 u; for well-conditioned R compare directly,
    # otherwise compare residuals.
    if kappa <= 1e2:
        assert np.linalg.norm(d - eo) <= 100 * n * U * kappa ** 2 * np.linalg.norm(eo)
    lhs = R.T @ (R @ d) - c
    assert np.linalg.norm(lhs) <= 100 * n * U * np.linalg.norm(R, 2) ** 2 * np.linalg.norm(d) + 1e-12 * np.linalg.norm(c)


def test_iterate_one_step_matches_oracle(ctx):
    p = make_problem_cpu(ProblemSpec(m=4000, n=50, kappa=1e2, beta=1e-3, d=1000, seed=3))
    n, d = 50, 1000
    xq, xh, R, rn = oracle.iterative_sketching(p.A, p.b, n, d, 5, seed=p.spec.sketch_seed, history=True)
    A, b, Rd = dev(p.A)[:, :n], dev(p.b), dev(R)
    for i in range(5):
        x = dev(xh[i])
        rr = torch.zeros(1, dtype=torch.float64, device="cuda")
        ctx.iterate(A, b, Rd, x, 1, rnorm2=rr)
        assert np.linalg.norm(host(x) - xh[i + 1]) <= 1e-12 * np.linalg.norm(xh[i + 1])
        assert abs(host(rr)[0] - rn[i]) <= 1e-9 * rn[i]


def test_iterate_trajectory_ill_conditioned(ctx):
    p = make_problem_cpu(ProblemSpec(m=4000, n=50, kappa=1e10, beta=1e-6, d=1000, seed=1))
    n, d, q = 50, 1000, 40
    xq, xh, R, _ = oracle.iterative_sketching(p.A, p.b, n, d, q, seed=p.spec.sketch_seed, history=True)
    x = dev(xh[0])
    rn = torch.zeros(q, dtype=torch.float64, device="cuda")
    ctx.iterate(dev(p.A)[:, :n], dev(p.b), dev(R), x, q, rnorm2=rn)
    ctx.sync()
    fe_gpu = np.linalg.norm(host(x) - p.x_true)
    fe_or = np.linalg.norm(xq - p.x_true)
    fe_hh = np.linalg.norm(oracle.householder_lstsq(p.Aview, p.b)[0] - p.x_true)
    assert fe_gpu <= 10 * fe_hh
    assert fe_gpu <= 10 * fe_or


def test_iterate_q0_leaves_x(ctx):
    x = torch.arange(5, dtype=torch.float64, device="cuda")
    A = torch.ones((10, 5), dtype=torch.float64, device="cuda")
    R = torch.eye(5, dtype=torch.float64, device="cuda")
    ctx.iterate(A, torch.ones(10, dtype=torch.float64, device="cuda"), R, x, 0)
    assert np.array_equal(host(x), np.arange(5.0))


# ------------------------------------------------------------------------ whole solve

@pytest.mark.parametrize("kappa,beta", [(1e1, 1e-12), (1e10, 1e-6), (1e10, 1e-3), (1e15, 1e-12)])
def test_solve_matches_householder_accuracy(ctx, kappa, beta):
    spec = ProblemSpec(m=4000, n=50, kappa=kappa, beta=beta, d=1000, seed=2)
    p = make_problem_cpu(spec)
    ctx.set_option(ls.OPT_SEED, spec.sketch_seed)
    x = host(ctx.solve(dev(p.A)[:, :50], dev(p.b), 1000, 60))
    fe = np.linalg.norm(x - p.x_true)
    fe_hh = np.linalg.norm(oracle.householder_lstsq(p.Aview, p.b)[0] - p.x_true)
    fe_is = np.linalg.norm(oracle.iterative_sketching(p.A, p.b, 50, 1000, 60, seed=spec.sketch_seed) - p.x_true)
    assert fe <= 10 * max(fe_hh, 1e-15)
    assert fe <= 10 * max(fe_is, 1e-15)


def test_solve_config1_q30_and_determinism(ctx):
    spec = ProblemSpec(m=4000, n=50, kappa=1e10, beta=1e-6, d=1000, q=30, seed=0)
    p = make_problem_cpu(spec)
    ctx.set_option(ls.OPT_SEED, spec.sketch_seed)
    A, b = dev(p.A)[:, :50], dev(p.b)
    x1 = host(ctx.solve(A, b, 1000, 30))
    x2 = host(ctx.solve(A, b, 1000, 30))
    assert np.array_equal(x1, x2)                       # bitwise deterministic
    fe_hh = np.linalg.norm(oracle.householder_lstsq(p.Aview, p.b)[0] - p.x_true)
    assert np.linalg.norm(x1 - p.x_true) <= 10 * fe_hh


def test_solve_kappa1_reaches_1e12(ctx):
    spec = ProblemSpec(m=4000, n=50, kappa=1.0, beta=1e-6, d=1000, seed=3)
    p = make_problem_cpu(spec)
    ctx.set_option(ls.OPT_SEED, spec.sketch_seed)
    x = host(ctx.solve(dev(p.A)[:, :50], dev(p.b), 1000, 40))
    assert np.linalg.norm(x - p.x_true) <= 1e-12


def test_solve_q0_is_sketch_and_solve(ctx):
    spec = ProblemSpec(m=3000, n=40, kappa=1e3, beta=1e-2, d=800, seed=4)
    p = make_problem_cpu(spec)
    ctx.set_option(ls.OPT_SEED, spec.sketch_seed)
    x0 = host(ctx.solve(dev(p.A)[:, :40], dev(p.b), 800, 0))
    xo = oracle.iterative_sketching(p.A, p.b, 40, 800, 0, seed=spec.sketch_seed)
    B, Sb = oracle.sketch(p.A, p.b, 40, 800, 8, spec.sketch_seed)
    kap = np.linalg.cond(B)
    res = np.linalg.norm(Sb - B @ xo)
    assert np.linalg.norm(x0 - xo) <= 100 * kap * U * (np.linalg.norm(xo) + kap * res / np.linalg.norm(B, 2))


@pytest.mark.parametrize("m,n", [(20000, 200), (60000, 300)])
def test_solve_medium_vs_oracle(ctx, m, n):
    spec = ProblemSpec(m=m, n=n, kappa=1e8, beta=1e-4, seed=5)
    p = make_problem_cpu(spec)
    ctx.set_option(ls.OPT_SEED, spec.sketch_seed)
    x = host(ctx.solve(dev(p.A)[:, :n], dev(p.b), spec.d, 50))
    fe_hh = np.linalg.norm(oracle.householder_lstsq(p.Aview, p.b)[0] - p.x_true)
    assert np.linalg.norm(x - p.x_true) <= 10 * fe_hh


def test_solve_flags_rank_and_nonfinite(ctx):
    p = make_problem_cpu(ProblemSpec(m=2000, n=20, kappa=1e2, beta=1e-3))
    A = p.A.copy()
    A[:, 7] = 0.0
    with pytest.raises(ls.LSError) as e:
        ctx.solve(dev(A)[:, :20], dev(p.b), 400, 5)
    assert e.value.status == ls.LS_ERR_RANK
    b = p.b.copy()
    b[17] = np.nan
    with pytest.raises(ls.LSError) as e:
        ctx.solve(dev(p.A)[:, :20], dev(b), 400, 5)
    assert e.value.status == ls.LS_ERR_NONFINITE
    x = ctx.solve(dev(p.A)[:, :20], dev(p.b), 400, 5)   # status was cleared
    assert np.all(np.isfinite(host(x)))


def test_device_argument_errors(ctx):
    A = torch.zeros((10, 4), dtype=torch.float64, device="cuda")
    with pytest.raises(ls.LSError) as e:
        ctx.solve(A, torch.zeros(10, dtype=torch.float64, device="cuda"), 2, 3)   # d < n
    assert e.value.status == ls.LS_ERR_ARG


# --------------------------------------------------------- damping / momentum (Section 6)

@pytest.mark.parametrize("update", [1, 2])
def test_iterate_damping_momentum_matches_oracle(ctx, update):
    p = make_problem_cpu(ProblemSpec(m=4000, n=50, kappa=1e3, beta=1e-3, d=1000, seed=6))
    n, d, q = 50, 1000, 12
    eps2 = n / d
    alpha = (1 - eps2) ** 2 / (1 + eps2) if update == 1 else (1 - eps2) ** 2
    beta = 0.0 if update == 1 else eps2
    xq, xh = oracle.iterative_sketching_dm(p.A, p.b, n, d, q, alpha, beta, seed=p.spec.sketch_seed)
    _, _, R, _ = oracle.iterative_sketching(p.A, p.b, n, d, 0, seed=p.spec.sketch_seed, history=True)
    ctx.set_option(ls.OPT_UPDATE, update)
    ctx.set_option(ls.OPT_ALPHA, 0, alpha)
    ctx.set_option(ls.OPT_BETA, 0, beta)
    try:
        x = dev(xh[0])
        ctx.iterate(dev(p.A)[:, :n], dev(p.b), dev(R), x, q)
        ctx.sync()
    finally:
        ctx.set_option(ls.OPT_UPDATE, 0)
        ctx.set_option(ls.OPT_ALPHA, 0, 0.0)
        ctx.set_option(ls.OPT_BETA, 0, -1.0)
    assert np.linalg.norm(host(x) - xq) <= 1e-10 * np.linalg.norm(xq)


def test_solve_momentum_converges_faster(ctx):
    """Theorem 6.1: momentum contracts at about eps = sqrt(n/d) per step, plain at about 2 eps."""
    spec = ProblemSpec(m=4000, n=50, kappa=1e6, beta=1e-3, d=1000, seed=7)
    p = make_problem_cpu(spec)
    A, b = dev(p.A)[:, :50], dev(p.b)
    ctx.set_option(ls.OPT_SEED, spec.sketch_seed)
    fe_hh = np.linalg.norm(oracle.householder_lstsq(p.Aview, p.b)[0] - p.x_true)
    x_plain = host(ctx.solve(A, b, 1000, 12))
    ctx.set_option(ls.OPT_UPDATE, 2)
    try:
        x_mom = host(ctx.solve(A, b, 1000, 12))
        x_mom40 = host(ctx.solve(A, b, 1000, 40))
    finally:
        ctx.set_option(ls.OPT_UPDATE, 0)
    e_plain = np.linalg.norm(x_plain - p.x_true)
    e_mom = np.linalg.norm(x_mom - p.x_true)
    assert e_mom < e_plain
    assert np.linalg.norm(x_mom40 - p.x_true) <= 10 * fe_hh
    xo, _ = oracle.iterative_sketching_dm(p.A, p.b, 50, 1000, 12, (1 - 0.05) ** 2, 0.05, seed=spec.sketch_seed)
    assert np.linalg.norm(x_mom - xo) <= 1e-6 * np.linalg.norm(xo) + 10 * fe_hh
