"""GPU parity at the shapes of the larger workloads: m = 1,000,000, n = 1000, d = 20,000 (the
mixed-precision shape) and m = 4,000,000, n = 2000, d = 40,000 (the large tall problem).

* QR of the sketch (Algorithm 2, third line; eq. it-sk-qr) at n = 1000, 2000 and 2048, on both
  panel paths, which must also agree bit for bit: against the oracle's unblocked Householder QR
  where it finishes in about a minute (d = 20,000 at n = 1000; d = 8192 at n = 2000, the first d of
  the 512-row panels), and against the oracle's TSQR form at the full d = 40,000, n = 2000 (R is
  unique up to row signs, so the TSQR R is compared after matching the diagonal signs).
* The column-sliced sketch gather at n = 2000, d = 40,000 (four slice groups, several launches per
  group), bit-exact against the oracle's sum over j (eq. sparse_sign).
* Whole solves at the mixed-precision shape, FP64 and mixed, with the stopping rule of Section 3.3:
  the forward error must be within 10x that of the backward-stable Householder solution (the oracle
  in TSQR form on the same A and b, Section 2.1 / eq. ls_forward).
"""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_2311_04362_amd import ls  # noqa: E402
from synth import ProblemSpec, make_problem_gpu  # noqa: E402

pytestmark = pytest.mark.gpu
U = 2.0 ** -53
U32 = 2.0 ** -24
THREADS = min(16, len(os.sched_getaffinity(0)))


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


def graded(d, n, kappa, seed, dtype=np.float64):
    """d x n matrix with singular values log-spaced from 1 to 1/kappa, and a Gaussian right side."""
    rng = np.random.default_rng(seed)
    Uq, _ = np.linalg.qr(rng.standard_normal((d, n)))
    Vq, _ = np.linalg.qr(rng.standard_normal((n, n)))
    B = ((Uq * kappa ** (-np.arange(n) / (n - 1))) @ Vq.T).astype(dtype)
    return B, rng.standard_normal(d).astype(dtype)


def both_panels(ctx, fn):
    out = []
    for panel in (0, 1):
        ctx.set_option(ls.OPT_QR_PANEL, panel)
        try:
            out.append(fn())
            ctx.sync()
        finally:
            ctx.set_option(ls.OPT_QR_PANEL, 0)
    return out


# ------------------------------------------------------------------------ QR, FP64

@pytest.mark.parametrize("d,n,kappa", [(20000, 1000, 1e4), (8192, 2000, 1e3), (8192, 2048, 1e2)])
def test_qr_wide_vs_oracle(ctx, d, n, kappa):
    B, Sb = graded(d, n, kappa, d + n)
    (R0, x0), (R1, x1) = both_panels(ctx, lambda: ctx.qr_sketch(dev(B), dev(Sb)))
    assert torch.equal(R0, R1) and torch.equal(x0, x1)      # both panel paths, same bits
    R, x0 = host(R0), host(x0)
    xo, Ro, _, res = oracle.householder_lstsq(B, Sb)
    nB = np.linalg.norm(B)
    assert np.all(np.tril(R, -1) == 0)
    assert np.linalg.norm(R.T @ R - B.T @ B) <= 20 * n * U * nB ** 2        # backward stability
    assert np.array_equal(np.sign(np.diag(R)), np.sign(np.diag(Ro)))       # beta = -sign(alpha) sigma
    assert np.linalg.norm(R - Ro) <= 50 * n * U * kappa * nB
    tol = 100 * kappa * U * (np.linalg.norm(xo) + kappa * res)              # Wedin floor, ||B|| = 1
    assert np.linalg.norm(x0 - xo) <= tol


def test_qr_large_shape_vs_tsqr(ctx):
    """The QR the large tall problem factors (d = 40,000, n = 2000): 63 panels on 79 work-groups."""
    d, n, kappa = 40000, 2000, 1e3
    B, Sb = graded(d, n, kappa, 7)
    (R0, x0), (R1, x1) = both_panels(ctx, lambda: ctx.qr_sketch(dev(B), dev(Sb)))
    assert torch.equal(R0, R1) and torch.equal(x0, x1)
    R, x0 = host(R0), host(x0)
    xo, Ro, res = oracle.tsqr_lstsq(B, Sb, block_rows=8192, threads=THREADS)
    nB = np.linalg.norm(B)
    assert np.all(np.tril(R, -1) == 0)
    assert np.linalg.norm(R.T @ R - B.T @ B) <= 20 * n * U * nB ** 2
    D = np.sign(np.diag(R)) * np.sign(np.diag(Ro))                           # row signs
    assert np.linalg.norm(R - D[:, None] * Ro) <= 50 * n * U * kappa * nB
    tol = 100 * kappa * U * (np.linalg.norm(xo) + kappa * res)
    assert np.linalg.norm(x0 - xo) <= tol


# ------------------------------------------------------------------------ QR, FP32

def test_qr_f32_n1000_vs_oracle(ctx):
    d, n, kappa = 20000, 1000, 1e3
    B, Sb = graded(d, n, kappa, 11, np.float32)
    (R0, x0), (R1, x1) = both_panels(ctx, lambda: ctx.qr_sketch_f32(dev(B), dev(Sb)))
    assert torch.equal(R0, R1) and torch.equal(x0, x1)
    R, x0 = host(R0).astype(np.float64), host(x0)
    xo, Ro, _ = oracle.householder_lstsq_f32(B, Sb)
    B64, Ro = B.astype(np.float64), Ro.astype(np.float64)
    nB = np.linalg.norm(B64)
    assert np.all(np.tril(R, -1) == 0)
    assert np.linalg.norm(R.T @ R - B64.T @ B64) <= 8 * n * U32 * nB ** 2
    assert np.array_equal(np.sign(np.diag(R)), np.sign(np.diag(Ro)))
    kap = np.linalg.cond(B64)
    assert np.linalg.norm(R - Ro) <= 50 * n * U32 * kap * nB
    x64 = np.linalg.lstsq(B64, Sb.astype(np.float64), rcond=None)[0]
    res = np.linalg.norm(B64 @ x64 - Sb)
    tol = 100 * n * kap * U32 * (np.linalg.norm(x64) + kap * res / np.linalg.norm(B64, 2))
    assert np.linalg.norm(x0 - x64) <= tol
    assert np.linalg.norm(xo - x64) <= tol


# ------------------------------------------------------------------ column-sliced gather

def test_window_gather_n2000_bit_exact(ctx):
    """n = 2000 at d = 40,000: 32 slices in four groups of eight, each group in several launches."""
    m, n, d = 70001, 2000, 40000
    rng = np.random.default_rng(2000)
    A = rng.standard_normal((m, n))
    b = rng.standard_normal(m)
    B, Sb = ctx.sketch(dev(A), dev(b), d, 8, 53)
    eB, eSb = oracle.sketch(A, b, n, d, 8, 53)
    assert np.array_equal(host(B), eB)
    assert np.array_equal(host(Sb), eSb)


# ------------------------------------------------ whole solves at the mixed-precision shape

@pytest.fixture(scope="module")
def tsqr_cases():
    """Problems m = 1e6, n = 1000 (kappa in {1e2, 1e6}, ||r|| = 1e-3) and the forward error of
    their Householder (TSQR) least-squares solutions."""
    out = {}

    def get(kappa, beta):
        key = (kappa, beta)
        if key not in out:
            for k in list(out):
                del out[k]
            torch.cuda.empty_cache()
            spec = ProblemSpec(m=1_000_000, n=1000, kappa=kappa, beta=beta, d=20_000, seed=0)
            p = make_problem_gpu(spec)
            n = spec.n
            Ah = p.A[:, :n].cpu().numpy()
            xo, _, res = oracle.tsqr_lstsq(Ah, p.b.cpu().numpy(), block_rows=16384, threads=THREADS)
            del Ah
            fe_o = float(np.linalg.norm(xo - p.x_true.cpu().numpy()))
            out[key] = (spec, p, fe_o, res)
        return out[key]

    yield get
    out.clear()
    torch.cuda.empty_cache()


@pytest.mark.parametrize("kappa,precision", [(1e2, 0), (1e2, 1), (1e6, 0), (1e6, 1)])
def test_solve_mixed_shape_vs_tsqr(ctx, tsqr_cases, kappa, precision):
    spec, p, fe_o, res = tsqr_cases(kappa, 1e-3)
    assert abs(res - 1e-3) <= 1e-3 * 1e-6                # ||b - A x_o|| = ||r|| (generator)
    n = spec.n
    ctx.set_option(ls.OPT_SEED, spec.sketch_seed)
    ctx.set_option(ls.OPT_PRECISION, precision)
    ctx.set_option(ls.OPT_STOP, 1)
    try:
        x = ctx.solve(p.A[:, :n], p.b, spec.d, 200)
        _, steps, _, ce, used = ctx.solve_info()
    finally:
        ctx.set_option(ls.OPT_PRECISION, 0)
        ctx.set_option(ls.OPT_STOP, 0)
    fe = float(torch.linalg.norm(x - p.x_true))
    print(f"kappa={kappa:.0e} precision={precision} used={used} steps={steps} condest={ce:.3e} "
          f"fe={fe:.3e} oracle fe={fe_o:.3e}")
    assert steps < 200
    assert fe <= 10 * fe_o
    if precision == 1 and kappa == 1e2:
        assert used == ls.PRECISION_MIXED
