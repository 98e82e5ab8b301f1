"""Parity at the benchmark's full size (m = 2,000,000, n = 500, d = 10,000, zeta = 8, q = 40,
kappa = 1e10, ||r|| = 1e-6), through the same C-ABI calls bench.py times.

The oracle cannot run Algorithm 2 end to end at this size in reasonable time, so each step is
checked where the oracle can compute the answer: the whole embedding and its CSR (bit-exact),
sampled rows of the sketch (bit-exact, each row summed by the oracle from its own terms), the QR of
the sketch (the oracle factors the same B), the full pass c = A^T (b - A x) (the oracle's plain
loop over all of A), and the whole solve against the oracle's Householder least-squares solution of
the same problem (in TSQR form, on the host's cores): forward error within 10x of the oracle's."""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_2311_04362_amd import ls  # noqa: E402
from synth import ProblemSpec, make_problem_gpu  # noqa: E402
from synth.problems import wedin_floor  # noqa: E402

pytestmark = pytest.mark.gpu
U = 2.0 ** -53
SPEC = dict(m=2_000_000, n=500, d=10_000, q=40, kappa=1e10, beta=1e-6, seed=0)


@pytest.fixture(scope="module")
def big():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    spec = ProblemSpec(**SPEC)
    p = make_problem_gpu(spec)
    ctx = ls.Context(0)
    ctx.set_option(ls.OPT_SEED, spec.sketch_seed)
    yield spec, p, ctx
    ctx.close()
    del p
    torch.cuda.empty_cache()


def test_fullsize_embedding_and_csr(big):
    spec, p, ctx = big
    m, d, s = spec.m, spec.d, spec.sketch_seed
    rows, signs = ctx.sketch_embedding(m, d, 8, s)
    er, es = oracle.sparse_sign(m, d, 8, s)
    assert np.array_equal(rows.cpu().numpy(), er)
    assert np.array_equal(signs.cpu().numpy(), es)
    rowptr, cols = ctx.sketch_csr(m, d, 8, s)
    r = er.ravel().astype(np.int64)
    j = np.repeat(np.arange(m, dtype=np.int64), 8)
    order = np.lexsort((j, r))
    exp_cols = (j[order] | ((es.ravel()[order] < 0).astype(np.int64) << 31)).astype(np.uint32).view(np.int32)
    exp_ptr = np.concatenate([[0], np.cumsum(np.bincount(r, minlength=d))]).astype(np.int32)
    assert np.array_equal(rowptr.cpu().numpy(), exp_ptr)
    assert np.array_equal(cols.cpu().numpy(), exp_cols)


def test_fullsize_sketch_rows_and_qr(big):
    spec, p, ctx = big
    m, n, d, s = spec.m, spec.n, spec.d, spec.sketch_seed
    A = p.A[:, :n]
    B, Sb = ctx.sketch(A, p.b, d, 8, s)
    er, es = oracle.sparse_sign(m, d, 8, s)
    Bh, Sbh = B.cpu().numpy(), Sb.cpu().numpy()
    for k in [0, 1, 4999, 7777, d - 1]:
        jj, ee = np.nonzero(er == k)                 # ascending j
        idx = torch.from_numpy(jj).cuda()
        rows_k = A.index_select(0, idx).cpu().numpy()
        bk = p.b.index_select(0, idx).cpu().numpy()[:, None]
        sg = es[jj, ee]
        assert np.array_equal(Bh[k], oracle.sketch_row(rows_k, sg, 8))
        assert Sbh[k] == oracle.sketch_row(bk, sg, 8)[0]
    # the whole sketch equals the per-row gather's (LS_OPT_GATHER = 1) bit for bit
    ctx.set_option(ls.OPT_GATHER, 1)
    try:
        B1, Sb1 = ctx.sketch(A, p.b, d, 8, s)
    finally:
        ctx.set_option(ls.OPT_GATHER, 0)
    assert torch.equal(B1, B) and torch.equal(Sb1, Sb)
    del B1, Sb1
    # QR of this sketch against the oracle's Householder QR of the same B, Sb
    R, x0 = ctx.qr_sketch(B, Sb)
    ctx.sync()
    R, x0 = R.cpu().numpy(), x0.cpu().numpy()
    xo, Ro, _, res = oracle.householder_lstsq(Bh, Sbh)
    nB = np.linalg.norm(Bh)
    assert np.all(np.tril(R, -1) == 0)
    assert np.linalg.norm(R.T @ R - Bh.T @ Bh) <= 20 * n * U * nB ** 2
    assert np.array_equal(np.sign(np.diag(R)), np.sign(np.diag(Ro)))
    # x0 agrees with the oracle's within the sketched problem's Wedin floor
    kap = np.linalg.cond(Bh)
    tol = 100 * kap * U * (np.linalg.norm(xo) + kap * res / np.linalg.norm(Bh, 2))
    assert np.linalg.norm(x0 - xo) <= tol


def test_fullsize_pass(big):
    spec, p, ctx = big
    n = spec.n
    A = p.A[:, :n]
    x = p.x_true + 1e-3 * torch.ones_like(p.x_true)
    c, rr = ctx.gradient(A, p.b, x)
    Ah = A.cpu().numpy()
    bh, xh = p.b.cpu().numpy(), x.cpu().numpy()
    ec, err = oracle.residual_gradient(Ah, bh, xh)
    aA = np.abs(Ah)
    r = bh - Ah @ xh
    m = spec.m
    bound = (n + 2) * U * (aA.T @ (np.abs(bh) + aA @ np.abs(xh))) + (m + 1) * U * (aA.T @ np.abs(r))
    assert np.all(np.abs(c.cpu().numpy() - ec) <= 2 * bound)
    assert abs(rr.cpu().numpy()[0] - err) <= 1e-9 * err


def test_fullsize_solve(big):
    spec, p, ctx = big
    n = spec.n
    A = p.A[:, :n]
    x1 = ctx.solve(A, p.b, spec.d, spec.q)
    x2 = ctx.solve(A, p.b, spec.d, spec.q)
    assert torch.equal(x1, x2)                           # deterministic
    fe = float(torch.linalg.norm(x1 - p.x_true))
    # The oracle: Householder least squares (Section 2.1, backward stable) in TSQR form on all of A
    # and b, on the host's cores.  Its forward error is the floor a backward-stable solver reaches
    # on this very problem (eq. ls_forward); the solve must land within 10x of it.
    xo, _, res = oracle.tsqr_lstsq(A.cpu().numpy(), p.b.cpu().numpy(), block_rows=8192,
                                   threads=min(16, len(os.sched_getaffinity(0))))
    fe_o = float(np.linalg.norm(xo - p.x_true.cpu().numpy()))
    print(f"forward error: GPU {fe:.3e}, Householder (TSQR) oracle {fe_o:.3e}, "
          f"Wedin floor {wedin_floor(spec.kappa, spec.beta):.3e}")
    assert abs(res - spec.beta) <= 1e-6 * spec.beta      # ||b - A x_o|| = ||r|| by construction
    assert fe <= 10 * fe_o
    assert fe_o <= wedin_floor(spec.kappa, spec.beta)
    r_true = p.b - A @ p.x_true
    re = float(torch.linalg.norm(r_true - (p.b - A @ x1)) / torch.linalg.norm(r_true))
    assert re <= 1e-3
