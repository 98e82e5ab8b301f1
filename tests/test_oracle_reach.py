"""Pins for the oracle functions that reach the benchmark sizes, and for two oracle helpers the GPU
tests lean on.

* orc_tsqr_lstsq: Householder least squares (Section 2.1) in TSQR form, checked against closed
  forms, exact rational arithmetic on tiny float problems, the residual evaluated in extended
  precision, LAPACK's R, the generator's known solution with Wedin's bound (eq. ls_forward), and the
  unblocked Householder solver; its tree must not depend on the thread count.
* orc_sketch_row: the per-row sum the full-size sketch test uses, bit-exact against orc_sketch.
* The stopping step of orc_iterative_sketching_stop (Section 3.3): the rule re-evaluated in x86
  extended precision on the oracle's own iterates stops at the same step.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
from synth import ProblemSpec, make_problem_cpu
from synth.problems import wedin_floor

U = 2.0 ** -53


# ------------------------------------------------------------------------------ TSQR form ---

@pytest.mark.parametrize("block_rows", [21, 42, 100, 4096])
def test_tsqr_kappa1_closed_form(block_rows):
    """kappa = 1: A = U1 V^T has orthonormal columns, so x = A^T b and ||b - A x|| = ||r||; a tree
    of many levels (fan-in 2 at block_rows = 42, n = 20) must still land on it."""
    p = make_problem_cpu(ProblemSpec(m=3001, n=20, kappa=1.0, beta=1e-3, seed=5))
    A = p.Aview
    x, R, res = oracle.tsqr_lstsq(p.A, p.b, 20, block_rows=block_rows, threads=4)
    assert np.linalg.norm(x - A.T @ p.b) < 2e-14
    assert np.linalg.norm(x - p.x_true) < 2e-14
    assert abs(res - 1e-3) < 1e-14
    # R^T R = A^T A = I
    assert np.linalg.norm(R.T @ R - np.eye(20)) < 1e-13


def test_tsqr_n1_closed_form():
    a = np.random.default_rng(15).standard_normal((997, 1))
    b = np.random.default_rng(16).standard_normal(997)
    x, R, res = oracle.tsqr_lstsq(a, b, block_rows=7, threads=3)
    assert abs(x[0] - (a[:, 0] @ b) / (a[:, 0] @ a[:, 0])) < 1e-14 * abs(x[0])
    assert abs(abs(R[0, 0]) - np.linalg.norm(a)) < 1e-14 * np.linalg.norm(a)
    assert abs(res - np.linalg.norm(b - a[:, 0] * x[0])) < 1e-13 * res


def _exact_lstsq(A, b):
    """Exact least-squares solution of the float data (every double is a dyadic rational) by the
    normal equations in rational arithmetic."""
    m, n = A.shape
    Af = [[Fraction(float(A[i, c])) for c in range(n)] for i in range(m)]
    bf = [Fraction(float(b[i])) for i in range(m)]
    G = [[sum(Af[i][r] * Af[i][c] for i in range(m)) for c in range(n)] for r in range(n)]
    h = [sum(Af[i][r] * bf[i] for i in range(m)) for r in range(n)]
    for k in range(n):
        piv = next(r for r in range(k, n) if G[r][k] != 0)
        G[k], G[piv] = G[piv], G[k]
        h[k], h[piv] = h[piv], h[k]
        for r in range(n):
            if r != k and G[r][k] != 0:
                f = G[r][k] / G[k][k]
                G[r] = [G[r][c] - f * G[k][c] for c in range(n)]
                h[r] -= f * h[k]
    x = [h[k] / G[k][k] for k in range(n)]
    r2 = sum((bf[i] - sum(Af[i][c] * x[c] for c in range(n))) ** 2 for i in range(m))
    return np.array([float(v) for v in x]), math.sqrt(float(r2))


@pytest.mark.parametrize("seed", range(5))
def test_tsqr_brute_force_rational(seed):
    """Tiny float problems, several row blocks and levels, ragged last blocks: against the exact
    rational solution, within the perturbation bound of a backward-stable solver."""
    rng = np.random.default_rng(200 + seed)
    n = int(rng.integers(1, 5))
    m = int(rng.integers(6 * (n + 1), 60))
    A = rng.standard_normal((m, n)) * np.logspace(0, -3, n)
    b = rng.standard_normal(m)
    xex, rex = _exact_lstsq(A, b)
    for br in sorted({n + 1, 2 * (n + 1) + 1, 3 * (n + 1)}):
        x, R, res = oracle.tsqr_lstsq(A, b, block_rows=br, threads=2)
        kap = np.linalg.cond(A)
        bound = 50 * kap * U * (np.linalg.norm(xex) + kap * rex / np.linalg.norm(A, 2)) + 50 * U * np.linalg.norm(xex)
        assert np.linalg.norm(x - xex) <= bound, (br, np.linalg.norm(x - xex), bound)
        assert abs(res - rex) <= 1e-12 * max(rex, 1.0)


@pytest.mark.parametrize("kappa,beta", [(1e2, 1e-3), (1e10, 1e-6), (1e10, 1e-3), (1e14, 1e-12)])
def test_tsqr_forward_error_within_wedin(kappa, beta):
    """The generator's x is the least-squares solution: a backward-stable solver lands within a
    small multiple of kappa u (||x|| + kappa ||r||) of it, as the unblocked solver does."""
    p = make_problem_cpu(ProblemSpec(m=6000, n=40, kappa=kappa, beta=beta, seed=6))
    x, _, res = oracle.tsqr_lstsq(p.A, p.b, 40, block_rows=512, threads=4)
    xh, _, _, _ = oracle.householder_lstsq(p.Aview, p.b)
    floor = wedin_floor(kappa, beta)
    assert np.linalg.norm(x - p.x_true) <= 100 * floor
    assert np.linalg.norm(x - xh) <= 200 * floor
    if kappa <= 1e10:
        assert abs(res - beta) <= 1e-2 * beta + 10 * U * np.linalg.norm(p.b)


@pytest.mark.parametrize("kappa", [1e2, 1e8])
def test_tsqr_residual_extended_precision(kappa):
    """|T[n, n]| is ||b - A x||: re-evaluated in x86 extended precision; and the normal equations
    A^T (b - A x) = 0 hold to the backward-stable level."""
    p = make_problem_cpu(ProblemSpec(m=5000, n=30, kappa=kappa, beta=1e-4, seed=7))
    A = p.Aview
    x, _, res = oracle.tsqr_lstsq(p.A, p.b, 30, block_rows=300, threads=4)
    Al, bl, xl = (v.astype(np.longdouble) for v in (A, p.b, x))
    r = bl - Al @ xl
    rn = float(np.sqrt((r * r).sum()))
    assert abs(res - rn) <= 1e-9 * rn
    g = np.linalg.norm((Al.T @ r).astype(np.float64))
    assert g / (np.linalg.norm(x) + kappa * rn) < 1e3 * U


@pytest.mark.parametrize("kappa", [1e1, 1e4])
def test_tsqr_R_matches_lapack_up_to_row_signs(kappa):
    """R is unique up to the signs of its rows: D R_tsqr against LAPACK's geqrf R."""
    p = make_problem_cpu(ProblemSpec(m=4000, n=25, kappa=kappa, beta=1e-2, seed=8))
    A = p.Aview
    _, R, _ = oracle.tsqr_lstsq(p.A, p.b, 25, block_rows=130, threads=4)
    Rl = np.linalg.qr(A, mode="r")
    D = np.sign(np.diag(R)) * np.sign(np.diag(Rl))
    assert np.all(np.tril(R, -1) == 0)
    assert np.allclose(D[:, None] * R, Rl, rtol=0, atol=1e3 * 25 * U * kappa * np.linalg.norm(A, 2))


def test_tsqr_threads_and_tree_invariants():
    """The tree does not depend on the thread count (bitwise); a single block is the unblocked
    solver exactly; a different tree still agrees within the floor."""
    p = make_problem_cpu(ProblemSpec(m=9001, n=33, kappa=1e6, beta=1e-6, seed=9))
    a = oracle.tsqr_lstsq(p.A, p.b, 33, block_rows=250, threads=1)
    b = oracle.tsqr_lstsq(p.A, p.b, 33, block_rows=250, threads=7)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and a[2] == b[2]
    one = oracle.tsqr_lstsq(p.A, p.b, 33, block_rows=9001, threads=3)
    xh, Rh, _, resh = oracle.householder_lstsq(p.Aview, p.b)
    assert np.array_equal(one[0], xh) and np.array_equal(one[1], Rh) and one[2] == resh
    assert np.linalg.norm(a[0] - xh) <= 100 * wedin_floor(1e6, 1e-6)


def test_tsqr_bad_arguments():
    A = np.ones((10, 3))
    with pytest.raises(ValueError):
        oracle.tsqr_lstsq(A, np.ones(10), block_rows=3)       # block_rows < n + 1
    A = np.random.default_rng(0).standard_normal((400, 4))
    A[:, 2] = 0.0
    with pytest.raises(np.linalg.LinAlgError):
        oracle.tsqr_lstsq(A, np.ones(400), block_rows=50)


# --------------------------------------------------------------------------- orc_sketch_row ---

@pytest.mark.parametrize("m,n,d,zeta", [(3000, 7, 200, 8), (1500, 33, 40, 4), (700, 5, 9, 8)])
def test_sketch_row_equals_full_sketch(m, n, d, zeta):
    """Every row of orc_sketch equals orc_sketch_row on that row's terms in ascending j."""
    rng = np.random.default_rng(m + n)
    A = rng.standard_normal((m, n)) * rng.choice([1.0, 1e-8, 1e8], size=(m, 1))
    b = rng.standard_normal(m)
    B, Sb = oracle.sketch(A, b, n, d, zeta, 21)
    rows, signs = oracle.sparse_sign(m, d, zeta, 21)
    for k in range(d):
        jj, ee = np.nonzero(rows == k)            # row-major scan: ascending j
        sg = signs[jj, ee]
        assert np.array_equal(B[k], oracle.sketch_row(A[jj], sg, zeta))
        assert Sb[k] == oracle.sketch_row(b[jj, None], sg, zeta)[0]


# ------------------------------------------------------------ Section 3.3 stopping step ---

@pytest.mark.parametrize("kappa,beta,seed", [(1e10, 1e-6, 8), (1e4, 1e-3, 3), (1.0, 1e-6, 4), (1e12, 1e-10, 5)])
def test_stopping_step_reevaluated_in_extended_precision(kappa, beta, seed):
    """Run Algorithm 2 for qmax steps (orc_iterative_sketching keeps every iterate); evaluate the
    Section 3.3 rule on x_{i+1} against x_i in long double with the oracle's normest and condest:
    the first step that satisfies it is the one orc_iterative_sketching_stop returned.  A rule on
    ||r(x_i)|| in place of ||r(x_{i+1})||, or one step late or early, gives a different index."""
    p = make_problem_cpu(ProblemSpec(m=4000, n=50, kappa=kappa, beta=beta, seed=seed))
    n, d, qmax = 50, 1000, 120
    g = oracle.normest_start(n, 99)
    x_stop, it, ne, ce = oracle.iterative_sketching_stop(p.A, p.b, n, d, qmax, g, seed=p.spec.sketch_seed)
    _, xh, _, _ = oracle.iterative_sketching(p.A, p.b, n, d, qmax, seed=p.spec.sketch_seed, history=True)
    assert np.array_equal(xh[it], x_stop)            # the same iterates
    Al = p.Aview.astype(np.longdouble)
    bl = p.b.astype(np.longdouble)
    u = np.longdouble(U)
    first, margins = None, []
    for i in range(qmax):
        xi, xn = xh[i].astype(np.longdouble), xh[i + 1].astype(np.longdouble)
        dr = np.sqrt(((Al @ (xn - xi)) ** 2).sum())
        rr = np.sqrt(((bl - Al @ xn) ** 2).sum())
        rhs = u * (np.longdouble(1.0) * np.longdouble(ne) * np.sqrt((xn * xn).sum())
                   + np.longdouble(0.04) * np.longdouble(ce) * rr)
        margins.append(float(abs(dr - rhs) / rhs))
        if dr <= rhs:
            first = i + 1
            break
    assert first is not None
    assert 2 <= it < qmax
    assert margins[-1] > 1e-6          # the decision is not within rounding of the threshold
    assert first == it


def test_stopping_step_uses_the_new_residual():
    """The rule compares ||r(x_{i+1}) - r(x_i)|| with rho condest ||r(x_{i+1})|| (gamma = 0 here).
    With rho set strictly between the values at which the first step would stop under
    ||r(x_{i+1})|| and under ||r(x_i)|| (the latter is larger), only the correct reading goes on
    past the first step, and it must stop where the extended-precision evaluation says."""
    p = make_problem_cpu(ProblemSpec(m=4000, n=50, kappa=1e3, beta=1e-9, seed=12))
    n, d, qmax = 50, 1000, 60
    g = oracle.normest_start(n, 99)
    _, xh, _, _ = oracle.iterative_sketching(p.A, p.b, n, d, qmax, seed=p.spec.sketch_seed, history=True)
    _, _, ne, ce = oracle.iterative_sketching_stop(p.A, p.b, n, d, 1, g, seed=p.spec.sketch_seed)
    Al, bl = p.Aview.astype(np.longdouble), p.b.astype(np.longdouble)
    u = np.longdouble(U)

    def parts(i):
        xi, xn = xh[i].astype(np.longdouble), xh[i + 1].astype(np.longdouble)
        dr = np.sqrt(((Al @ (xn - xi)) ** 2).sum())
        return dr, np.sqrt(((bl - Al @ xi) ** 2).sum()), np.sqrt(((bl - Al @ xn) ** 2).sum())

    dr0, r0, r1 = parts(0)
    P0 = dr0 / (u * np.longdouble(ce) * r1)          # smallest rho that stops at step 1 (correct)
    M0 = dr0 / (u * np.longdouble(ce) * r0)          # the same under ||r(x_0)||
    assert M0 < P0 * (1 - 1e-6)
    rho = float(np.sqrt(M0 * P0))
    first = None
    for i in range(qmax):
        dr, _, rn = parts(i)
        if dr <= u * np.longdouble(rho) * np.longdouble(ce) * rn:
            first = i + 1
            break
    _, it, _, _ = oracle.iterative_sketching_stop(p.A, p.b, n, d, qmax, g, seed=p.spec.sketch_seed,
                                                  gamma=0.0, rho=rho)
    assert first is not None and first >= 2
    assert it == first
