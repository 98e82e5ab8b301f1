"""Pins for the CPU oracle: each checks it against something other than itself.

Sources of truth used here: published SplitMix64 outputs (tests/golden), closed forms (kappa = 1,
n = 1), exact rational arithmetic on tiny integer problems, the problem generator's known solution
with Wedin's bound (Fact 2.1 / eq. ls_forward), the normal equations evaluated in extended
precision, LAPACK (numpy/scipy) as an independent implementation, the singular-value bounds of a
subspace embedding (Fact 2.2), and the convergence theorems of Sections 3.1 and 6.
"""
import math
import os
from fractions import Fraction

import numpy as np
import pytest
import scipy.linalg
import scipy.special

import oracle
from synth import ProblemSpec, integer_problem, make_problem_cpu
from synth.problems import wedin_floor

U = 2.0 ** -53
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def dense_S(m, d, zeta, seed, scaled=True):
    rows, signs = oracle.sparse_sign(m, d, zeta, seed)
    S = np.zeros((d, m))
    for j in range(m):
        S[rows[j], j] = signs[j]
    return S / math.sqrt(zeta) if scaled else S


# ---------------------------------------------------------------- SplitMix64 / sparse sign ---

def test_splitmix64_published_outputs():
    with open(os.path.join(GOLDEN, "splitmix64_seed0.txt")) as f:
        rows = [ln.split() for ln in f if ln.strip() and not ln.startswith("#")]
    for k, hx in rows:
        assert oracle.splitmix64(0, int(k)) == int(hx, 16)


@pytest.mark.parametrize("m,d,zeta", [(5000, 1000, 8), (3000, 16, 8), (200, 8, 8), (100, 3, 1)])
def test_sparse_sign_structure(m, d, zeta):
    rows, signs = oracle.sparse_sign(m, d, zeta, seed=7)
    assert rows.min() >= 0 and rows.max() < d
    for j in range(m):
        assert len(set(rows[j].tolist())) == zeta          # exactly zeta distinct positions
    assert set(np.unique(signs).tolist()) <= {-1, 1}
    S = dense_S(m, d, zeta, 7)
    assert np.allclose(np.linalg.norm(S, axis=0), 1.0, rtol=0, atol=4 * U)  # unit columns


def test_sparse_sign_uniform_positions_and_signs():
    m, d, zeta = 40000, 100, 8
    rows, signs = oracle.sparse_sign(m, d, zeta, seed=11)
    counts = np.bincount(rows.ravel(), minlength=d)
    expect = m * zeta / d
    chi2 = float(((counts - expect) ** 2 / expect).sum())
    # positions without replacement are still marginally uniform; chi-square with d-1 dof
    from scipy.stats import chi2 as chi2dist
    assert chi2 < chi2dist.ppf(0.9999, d - 1)
    npos = int((signs > 0).sum())
    tot = signs.size
    assert abs(npos - tot / 2) < 5 * math.sqrt(tot / 4)     # fair signs
    # signs independent of positions: positive fraction similar in every row
    posfrac = np.bincount(rows.ravel(), weights=(signs.ravel() > 0), minlength=d) / counts
    assert np.all(np.abs(posfrac - 0.5) < 6 * np.sqrt(0.25 / counts))


def test_sparse_sign_seed_and_determinism():
    a = oracle.sparse_sign(1000, 500, 8, 1)
    b = oracle.sparse_sign(1000, 500, 8, 1)
    c = oracle.sparse_sign(1000, 500, 8, 2)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert not np.array_equal(a[0], c[0])
    # columns are a prefix-stable function of j: a longer m leaves earlier columns unchanged
    e = oracle.sparse_sign(1500, 500, 8, 1)
    assert np.array_equal(e[0][:1000], a[0])


def test_sparse_sign_is_subspace_embedding():
    """Fact 2.2 input: for d = 20 n the singular values of S U1 lie near 1 +- sqrt(n/d)."""
    m, n, d = 4000, 50, 1000
    U1, _ = np.linalg.qr(np.random.default_rng(0).standard_normal((m, n)))
    sv = np.linalg.svd(dense_S(m, d, 8, 3) @ U1, compute_uv=False)
    eps = math.sqrt(n / d)
    assert sv.max() < 1 + 1.5 * eps and sv.min() > 1 - 1.5 * eps


# ----------------------------------------------------------------------------- sketch B = S A

def test_sketch_integer_exact():
    m, n, d, zeta = 700, 9, 60, 8
    A, b, _ = integer_problem(m, n, seed=4)
    B, Sb = oracle.sketch(A, b, n, d, zeta, seed=5)
    S1 = dense_S(m, d, zeta, 5, scaled=False)              # +-1 entries
    s = 1.0 / math.sqrt(zeta)
    assert np.array_equal(B, (S1 @ A[:, :n]) * s)          # integer sums are exact in FP64
    assert np.array_equal(Sb, (S1 @ b) * s)


def test_sketch_float_within_summation_bound():
    m, n, d, zeta = 3000, 17, 200, 8
    A = np.random.default_rng(1).standard_normal((m, n))
    b = np.random.default_rng(2).standard_normal(m)
    B, Sb = oracle.sketch(A, b, n, d, zeta, seed=9)
    S = dense_S(m, d, zeta, 9)
    Bx = (S.astype(np.longdouble) @ A.astype(np.longdouble))
    k = int(np.count_nonzero(S, axis=1).max())
    bound = (k + 1) * U * (np.abs(S) @ np.abs(A))
    assert np.all(np.abs(B - Bx) <= bound)
    assert np.allclose(Sb, S @ b, rtol=0, atol=1e-12)


def test_sketch_padded_lda():
    m, n, d = 500, 7, 70
    A, b, _ = integer_problem(m, n, lda=16, seed=8)
    B1, _ = oracle.sketch(A, b, n, d, 8, 3)
    B2, _ = oracle.sketch(np.ascontiguousarray(A[:, :n]), b, n, d, 8, 3)
    assert np.array_equal(B1, B2)


# --------------------------------------------------------------- Householder least squares ---

def test_lstsq_kappa1_closed_form():
    """kappa = 1: A has orthonormal columns, so x = A^T b."""
    p = make_problem_cpu(ProblemSpec(m=2000, n=40, kappa=1.0, beta=1e-3, seed=1))
    A = p.Aview
    x, R, _, res = oracle.householder_lstsq(A, p.b)
    assert np.linalg.norm(x - A.T @ p.b) < 1e-14
    assert np.linalg.norm(x - p.x_true) < 1e-14
    assert abs(res - 1e-3) < 1e-15


def test_lstsq_n1_closed_form():
    a = np.random.default_rng(5).standard_normal((300, 1))
    b = np.random.default_rng(6).standard_normal(300)
    x, R, _, _ = oracle.householder_lstsq(a, b)
    assert abs(x[0] - (a[:, 0] @ b) / (a[:, 0] @ a[:, 0])) < 1e-14 * abs(x[0])
    assert abs(abs(R[0, 0]) - np.linalg.norm(a)) < 1e-14 * np.linalg.norm(a)


@pytest.mark.parametrize("seed", range(6))
def test_lstsq_brute_force_rational(seed):
    rng = np.random.default_rng(100 + seed)
    m, n = int(rng.integers(5, 17)), int(rng.integers(1, 5))
    A = rng.integers(-3, 4, size=(m, n)).astype(float)
    if np.linalg.matrix_rank(A) < n:
        A[:n, :n] += 7 * np.eye(n)
    b = rng.integers(-3, 4, size=m).astype(float)
    # exact x from the normal equations in rational arithmetic
    G = [[Fraction(int(sum(A[i, r] * A[i, c] for i in range(m)))) for c in range(n)] for r in range(n)]
    h = [Fraction(int(sum(A[i, r] * b[i] for i in range(m)))) for r in range(n)]
    for k in range(n):                                      # Gauss-Jordan, exact
        piv = next(r for r in range(k, n) if G[r][k] != 0)
        G[k], G[piv] = G[piv], G[k]
        h[k], h[piv] = h[piv], h[k]
        for r in range(n):
            if r != k and G[r][k] != 0:
                f = G[r][k] / G[k][k]
                G[r] = [G[r][c] - f * G[k][c] for c in range(n)]
                h[r] -= f * h[k]
    xex = np.array([float(h[k] / G[k][k]) for k in range(n)])
    x, _, _, _ = oracle.householder_lstsq(A, b)
    kap = np.linalg.cond(A)
    assert np.linalg.norm(x - xex) <= 50 * kap ** 2 * U * max(1.0, np.linalg.norm(xex))


@pytest.mark.parametrize("kappa,beta", [(1e1, 1e-12), (1e10, 1e-6), (1e10, 1e-3), (1e15, 1e-12)])
def test_lstsq_forward_error_within_wedin(kappa, beta):
    """A backward-stable solver lands within a small multiple of kappa u (||x|| + kappa ||r||)."""
    p = make_problem_cpu(ProblemSpec(m=3000, n=40, kappa=kappa, beta=beta, seed=2))
    x, _, _, res = oracle.householder_lstsq(p.Aview, p.b)
    fe = np.linalg.norm(x - p.x_true)
    floor = wedin_floor(kappa, beta)
    assert fe <= 100 * floor
    if kappa <= 1e10:
        assert abs(res - beta) <= 1e-2 * beta + 10 * U * np.linalg.norm(p.b)


@pytest.mark.parametrize("kappa", [1e2, 1e8, 1e12])
def test_lstsq_normal_equations_extended_precision(kappa):
    p = make_problem_cpu(ProblemSpec(m=2500, n=30, kappa=kappa, beta=1e-4, seed=3))
    A = p.Aview
    x, _, _, _ = oracle.householder_lstsq(A, p.b)
    Al, bl, xl = (v.astype(np.longdouble) for v in (A, p.b, x))
    r = bl - Al @ xl
    g = np.linalg.norm((Al.T @ r).astype(np.float64))
    scale = 1.0 * (1.0 * np.linalg.norm(x) + kappa * float(np.linalg.norm(r.astype(np.float64))))
    assert g / scale < 1e3 * U


@pytest.mark.parametrize("kappa", [1e2, 1e6])
def test_lstsq_matches_lapack(kappa):
    p = make_problem_cpu(ProblemSpec(m=1500, n=25, kappa=kappa, beta=1e-2, seed=4))
    A = p.Aview
    x, R, _, _ = oracle.householder_lstsq(A, p.b)
    xl = np.linalg.lstsq(A, p.b, rcond=None)[0]
    assert np.linalg.norm(x - xl) <= 20 * wedin_floor(kappa, 1e-2)
    Rl = np.linalg.qr(A, mode="r")          # LAPACK geqrf: same beta = -sign(alpha)||x|| rule
    assert np.allclose(R, Rl, rtol=0, atol=1e3 * U * np.linalg.norm(A, 2))
    assert np.allclose(np.tril(R, -1), 0.0)


def test_lstsq_rank_deficient_raises():
    A = np.random.default_rng(0).standard_normal((50, 4))
    A[:, 2] = 0.0
    with pytest.raises(np.linalg.LinAlgError):
        oracle.householder_lstsq(A, np.ones(50))


# ------------------------------------------------------------- residual gradient / solves ---

def test_residual_gradient_integer_exact():
    A, b, x = integer_problem(400, 11, seed=3)
    c, rr = oracle.residual_gradient(A, b, x, n=11)
    Ai = A[:, :11].astype(np.int64)
    r = b.astype(np.int64) - Ai @ x.astype(np.int64)
    assert np.array_equal(c, (Ai.T @ r).astype(float))
    assert rr == float(r @ r)


def test_residual_gradient_float_bound():
    m, n = 5000, 23
    rng = np.random.default_rng(8)
    A, b, x = rng.standard_normal((m, n)), rng.standard_normal(m), rng.standard_normal(n)
    c, rr = oracle.residual_gradient(A, b, x)
    Al = A.astype(np.longdouble)
    r = b - Al @ x
    cx = Al.T @ r
    aA = np.abs(A)
    bound = (n + 2) * U * aA.T @ (np.abs(b) + aA @ np.abs(x)) + (m + 1) * U * aA.T @ np.abs(r.astype(float))
    assert np.all(np.abs(c - cx.astype(float)) <= bound)
    assert abs(rr - float(r @ r)) <= 1e-12 * float(r @ r)


def test_triangular_solves_match_lapack():
    n = 60
    rng = np.random.default_rng(9)
    R = np.triu(rng.standard_normal((n, n))) + 4 * np.eye(n)
    c = rng.standard_normal(n)
    y = oracle.solve_rt(R, c)
    d = oracle.solve_r(R, y)
    y2 = scipy.linalg.solve_triangular(R, c, trans="T", lower=False)
    d2 = scipy.linalg.solve_triangular(R, y2, lower=False)
    assert np.allclose(y, y2, rtol=1e-12, atol=1e-12)
    assert np.allclose(d, d2, rtol=1e-12, atol=1e-12)
    # componentwise backward error of substitution (Higham Thm 8.5): |T y - c| <= gamma_n |T||y|
    assert np.all(np.abs(R.T @ y - c) <= (n + 1) * U * (np.abs(R.T) @ np.abs(y)) * 2)
    assert np.all(np.abs(R @ d - y) <= (n + 1) * U * (np.abs(R) @ np.abs(d)) * 2)


def test_triangular_solves_integer_exact():
    n = 12
    rng = np.random.default_rng(10)
    R = np.triu(rng.integers(-2, 3, size=(n, n)).astype(float), 1) + np.eye(n)
    xt = rng.integers(-3, 4, size=n).astype(float)
    assert np.array_equal(oracle.solve_r(R, R @ xt), xt)
    assert np.array_equal(oracle.solve_rt(R, R.T @ xt), xt)


# ---------------------------------------------------------------- iterative sketching (Alg 2)

def _config1(kappa=1e10, beta=1e-6, seed=0, m=4000, n=50):
    return make_problem_cpu(ProblemSpec(m=m, n=n, kappa=kappa, beta=beta, seed=seed, d=20 * n))


def test_q0_is_sketch_and_solve():
    """x_0 = argmin ||S b - S A y|| (eq. sketched_ls), checked with LAPACK on the dense sketch."""
    p = _config1(kappa=1e3, beta=1e-2)
    n, d, s = 50, 1000, p.spec.sketch_seed
    x0 = oracle.iterative_sketching(p.A, p.b, n, d, 0, seed=s)
    S = dense_S(p.spec.m, d, 8, s)
    SA, Sb = S @ p.Aview, S @ p.b
    xl = np.linalg.lstsq(SA, Sb, rcond=None)[0]
    kap = np.linalg.cond(SA)
    rs = np.linalg.norm(Sb - SA @ xl)
    assert np.linalg.norm(x0 - xl) <= 50 * kap * U * (np.linalg.norm(xl) + kap * rs)
    # Fact 2.3: sketch-and-solve residual within (1+eps)/(1-eps) of optimal
    eps = math.sqrt(n / d)
    assert np.linalg.norm(p.b - p.Aview @ x0) <= (1 + 2 * eps) / (1 - 2 * eps) * 1e-2


def test_contraction_by_G():
    """Section 3.4: ||R(x - x_{i+1})|| <= ||G|| ||R(x - x_i)||, G = I - R^{-T} A^T A R^{-1}."""
    p = _config1(kappa=1e4, beta=1e-3, seed=1)
    n, d = 50, 1000
    xq, xh, R, _ = oracle.iterative_sketching(p.A, p.b, n, d, 25, seed=p.spec.sketch_seed,
                                              history=True)
    A = p.Aview
    AR = scipy.linalg.solve_triangular(R, A.T, trans="T", lower=False).T   # A R^{-1}
    G = np.eye(n) - AR.T @ AR
    g = np.linalg.norm(G, 2)
    sv = np.linalg.svd(AR, compute_uv=False)
    eps = max(1 - 1 / sv.max(), 1 / sv.min() - 1)                  # realised distortion
    assert g <= (2 - eps) * eps / (1 - eps) ** 2 + 1e-12             # eq. itsk-rate
    errs = [np.linalg.norm(R @ (p.x_true - xh[i])) for i in range(26)]
    # ||R e|| ~ ||A e||, whose floor is u (||A|| ||x|| + kappa ||r||) (eq. residual_error)
    floor = 100 * U * (1 + 1e4 * 1e-3) * np.linalg.norm(R, 2)
    checked = 0
    for i in range(25):
        if errs[i] > 1e3 * floor:
            assert errs[i + 1] <= g * errs[i] * (1 + 1e-6) + floor
            checked += 1
    assert checked >= 5


@pytest.mark.parametrize("kappa,beta", [(1e1, 1e-12), (1e10, 1e-6), (1e10, 1e-3), (1e15, 1e-12)])
def test_converges_to_householder_accuracy(kappa, beta):
    """Theorem 5.1 / Fig. numerical: forward and residual errors reach Householder's level."""
    p = _config1(kappa=kappa, beta=beta, seed=2)
    n = 50
    xh_ref, _, _, _ = oracle.householder_lstsq(p.Aview, p.b)
    fe_ref = np.linalg.norm(xh_ref - p.x_true)
    x = oracle.iterative_sketching(p.A, p.b, n, 1000, 60, seed=p.spec.sketch_seed)
    fe = np.linalg.norm(x - p.x_true)
    assert fe <= 10 * max(fe_ref, 1e-15) + 10 * U
    r_true = p.b - p.Aview @ p.x_true
    re = np.linalg.norm(r_true - (p.b - p.Aview @ x)) / np.linalg.norm(r_true)
    re_ref = np.linalg.norm(r_true - (p.b - p.Aview @ xh_ref)) / np.linalg.norm(r_true)
    assert re <= 10 * re_ref + 1e-15 / beta


def test_kappa1_reaches_1e12():
    p = _config1(kappa=1.0, beta=1e-6, seed=3)
    x = oracle.iterative_sketching(p.A, p.b, 50, 1000, 40, seed=p.spec.sketch_seed)
    assert np.linalg.norm(x - p.x_true) <= 1e-12


def test_config1_q30_within_10x_householder():
    p = _config1()
    xh_ref, _, _, _ = oracle.householder_lstsq(p.Aview, p.b)
    x = oracle.iterative_sketching(p.A, p.b, 50, 1000, 30, seed=p.spec.sketch_seed)
    assert np.linalg.norm(x - p.x_true) <= 10 * np.linalg.norm(xh_ref - p.x_true)


def test_negative_controls_fail():
    """The unstable variants of Section 3.2 must fail the same tolerance (kappa=1e10, ||r||=1e-6)."""
    p = _config1(seed=4)
    n, d, q = 50, 1000, 60
    A, b = p.Aview, p.b
    xh_ref, _, _, _ = oracle.householder_lstsq(A, b)
    tol = 10 * np.linalg.norm(xh_ref - p.x_true)
    _, _, R, _ = oracle.iterative_sketching(p.A, b, n, d, 0, seed=p.spec.sketch_seed, history=True)
    x0 = oracle.iterative_sketching(p.A, b, n, d, 0, seed=p.spec.sketch_seed)
    # bad residual: A^T b - A^T (A x)
    Atb = A.T @ b
    x = x0.copy()
    for _ in range(q):
        c = Atb - A.T @ (A @ x)
        x = x + oracle.solve_r(R, oracle.solve_rt(R, c))
    assert np.linalg.norm(x - p.x_true) > tol
    # bad matrix: factor the explicit Gram matrix (SA)^T (SA) by LU
    B, Sb = oracle.sketch(p.A, b, n, d, 8, p.spec.sketch_seed)
    lu = scipy.linalg.lu_factor(B.T @ B)
    x = x0.copy()
    for _ in range(q):
        c, _ = oracle.residual_gradient(A, b, x)
        x = x + scipy.linalg.lu_solve(lu, c)
    assert not np.all(np.isfinite(x)) or np.linalg.norm(x - p.x_true) > tol
    # bad initial x_0 = 0: same q reaches far less accuracy
    x = np.zeros(n)
    for _ in range(30):
        c, _ = oracle.residual_gradient(A, b, x)
        x = x + oracle.solve_r(R, oracle.solve_rt(R, c))
    x30 = oracle.iterative_sketching(p.A, b, n, d, 30, seed=p.spec.sketch_seed)
    assert np.linalg.norm(x - p.x_true) > 10 * np.linalg.norm(x30 - p.x_true)


def test_wrong_scale_breaks_convergence():
    """A planted mistake in the sketch scale must be visible.  With S too large by sqrt(zeta) each
    step d_i is zeta times too short (convergence stalls); with S too small by sqrt(zeta) each step
    is zeta times too long (divergence)."""
    p = _config1(kappa=1e3, beta=1e-6, seed=5)
    n, d = 50, 1000
    good = oracle.iterative_sketching(p.A, p.b, n, d, 30, seed=p.spec.sketch_seed)
    e_good = np.linalg.norm(good - p.x_true)
    assert e_good < 1e-9
    B, Sb = oracle.sketch(p.A, p.b, n, d, 8, p.spec.sketch_seed)
    for f in (math.sqrt(8), 1 / math.sqrt(8)):
        x0, R, _, _ = oracle.householder_lstsq(B * f, Sb * f)
        x = x0.copy()
        for _ in range(30):
            c, _ = oracle.residual_gradient(p.A, p.b, x, n=n)
            x = x + oracle.solve_r(R, oracle.solve_rt(R, c))
        assert not np.isfinite(np.linalg.norm(x)) or np.linalg.norm(x - p.x_true) > 100 * e_good


# ---------------------------------------------------------------- damping / momentum (Sec 6)

def test_damping_momentum_rates():
    """Theorem 6.1: damping contracts at 2 eps/(1+eps^2), momentum at eps; both beat plain."""
    p = _config1(kappa=1e3, beta=1e-2, seed=6)
    n, d, q = 50, 1000, 25
    eps = math.sqrt(n / d)
    xr = oracle.householder_lstsq(p.Aview, p.b)[0]
    _, hp, _, _ = oracle.iterative_sketching(p.A, p.b, n, d, q, seed=p.spec.sketch_seed, history=True)
    _, hd = oracle.iterative_sketching_dm(p.A, p.b, n, d, q, (1 - eps**2) ** 2 / (1 + eps**2), 0.0,
                                          seed=p.spec.sketch_seed)
    _, hm = oracle.iterative_sketching_dm(p.A, p.b, n, d, q, (1 - eps**2) ** 2, eps**2,
                                          seed=p.spec.sketch_seed)

    def rate(h, i0=2, i1=12):
        e = np.linalg.norm(h - xr, axis=1)
        return (e[i1] / e[i0]) ** (1.0 / (i1 - i0))
    rp, rd, rm = rate(hp), rate(hd), rate(hm)
    assert rd < rp and rm < rd
    assert rm < 1.5 * eps and rd < 1.5 * 2 * eps / (1 + eps ** 2)
    # damping with alpha = 1, beta = 0 is exactly Algorithm 2
    _, h1 = oracle.iterative_sketching_dm(p.A, p.b, n, d, 5, 1.0, 0.0, seed=p.spec.sketch_seed)
    assert np.array_equal(h1, hp[:6])


# ----------------------------------------------------------------- Section 3.3 estimators ---

def test_normest_condest():
    n = 80
    rng = np.random.default_rng(12)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    R = np.linalg.qr(Q * np.logspace(0, -6, n), mode="r")
    g = rng.standard_normal(n)
    est = oracle.normest(R, g, int(math.ceil(math.log(n))) + 10)
    true2 = np.linalg.norm(R, 2)
    assert 0.8 * true2 <= est <= true2 * (1 + 1e-12)
    ce = oracle.condest_1(R)
    k1 = np.linalg.norm(R, 1) * np.linalg.norm(np.linalg.inv(R), 1)
    assert k1 / 10 <= ce <= k1 * (1 + 1e-9)


def test_dimension_rule():
    for m, n in [(4000, 50), (2_000_000, 500), (10**6, 1000), (4 * 10**6, 2000), (100, 10)]:
        d = oracle.dimension(m, n)
        a, c = 6 + 4 * math.sqrt(2), 6 - 4 * math.sqrt(2)
        w = scipy.special.lambertw(c * m / n**2 * math.log(2.0**53)).real
        assert d == max(math.ceil(a * n * math.exp(w)), 20 * n)
        assert d >= 20 * n


# ------------------------------------------------------- Section 3.3 stopping rule (NEXT-4)

@pytest.mark.parametrize("kappa,beta", [(1e1, 1e-12), (1e10, 1e-6), (1e10, 1e-3), (1e15, 1e-12), (1.0, 1e-6)])
def test_stopping_rule_reaches_householder_accuracy(kappa, beta):
    """Section 3.3: the rule stops at forward and residual errors a small multiple of Householder's."""
    p = _config1(kappa=kappa, beta=beta, seed=8)
    n, d = 50, 1000
    g = oracle.normest_start(n, 99)
    x, it, ne, ce = oracle.iterative_sketching_stop(p.A, p.b, n, d, 200, g, seed=p.spec.sketch_seed)
    xh = oracle.householder_lstsq(p.Aview, p.b)[0]
    fe, fe_h = np.linalg.norm(x - p.x_true), np.linalg.norm(xh - p.x_true)
    assert 1 <= it < 200
    assert fe <= 10 * max(fe_h, 1e-15) + 10 * U
    # the estimates are within their known factors of the true values
    _, _, R, _ = oracle.iterative_sketching(p.A, p.b, n, d, 0, seed=p.spec.sketch_seed, history=True)
    assert 0.3 * np.linalg.norm(R, 2) <= ne <= np.linalg.norm(R, 2) * (1 + 1e-12)
    k1 = np.linalg.norm(R, 1) * np.linalg.norm(np.linalg.inv(R), 1)
    assert k1 / 20 <= ce <= k1 * (1 + 1e-6 + 10 * k1 * 2.0 ** -53)   # the reference is exact to ~kappa u


def test_stopping_rule_stops_later_for_ill_conditioned():
    """More conditioning -> larger error floor -> the rule stops no later than for kappa = 1 at the
    same residual; and at kappa = 1e10, ||r|| = 1e-6 it stops well before a fixed 60 steps."""
    p1 = _config1(kappa=1e10, beta=1e-6, seed=9)
    g = oracle.normest_start(50, 7)
    _, it1, _, _ = oracle.iterative_sketching_stop(p1.A, p1.b, 50, 1000, 200, g, seed=p1.spec.sketch_seed)
    assert it1 < 60


def test_normest_start_is_uniform():
    g = oracle.normest_start(20000, 5)
    assert -1.0 <= g.min() and g.max() < 1.0
    assert abs(g.mean()) < 0.02 and abs(g.var() - 1.0 / 3.0) < 0.01


# ---------------------------------------------------------------- mixed precision -----------
# The paper runs in FP64 only; the mixed-precision reading (FP32 sketch, QR and solves, FP64 pass
# and update, with a fallback to FP64) is pinned by exact small cases, LAPACK's single-precision QR,
# power-of-two scaling identities and the convergence of refinement to FP64 accuracy.
U32 = 2.0 ** -24


def test_f32_qr_exact_case_and_sign_convention():
    # orthogonal columns with integer norms: R is exact in float, beta = -sign(alpha) sigma with
    # sign(0) = +1 (second column's pivot is 0 after the first reflection)
    M = np.array([[3, 0], [4, 0], [0, 5]], dtype=np.float32)
    x, R, qtb = oracle.householder_lstsq_f32(M, np.array([1, 2, 3], dtype=np.float32))
    assert R.dtype == np.float32
    assert np.array_equal(R, np.array([[-5, 0], [0, -5]], dtype=np.float32))
    # the least-squares solution is (M^T M)^{-1} M^T rhs = (11, 15) / 25 exactly; float arithmetic
    # puts it within a few u_32 of that, and not within FP64 rounding (it is not a double solve)
    exact = np.array([0.44, 0.6])
    assert np.all(np.abs(x - exact) <= 8 * U32 * exact)
    assert np.abs(x - exact).max() > 1e-12


@pytest.mark.parametrize("kappa", [1e1, 1e3])
def test_f32_qr_backward_error_and_lapack(kappa):
    rng = np.random.default_rng(5)
    rows, n = 400, 24
    U_, _ = np.linalg.qr(rng.standard_normal((rows, n)))
    V_, _ = np.linalg.qr(rng.standard_normal((n, n)))
    M = ((U_ * np.logspace(0, -np.log10(kappa), n)) @ V_.T).astype(np.float32)
    rhs = rng.standard_normal(rows).astype(np.float32)
    _, R, _ = oracle.householder_lstsq_f32(M, rhs)
    M64, R64 = M.astype(np.float64), R.astype(np.float64)
    err = np.linalg.norm(R64.T @ R64 - M64.T @ M64)
    scale = np.linalg.norm(M64) ** 2
    assert err <= 4 * n * U32 * scale            # backward stable at single precision
    assert err >= 1e-3 * U32 * scale              # ... and really computed in single precision
    # LAPACK's single-precision QR agrees up to the signs of R's rows, within kappa u_32
    Rl = np.linalg.qr(M, mode="r").astype(np.float64)
    sg = np.sign(np.diag(R64)) * np.sign(np.diag(Rl))
    assert np.linalg.norm(R64 - sg[:, None] * Rl) <= 50 * kappa * n * U32 * np.linalg.norm(R64)


def test_f32_triangular_solves_integer_exact():
    rng = np.random.default_rng(2)
    n = 12
    R = np.triu(rng.integers(-2, 3, (n, n))).astype(np.float64)
    np.fill_diagonal(R, 1.0)
    y = rng.integers(-3, 4, n).astype(np.float64)
    Rf = [[Fraction(int(v)) for v in row] for row in R]
    # exact solutions by rational substitution; integers small enough to be exact in float
    xr = [Fraction(0)] * n
    for i in range(n - 1, -1, -1):
        xr[i] = Fraction(int(y[i])) - sum(Rf[i][k] * xr[k] for k in range(i + 1, n))
    yr = [Fraction(0)] * n
    for i in range(n):
        yr[i] = Fraction(int(y[i])) - sum(Rf[k][i] * yr[k] for k in range(i))
    assert max(abs(v) for v in xr + yr) < 2 ** 24
    assert np.array_equal(oracle.solve_r_f32(R, y), np.array([float(v) for v in xr], dtype=np.float32))
    assert np.array_equal(oracle.solve_rt_f32(R, y), np.array([float(v) for v in yr], dtype=np.float32))


def test_precond_f32_power_of_two_scaling():
    rng = np.random.default_rng(9)
    n = 40
    R = np.triu(rng.standard_normal((n, n))) / np.sqrt(n)
    np.fill_diagonal(R, 1.0 + rng.random(n))
    R32 = R.astype(np.float32)
    c = rng.standard_normal(n)
    d0 = oracle.precond_f32(R32, c)
    # the right-hand side is rescaled by an exact power of two, so scaling c scales d exactly --
    # also where unscaled float arithmetic would underflow (2^-600) or overflow (2^600)
    for k in [-1000, -600, -100, 0, 50, 600]:
        assert np.array_equal(oracle.precond_f32(R32, np.ldexp(c, k)), np.ldexp(d0, k))
    assert np.array_equal(oracle.precond_f32(R32, np.zeros(n)), np.zeros(n))
    # against the FP64 solves with the same (float) factor: single-precision accuracy
    R64 = R32.astype(np.float64)
    d64 = scipy.linalg.solve_triangular(R64, scipy.linalg.solve_triangular(R64.T, c, lower=True))
    rel = np.linalg.norm(d0 - d64) / np.linalg.norm(d64)
    assert rel <= 20 * n * np.linalg.cond(R64) * U32
    assert rel >= 1e-12                                   # single precision, not double


def test_estimators_f32():
    rng = np.random.default_rng(4)
    n = 30
    U_, _ = np.linalg.qr(rng.standard_normal((n, n)))
    R = np.linalg.qr((U_ * np.logspace(0, -3, n)) @ np.linalg.qr(rng.standard_normal((n, n)))[0].T, mode="r")
    R32 = R.astype(np.float32)
    R64 = R32.astype(np.float64)
    k1 = np.linalg.norm(R64, 1) * np.linalg.norm(np.linalg.inv(R64), 1)
    ce = oracle.condest_1_f32(R32)
    assert k1 / 20 <= ce <= k1 * (1 + 1e-3)
    assert abs(ce - oracle.condest_1(R64)) <= 1e-3 * ce
    g = oracle.normest_start(n, 3)
    steps = int(math.ceil(math.log(n)))
    ne = oracle.normest_f32(R32, g, steps)
    assert abs(ne - oracle.normest(R64, g, steps)) <= 1e-5 * ne
    assert ne <= np.linalg.norm(R64, 2) * (1 + 1e-5)


@pytest.mark.parametrize("kappa", [1e1, 1e3, 1e5])
def test_mixed_refinement_reaches_fp64_accuracy(kappa):
    spec = ProblemSpec(m=4000, n=50, kappa=kappa, beta=1e-6, d=1000, seed=1)
    p = make_problem_cpu(spec)
    x, used, R32, rn = oracle.iterative_sketching_mixed(p.A, p.b, 50, 1000, 60, seed=spec.sketch_seed)
    assert used == oracle.MIXED
    fe_h = np.linalg.norm(oracle.householder_lstsq(p.Aview, p.b)[0] - p.x_true)
    assert np.linalg.norm(x - p.x_true) <= 10 * fe_h     # FP64 accuracy from an FP32 factor
    # the FP32 sketch-and-solve start alone is only single-precision accurate
    x0, _, _ = oracle.householder_lstsq_f32(*oracle.sketch(p.A, p.b, 50, 1000, 8, spec.sketch_seed))
    assert np.linalg.norm(x0 - p.x_true) >= 100 * fe_h
    # ||r_i||^2 is non-increasing up to rounding (the monitor never fired)
    assert np.all(rn[1:] <= rn[:-1] * (1 + 2.0 ** -20))


def test_mixed_falls_back_when_condest_too_large():
    spec = ProblemSpec(m=4000, n=50, kappa=1e12, beta=1e-6, d=1000, seed=1)
    p = make_problem_cpu(spec)
    x, used, R32, _ = oracle.iterative_sketching_mixed(p.A, p.b, 50, 1000, 30, seed=spec.sketch_seed)
    assert used == oracle.FELL_BACK_COND
    assert oracle.condest_1_f32(R32) * U32 > 0.05
    assert np.array_equal(x, oracle.iterative_sketching(p.A, p.b, 50, 1000, 30, seed=spec.sketch_seed))


def test_mixed_growth_monitor_falls_back():
    # d = n leaves S far from an embedding: the iteration diverges (Theorem 3.1 needs distortion
    # below 0.29) although the FP32 factor itself is well conditioned
    spec = ProblemSpec(m=2000, n=20, kappa=1e3, beta=1e-3, d=20, seed=0)
    p = make_problem_cpu(spec)
    x, used, R32, rn = oracle.iterative_sketching_mixed(p.A, p.b, 20, 20, 40, seed=spec.sketch_seed)
    assert used == oracle.FELL_BACK_GROWTH
    assert oracle.condest_1_f32(R32) * U32 <= 0.05
    assert rn[1] > rn[0] and rn[2] > rn[1] and rn[3] > rn[2]
    assert np.array_equal(x, oracle.iterative_sketching(p.A, p.b, 20, 20, 40, seed=spec.sketch_seed))


@pytest.mark.parametrize("kappa,beta", [(1e1, 1e-12), (1e3, 1e-3), (1e5, 1e-12)])
def test_mixed_start_is_fp64_sketch_and_solve(kappa, beta):
    """With q = 0 the mixed solve returns its refined start: the minimizer of ||S b - S A x|| of
    eq. (sketched_ls) to double accuracy (the double Householder solution of the same sketch),
    although its factor is single precision."""
    spec = ProblemSpec(m=8000, n=100, kappa=kappa, beta=beta, d=2000, seed=3)
    p = make_problem_cpu(spec)
    x, used, R32, _ = oracle.iterative_sketching_mixed(p.A, p.b, 100, 2000, 0, seed=spec.sketch_seed)
    assert used == oracle.MIXED
    B, Sb = oracle.sketch(p.A, p.b, 100, 2000, 8, spec.sketch_seed)
    xh, _, _, res = oracle.householder_lstsq(B, Sb)
    kap = np.linalg.cond(B)
    floor = kap * U * (np.linalg.norm(xh) + kap * res / np.linalg.norm(B, 2))
    assert np.linalg.norm(x - xh) <= 100 * floor
    x32, _, _ = oracle.householder_lstsq_f32(B, Sb)
    assert np.linalg.norm(x32 - xh) >= 1e4 * floor        # the unrefined FP32 start is not
    assert 2 <= oracle.mixed_start_steps(oracle.condest_1_f32(R32)) <= 8
