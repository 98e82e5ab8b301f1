"""GPU parity for the Section 3.3 implementation guidance: the stopping rule with its normest and
condest estimates, the divergence guard, and the embedding dimension of eq. (dimension)."""
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


@pytest.mark.parametrize("kappa,beta", [(1e1, 1e-12), (1e10, 1e-6), (1e10, 1e-3), (1e15, 1e-12), (1.0, 1e-6)])
def test_stopping_rule_matches_oracle(ctx, kappa, beta):
    spec = ProblemSpec(m=4000, n=50, kappa=kappa, beta=beta, d=1000, seed=8)
    p = make_problem_cpu(spec)
    n, d = spec.n, spec.d
    seed = spec.sketch_seed
    g = oracle.normest_start(n, (seed + ls.NORMEST_SEED_OFFSET) % (1 << 64))
    xo, it_o, ne_o, ce_o = oracle.iterative_sketching_stop(p.A, p.b, n, d, 200, g, seed=seed)
    ctx.set_option(ls.OPT_SEED, seed)
    ctx.set_option(ls.OPT_STOP, 1)
    try:
        x = ctx.solve(dev(p.A)[:, :n], dev(p.b), d, 200).cpu().numpy()
        d_used, steps, ne, ce, prec = ctx.solve_info()
    finally:
        ctx.set_option(ls.OPT_STOP, 0)
    assert d_used == d and prec == ls.PRECISION_FP64
    # normest: same start vector, same number of power steps; R agrees to rounding
    assert abs(ne - ne_o) <= 1e-8 * ne_o
    # condest: Hager's estimate; both are lower bounds of kappa_1(R) within its usual factor
    _, _, R, _ = oracle.iterative_sketching(p.A, p.b, n, d, 0, seed=seed, history=True)
    k1 = np.linalg.norm(R, 1) * np.linalg.norm(np.linalg.inv(R), 1)
    assert k1 / 20 <= ce <= k1 * (1 + 1e-6 + 10 * k1 * 2.0 ** -53)   # the reference is exact to ~kappa u
    assert ce_o / 3 <= ce <= 3 * ce_o
    # the stopping decision: same step within two, and Householder-level accuracy
    assert abs(steps - it_o) <= 2
    fe_h = np.linalg.norm(oracle.householder_lstsq(p.Aview, p.b)[0] - p.x_true)
    assert np.linalg.norm(x - p.x_true) <= 10 * max(fe_h, 1e-15) + 1e-15


@pytest.mark.parametrize("n", [1, 7, 63, 64, 65, 130, 333])
def test_estimators_match_oracle_across_sizes(ctx, n):
    """normest and condest at widths below one wave, at one and just past one block of 64 outputs,
    and with a ragged last block (the power-method products deal 64-output blocks to the waves)."""
    spec = ProblemSpec(m=4000, n=n, kappa=1e3, beta=1e-6, d=max(1000, 4 * n), seed=11)
    p = make_problem_cpu(spec)
    seed = spec.sketch_seed
    g = oracle.normest_start(n, (seed + ls.NORMEST_SEED_OFFSET) % (1 << 64))
    _, _, ne_o, ce_o = oracle.iterative_sketching_stop(p.A, p.b, n, spec.d, 2, g, seed=seed)
    ctx.set_option(ls.OPT_SEED, seed)
    ctx.set_option(ls.OPT_STOP, 1)
    try:
        ctx.solve(dev(p.A)[:, :n], dev(p.b), spec.d, 2)
        _, _, ne, ce, _ = ctx.solve_info()
    finally:
        ctx.set_option(ls.OPT_STOP, 0)
    assert abs(ne - ne_o) <= 1e-8 * ne_o
    assert ce_o / 3 <= ce <= 3 * ce_o


def test_stopping_rule_fewer_steps_and_q_cap(ctx):
    spec = ProblemSpec(m=4000, n=50, kappa=1e10, beta=1e-6, d=1000, seed=9)
    p = make_problem_cpu(spec)
    ctx.set_option(ls.OPT_SEED, spec.sketch_seed)
    ctx.set_option(ls.OPT_STOP, 1)
    try:
        ctx.solve(dev(p.A)[:, :50], dev(p.b), 1000, 200)
        _, steps, _, _, _ = ctx.solve_info()
        ctx.solve(dev(p.A)[:, :50], dev(p.b), 1000, 5)        # the cap wins
        _, steps5, _, _, _ = ctx.solve_info()
    finally:
        ctx.set_option(ls.OPT_STOP, 0)
    assert 10 < steps < 200
    assert steps5 == 5


def test_divergence_is_flagged(ctx):
    """d = n leaves the embedding far from an isometry: the iteration diverges (Theorem 3.1 needs
    distortion below 0.29), and the residual guard must end it with LS_ERR_DIVERGED."""
    spec = ProblemSpec(m=2000, n=20, kappa=1e3, beta=1e-3, d=20, seed=0)
    p = make_problem_cpu(spec)
    ctx.set_option(ls.OPT_SEED, spec.sketch_seed)
    ctx.set_option(ls.OPT_STOP, 1)
    try:
        with pytest.raises(ls.LSError) as e:
            ctx.solve(dev(p.A)[:, :20], dev(p.b), 20, 100)
        assert e.value.status == ls.LS_ERR_DIVERGED
        _, steps, _, _, _ = ctx.solve_info()
        assert steps < 100
    finally:
        ctx.set_option(ls.OPT_STOP, 0)
    ctx.sync()


@pytest.mark.parametrize("m,n", [(4000, 50), (20000, 100), (3000, 60)])
def test_dimension_rule(ctx, m, n):
    p = make_problem_cpu(ProblemSpec(m=m, n=n, kappa=1e2, beta=1e-6, seed=1))
    ctx.set_option(ls.OPT_SEED, p.spec.sketch_seed)
    x0 = ctx.solve(dev(p.A)[:, :n], dev(p.b), 0, 20)
    d_used, steps, _, _, _ = ctx.solve_info()
    assert d_used == oracle.dimension(m, n)
    assert steps == 20
    x1 = ctx.solve(dev(p.A)[:, :n], dev(p.b), d_used, 20)
    assert torch.equal(x0, x1)
