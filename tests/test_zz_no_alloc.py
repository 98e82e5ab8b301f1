"""ls_gradient_noalloc (the allocation-free form of ls_gradient, for callers that cannot allocate
device memory) against ls_gradient through the C ABI: the same kernels on the same inputs, so the
results must be the same bits.  Two calls in a row, the second on a smaller input, check that what
the first left in the shared scratch does not leak into the second."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2311_04362_amd import ls  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = ls.Context(0)
    yield c
    c.close()


def problem(m, n, seed, lda_pad=3):
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    A = torch.randn((m, n + lda_pad), generator=g, dtype=torch.float64, device="cuda")[:, :n]
    x = torch.randn((n,), generator=g, dtype=torch.float64, device="cuda")
    b = A @ x + 1e-3 * torch.randn((m,), generator=g, dtype=torch.float64, device="cuda")
    return A, b, x + 1e-2


@pytest.mark.parametrize("big,small", [((300_001, 2000), (70_001, 500)),     # widest pass, then narrower
                                       ((200_003, 500), (1_000, 33)),        # one partial per CU, then few rows
                                       ((50_000, 64), (3, 1))])
def test_noalloc_gradient_matches_gradient(ctx, big, small):
    for k, (m, n) in enumerate((big, small)):
        A, b, x = problem(m, n, 17 * m + n)
        c_ref, rr_ref = ctx.gradient(A, b, x)
        c = torch.full((n,), np.nan, dtype=torch.float64, device="cuda")
        rr = torch.full((1,), np.nan, dtype=torch.float64, device="cuda")
        ctx.gradient_noalloc(A, b, x, c, rr)
        torch.cuda.synchronize()
        assert torch.equal(c, c_ref), f"call {k}: c differs (m={m}, n={n})"
        assert torch.equal(rr, rr_ref), f"call {k}: ||r||^2 differs (m={m}, n={n})"


def test_noalloc_gradient_fresh_context_and_null_rnorm2():
    # A context that never grew a workspace: the call must not need one.
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c1 = ls.Context(0)
    c2 = ls.Context(0)
    try:
        A, b, x = problem(100_000, 257, 5)
        out = torch.empty(257, dtype=torch.float64, device="cuda")
        c1.gradient_noalloc(A, b, x, out, None)
        ref, _ = c2.gradient(A, b, x)
        torch.cuda.synchronize()
        assert torch.equal(out, ref)
    finally:
        c1.close()
        c2.close()
