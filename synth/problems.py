"""Seeded synthetic least-squares problems with a known solution.

The recipe follows the experimental setup of the paper (Section 1.1.1, "Experimental setup"):

* ``A = U1 diag(sigma) V^T`` with ``U1`` (m x n) having orthonormal columns, ``V`` (n x n) orthogonal,
  and ``sigma`` logarithmically equispaced from 1 down to ``1/kappa``;
* the solution ``x = w/||w||`` with ``w`` standard Gaussian;
* the residual ``r = beta * P z / ||P z||`` with ``z`` standard Gaussian and ``P`` the orthogonal
  projector onto the complement of range(A);
* ``b = A x + r``, so ``x`` is the least-squares solution and ``||r(x)|| = beta``.

The paper draws a full Haar ``U = [U1 U2]`` (m x m) and sets ``r = beta U2 z / ||U2 z||``.  That is
infeasible at m in the millions, so ``r`` is drawn as ``P z`` with ``P z = z - U1 (U1^T z)`` applied
twice (one projection leaves O(u) components in range(A); the second removes them).  ``P z/||P z||``
is uniformly distributed on the unit sphere of range(A)'s complement, exactly like ``U2 z/||U2 z||``.

This module holds no part of the solver: it only builds inputs.  Both the CPU oracle and the GPU
library consume its arrays.

Seeds: a problem seed ``s`` gives sub-seeds ``16 s + {0,1,2,3}`` for the streams G (for U1), V, w
and z; the sketch seed is ``16 s + 4``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Any

import numpy as np

__all__ = ["ProblemSpec", "Problem", "make_problem_cpu", "make_problem_gpu", "integer_problem",
           "sub_seeds", "CONFIGS", "padded_ld"]


def padded_ld(n: int, mult: int = 8) -> int:
    """Row stride rounded up to a multiple of ``mult`` doubles (64-byte rows)."""
    return ((n + mult - 1) // mult) * mult


def sub_seeds(seed: int) -> dict:
    return {"G": 16 * seed + 0, "V": 16 * seed + 1, "w": 16 * seed + 2, "z": 16 * seed + 3,
            "S": 16 * seed + 4}


@dataclass
class ProblemSpec:
    m: int
    n: int
    kappa: float = 1e10
    beta: float = 1e-6
    seed: int = 0
    d: int | None = None
    zeta: int = 8
    q: int = 40
    lda: int | None = None

    def __post_init__(self):
        if self.d is None:
            self.d = 20 * self.n
        if self.lda is None:
            self.lda = padded_ld(self.n)

    @property
    def sketch_seed(self) -> int:
        return sub_seeds(self.seed)["S"]


@dataclass
class Problem:
    spec: ProblemSpec
    A: Any          # m x lda storage, row-major; columns n..lda-1 are zero padding
    b: Any          # m
    x_true: Any     # n
    sigma: Any = field(default=None)   # singular values of A

    @property
    def Aview(self):
        return self.A[:, : self.spec.n]


def _sigma(n: int, kappa: float) -> np.ndarray:
    if n == 1:
        return np.ones(1)
    j = np.arange(n, dtype=np.float64)
    return kappa ** (-j / (n - 1))


def make_problem_cpu(spec: ProblemSpec) -> Problem:
    """NumPy generator for sizes that fit comfortably in host memory."""
    m, n = spec.m, spec.n
    s = sub_seeds(spec.seed)
    G = np.random.default_rng(s["G"]).standard_normal((m, n))
    U1, _ = np.linalg.qr(G)                       # orthonormal columns (LAPACK Householder)
    V, _ = np.linalg.qr(np.random.default_rng(s["V"]).standard_normal((n, n)))
    sig = _sigma(n, spec.kappa)
    A = (U1 * sig) @ V.T
    w = np.random.default_rng(s["w"]).standard_normal(n)
    x = w / np.linalg.norm(w)
    z = np.random.default_rng(s["z"]).standard_normal(m)
    for _ in range(2):
        z = z - U1 @ (U1.T @ z)
    r = spec.beta * z / np.linalg.norm(z) if spec.beta > 0 else np.zeros(m)
    b = A @ x + r
    As = np.zeros((m, spec.lda))
    As[:, :n] = A
    return Problem(spec, As, b, x, sig)


def make_problem_gpu(spec: ProblemSpec, device="cuda", chunk_rows: int = 1 << 19) -> Problem:
    """torch generator on the GPU for the large shapes (A of many GB).

    U1 comes from CholeskyQR2 of a Gaussian matrix.  That is safe here because an m x n Gaussian
    with m >> n has condition number close to 1; it is used for building inputs only.  Work is done
    in row chunks so that at most one m x n matrix plus the padded A are alive at once.
    """
    import torch

    m, n, lda = spec.m, spec.n, spec.lda
    s = sub_seeds(spec.seed)
    dt = torch.float64

    def gen(seed):
        g = torch.Generator(device=device)
        g.manual_seed(seed)
        return g

    # A's storage doubles as the Gaussian / U1 buffer (first n columns), then is overwritten by A.
    A = torch.zeros((m, lda), dtype=dt, device=device)
    U = A[:, :n]
    gG = gen(s["G"])
    for r0 in range(0, m, chunk_rows):
        r1 = min(m, r0 + chunk_rows)
        U[r0:r1] = torch.randn((r1 - r0, n), generator=gG, dtype=dt, device=device)
    for _ in range(2):                            # CholeskyQR2
        gram = torch.zeros((n, n), dtype=dt, device=device)
        for r0 in range(0, m, chunk_rows):
            blk = U[r0:min(m, r0 + chunk_rows)]
            gram += blk.T @ blk
        L = torch.linalg.cholesky(gram)
        Linv_T = torch.linalg.solve_triangular(L, torch.eye(n, dtype=dt, device=device),
                                               upper=False).T.contiguous()
        for r0 in range(0, m, chunk_rows):
            r1 = min(m, r0 + chunk_rows)
            U[r0:r1] = U[r0:r1] @ Linv_T
    gV = gen(s["V"])
    V, _ = torch.linalg.qr(torch.randn((n, n), generator=gV, dtype=dt, device=device))
    sig = torch.tensor(_sigma(n, spec.kappa), dtype=dt, device=device)
    w = torch.randn((n,), generator=gen(s["w"]), dtype=dt, device=device)
    x = w / torch.linalg.norm(w)
    z = torch.randn((m,), generator=gen(s["z"]), dtype=dt, device=device)
    for _ in range(2):
        z = z - U @ (U.T @ z)
    r = spec.beta * z / torch.linalg.norm(z) if spec.beta > 0 else torch.zeros_like(z)
    del z
    SVt = (sig[:, None] * V.T).contiguous()       # diag(sigma) V^T
    b = torch.empty((m,), dtype=dt, device=device)
    for r0 in range(0, m, chunk_rows):
        r1 = min(m, r0 + chunk_rows)
        blk = U[r0:r1] @ SVt
        U[r0:r1] = blk
        b[r0:r1] = blk @ x + r[r0:r1]
    del r
    torch.cuda.synchronize()
    return Problem(spec, A, b, x, sig.cpu().numpy())


def integer_problem(m: int, n: int, lo: int = -3, hi: int = 3, seed: int = 0, lda: int | None = None):
    """Small-integer A, b, x: every sum the solver forms on them is exact in FP64."""
    rng = np.random.default_rng(seed)
    lda = padded_ld(n) if lda is None else lda
    A = np.zeros((m, lda))
    A[:, :n] = rng.integers(lo, hi + 1, size=(m, n))
    b = rng.integers(lo, hi + 1, size=m).astype(np.float64)
    x = rng.integers(lo, hi + 1, size=n).astype(np.float64)
    return A, b, x


# The five workloads (shapes, distributions, iteration counts).
CONFIGS = {
    1: dict(m=4000, n=50, d=1000, kappa=1e10, beta=1e-6, q=30),
    2: dict(m=2_000_000, n=500, d=10_000, kappa=1e10, beta=1e-6, q=40),
    3: dict(m=1_000_000, n=1000, d=20_000, kappa=(1e2, 1e6, 1e12), beta=(1e-12, 1e-3, 1.0), q=40),
    4: dict(count=512, rate=200.0, m=(20_000, 200_000), n=(32, 64, 128, 256),
            kappa=(1e2, 1e12), beta=1e-6, q=40),
    5: dict(m=4_000_000, n=2000, d=40_000, kappa=1e10, beta=1e-6, q=40),
}


def wedin_floor(kappa: float, beta: float, normA: float = 1.0, normx: float = 1.0) -> float:
    """Relative forward error a backward-stable solver attains (eq. ls_forward, constant 1)."""
    u = 2.0 ** -53
    return kappa * u * (normx + kappa * beta / normA) / normx


def served_stream(count=512, rate=200.0, seed=2311):
    """Arrival times and shapes of the served-stream workload (Poisson arrivals)."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=count)
    t = np.cumsum(gaps) - gaps[0]
    ms = np.floor(np.exp(rng.uniform(math.log(2e4), math.log(2e5), size=count))).astype(np.int64)
    ns = rng.choice(np.array([32, 64, 128, 256]), size=count)
    kap = np.exp(rng.uniform(math.log(1e2), math.log(1e12), size=count))
    return t, ms, ns, kap
