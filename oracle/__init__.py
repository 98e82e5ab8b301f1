"""CPU oracle for iterative sketching (test infrastructure).

A plain C implementation (``ls_oracle.c``, FP64; FP32 only in the mixed-precision functions) of
what the solver computes, loaded through ctypes.
Only the test suite, the smoke check and the CPU-baseline leg of the benchmark may import this
package; the GPU library never does, and the two share no code.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ls_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_D = ctypes.POINTER(ctypes.c_double)
_F = ctypes.POINTER(ctypes.c_float)
_I32 = ctypes.POINTER(ctypes.c_int32)
_I8 = ctypes.POINTER(ctypes.c_int8)
_i64 = ctypes.c_int64
_i32 = ctypes.c_int32
_u64 = ctypes.c_uint64


def build(force: bool = True) -> str:
    """Compile the oracle with gcc: -O3 (independent elementwise loops vectorize; no reduction is
    reordered, so the bits equal a scalar build), no FMA contraction, no -ffast-math; OpenMP only
    spreads the independent row blocks of the TSQR form over host threads."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-ffp-contract=off", "-fno-fast-math", "-std=c11",
                               "-fopenmp", "-fPIC", "-shared", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        L.orc_splitmix64.restype = ctypes.c_uint64
        L.orc_splitmix64.argtypes = [_u64, _u64]
        L.orc_sparse_sign.restype = ctypes.c_int
        L.orc_sparse_sign.argtypes = [_i64, _i64, _i32, _u64, _I32, _I8]
        L.orc_sketch.restype = ctypes.c_int
        L.orc_sketch.argtypes = [_i64, _i64, _D, _i64, _D, _i64, _i32, _u64, _D, _i64, _D]
        L.orc_householder_lstsq.restype = ctypes.c_int
        L.orc_householder_lstsq.argtypes = [_i64, _i64, _D, _i64, _D, _D, _i64, _D, _D, _D]
        L.orc_tsqr_lstsq.restype = ctypes.c_int
        L.orc_tsqr_lstsq.argtypes = [_i64, _i64, _D, _i64, _D, _i64, _i32, _D, _D, _i64, _D]
        L.orc_residual_gradient.restype = None
        L.orc_residual_gradient.argtypes = [_i64, _i64, _D, _i64, _D, _D, _D, _D]
        L.orc_solve_r.restype = None
        L.orc_solve_r.argtypes = [_i64, _D, _i64, _D, _D]
        L.orc_solve_rt.restype = None
        L.orc_solve_rt.argtypes = [_i64, _D, _i64, _D, _D]
        L.orc_iterative_sketching.restype = ctypes.c_int
        L.orc_iterative_sketching.argtypes = [_i64, _i64, _D, _i64, _D, _i64, _i32, _u64, _i32, _D,
                                              _D, _D, _i64, _D]
        L.orc_iterative_sketching_dm.restype = ctypes.c_int
        L.orc_iterative_sketching_dm.argtypes = [_i64, _i64, _D, _i64, _D, _i64, _i32, _u64, _i32,
                                                 ctypes.c_double, ctypes.c_double, _D, _D]
        L.orc_normest.restype = ctypes.c_double
        L.orc_normest.argtypes = [_i64, _D, _i64, _D, _i32]
        L.orc_condest_1.restype = ctypes.c_double
        L.orc_condest_1.argtypes = [_i64, _D, _i64]
        L.orc_iterative_sketching_stop.restype = ctypes.c_int
        L.orc_iterative_sketching_stop.argtypes = [_i64, _i64, _D, _i64, _D, _i64, _i32, _u64, _i32,
                                                   ctypes.c_double, ctypes.c_double, _D, _D,
                                                   ctypes.POINTER(ctypes.c_int32), _D]
        L.orc_sketch_row.restype = None
        L.orc_sketch_row.argtypes = [_i64, _i64, _D, _i64, _I8, _i32, _D]
        L.orc_dimension.restype = ctypes.c_int64
        L.orc_dimension.argtypes = [_i64, _i64, ctypes.c_double]
        L.orc_solve_r_f32.restype = None
        L.orc_solve_r_f32.argtypes = [_i64, _F, _i64, _F, _F]
        L.orc_solve_rt_f32.restype = None
        L.orc_solve_rt_f32.argtypes = [_i64, _F, _i64, _F, _F]
        L.orc_householder_lstsq_f32.restype = ctypes.c_int
        L.orc_householder_lstsq_f32.argtypes = [_i64, _i64, _F, _i64, _F, _F, _i64, _F, _D]
        L.orc_precond_f32.restype = None
        L.orc_precond_f32.argtypes = [_i64, _F, _i64, _D, _D]
        L.orc_normest_f32.restype = ctypes.c_double
        L.orc_normest_f32.argtypes = [_i64, _F, _i64, _D, _i32]
        L.orc_condest_1_f32.restype = ctypes.c_double
        L.orc_condest_1_f32.argtypes = [_i64, _F, _i64]
        L.orc_mixed_start_steps.restype = ctypes.c_int32
        L.orc_mixed_start_steps.argtypes = [ctypes.c_double]
        L.orc_iterative_sketching_mixed.restype = ctypes.c_int
        L.orc_iterative_sketching_mixed.argtypes = [_i64, _i64, _D, _i64, _D, _i64, _i32, _u64, _i32,
                                                    _D, _F, _i64, _D, ctypes.POINTER(ctypes.c_int32)]
        _lib = L
    return _lib


def _dp(a):
    return None if a is None else a.ctypes.data_as(_D)


def _fp(a):
    return None if a is None else a.ctypes.data_as(_F)


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _mat(A):
    """(array, rows, cols, ld) for a 2-D float64 array whose rows may be padded."""
    A = np.asarray(A)
    if A.dtype != np.float64 or A.strides[1] != 8 or A.strides[0] % 8:
        A = _f64(A)
    return A, A.shape[0], A.shape[1], A.strides[0] // 8


def splitmix64(seed: int, k: int) -> int:
    return int(lib().orc_splitmix64(seed, k))


def sparse_sign(m: int, d: int, zeta: int, seed: int):
    """(rows[m, zeta] int32, signs[m, zeta] int8): the sparse-sign embedding's nonzeros."""
    rows = np.zeros((m, zeta), dtype=np.int32)
    signs = np.zeros((m, zeta), dtype=np.int8)
    rc = lib().orc_sparse_sign(m, d, zeta, seed, rows.ctypes.data_as(_I32), signs.ctypes.data_as(_I8))
    if rc:
        raise ValueError(f"orc_sparse_sign: bad arguments (rc={rc})")
    return rows, signs


def sketch(A, b, n: int, d: int, zeta: int, seed: int):
    """B = S A (d x n) and S b (d)."""
    A, m, _, lda = _mat(A)
    b = _f64(b) if b is not None else None
    B = np.zeros((d, n))
    Sb = np.zeros(d)
    rc = lib().orc_sketch(m, n, _dp(A), lda, _dp(b), d, zeta, seed, _dp(B), n, _dp(Sb))
    if rc:
        raise ValueError(f"orc_sketch failed (rc={rc})")
    return B, Sb


def sketch_row(rows, signs, zeta: int):
    """zeta^{-1/2} * sum_t signs[t] rows[t, :], summed in the given order."""
    rows = _f64(rows)
    signs = np.ascontiguousarray(signs, dtype=np.int8)
    cnt, n = rows.shape
    out = np.zeros(n)
    lib().orc_sketch_row(cnt, n, _dp(rows), n, signs.ctypes.data_as(_I8), zeta, _dp(out))
    return out


def householder_lstsq(M, rhs, n: int | None = None):
    """Householder-QR least squares: returns (x, R, Q^T rhs[:n], ||rhs - M x||)."""
    M, rows, cols, ldm = _mat(M)
    n = cols if n is None else n
    rhs = _f64(rhs)
    R = np.zeros((n, n))
    qtb = np.zeros(n)
    x = np.zeros(n)
    res = np.zeros(1)
    rc = lib().orc_householder_lstsq(rows, n, _dp(M), ldm, _dp(rhs), _dp(R), n, _dp(qtb), _dp(x),
                                     _dp(res))
    if rc == 1:
        raise ValueError("orc_householder_lstsq: bad arguments")
    if rc >= 3:
        raise np.linalg.LinAlgError(f"rank deficient at column {rc - 3}")
    if rc:
        raise MemoryError("orc_householder_lstsq")
    return x, R, qtb, float(res[0])


def tsqr_lstsq(A, b, n: int | None = None, block_rows: int = 4096, threads: int | None = None):
    """Householder least squares in TSQR form: (x, R, ||b - A x||).  threads defaults to the CPUs
    this process may use."""
    A, m, cols, lda = _mat(A)
    n = cols if n is None else n
    if threads is None:
        threads = len(os.sched_getaffinity(0))
    x = np.zeros(n)
    R = np.zeros((n, n))
    res = np.zeros(1)
    rc = lib().orc_tsqr_lstsq(m, n, _dp(A), lda, _dp(_f64(b)), block_rows, threads, _dp(x), _dp(R),
                              n, _dp(res))
    if rc == 1:
        raise ValueError("orc_tsqr_lstsq: bad arguments")
    if rc >= 3:
        raise np.linalg.LinAlgError(f"rank deficient (rc={rc})")
    if rc:
        raise MemoryError("orc_tsqr_lstsq")
    return x, R, float(res[0])


def residual_gradient(A, b, x, n: int | None = None):
    """(c, ||r||^2) with r = b - A x and c = A^T r."""
    A, m, cols, lda = _mat(A)
    n = cols if n is None else n
    c = np.zeros(n)
    rr = np.zeros(1)
    lib().orc_residual_gradient(m, n, _dp(A), lda, _dp(_f64(b)), _dp(_f64(x)), _dp(c), _dp(rr))
    return c, float(rr[0])


def solve_r(R, y):
    R = _f64(R)
    n = R.shape[0]
    x = np.zeros(n)
    lib().orc_solve_r(n, _dp(R), R.shape[1], _dp(_f64(y)), _dp(x))
    return x


def solve_rt(R, c):
    R = _f64(R)
    n = R.shape[0]
    y = np.zeros(n)
    lib().orc_solve_rt(n, _dp(R), R.shape[1], _dp(_f64(c)), _dp(y))
    return y


def iterative_sketching(A, b, n: int, d: int, q: int, zeta: int = 8, seed: int = 0,
                        history: bool = False):
    """Algorithm 2.  Returns x_q, or (x_q, x_hist[(q+1), n], R, rnorm2[q]) with history=True."""
    A, m, _, lda = _mat(A)
    b = _f64(b)
    x = np.zeros(n)
    xh = np.zeros((q + 1, n)) if history else None
    R = np.zeros((n, n)) if history else None
    rn = np.zeros(max(q, 1)) if history else None
    rc = lib().orc_iterative_sketching(m, n, _dp(A), lda, _dp(b), d, zeta, seed, q, _dp(x),
                                       _dp(xh), _dp(R), n, _dp(rn))
    if rc == 1:
        raise ValueError("orc_iterative_sketching: bad arguments")
    if rc >= 3:
        raise np.linalg.LinAlgError(f"sketch rank deficient at column {rc - 3}")
    if rc:
        raise MemoryError("orc_iterative_sketching")
    if history:
        return x, xh, R, rn[:q]
    return x


def iterative_sketching_dm(A, b, n: int, d: int, q: int, alpha: float, beta: float, zeta: int = 8,
                           seed: int = 0):
    """Damping / momentum form; returns (x_q, x_hist)."""
    A, m, _, lda = _mat(A)
    x = np.zeros(n)
    xh = np.zeros((q + 1, n))
    rc = lib().orc_iterative_sketching_dm(m, n, _dp(A), lda, _dp(_f64(b)), d, zeta, seed, q,
                                          alpha, beta, _dp(x), _dp(xh))
    if rc:
        raise ValueError(f"orc_iterative_sketching_dm failed (rc={rc})")
    return x, xh


def normest(R, g, steps: int) -> float:
    R = _f64(R)
    return float(lib().orc_normest(R.shape[0], _dp(R), R.shape[1], _dp(_f64(g)), steps))


def condest_1(R) -> float:
    R = _f64(R)
    return float(lib().orc_condest_1(R.shape[0], _dp(R), R.shape[1]))


def dimension(m: int, n: int, u: float = 2.0 ** -53) -> int:
    return int(lib().orc_dimension(m, n, u))


def iterative_sketching_stop(A, b, n: int, d: int, qmax: int, g, zeta: int = 8, seed: int = 0,
                             gamma: float = 1.0, rho: float = 0.04):
    """Algorithm 2 with the Section 3.3 stopping rule: (x, iterations, normest, condest)."""
    A, m, _, lda = _mat(A)
    x = np.zeros(n)
    it = ctypes.c_int32(0)
    est = np.zeros(2)
    rc = lib().orc_iterative_sketching_stop(m, n, _dp(A), lda, _dp(_f64(b)), d, zeta, seed, qmax,
                                            gamma, rho, _dp(_f64(g)), _dp(x), ctypes.byref(it),
                                            _dp(est))
    if rc:
        raise ValueError(f"orc_iterative_sketching_stop failed (rc={rc})")
    return x, it.value, float(est[0]), float(est[1])


def normest_start(n: int, seed: int):
    """Start vector of the randomized power method: g_i uniform on [-1, 1) from SplitMix64 output
    i of the stream seed (53 high bits), the same counter-based source as the embedding."""
    out = np.empty(n)
    for i in range(n):
        z = splitmix64(seed, i)
        out[i] = 2.0 * ((z >> 11) * 2.0 ** -53) - 1.0
    return out


# ---- mixed precision (FP32 sketch, QR and solves; FP64 pass and update) -------------------------
MIXED = 1            # the mixed path ran to the end
FELL_BACK_COND = 2   # condest(R) u_32 > 0.05: redone in FP64
FELL_BACK_GROWTH = 3 # ||r||^2 grew three steps in a row: redone in FP64


def solve_r_f32(R, y):
    R = _f32(R)
    n = R.shape[0]
    x = np.zeros(n, dtype=np.float32)
    lib().orc_solve_r_f32(n, _fp(R), R.shape[1], _fp(_f32(y)), _fp(x))
    return x


def solve_rt_f32(R, c):
    R = _f32(R)
    n = R.shape[0]
    y = np.zeros(n, dtype=np.float32)
    lib().orc_solve_rt_f32(n, _fp(R), R.shape[1], _fp(_f32(c)), _fp(y))
    return y


def householder_lstsq_f32(M, rhs):
    """Single-precision Householder QR of [M | rhs]: (x0 float64, R float32, Q^T rhs[:n] float32)."""
    M = _f32(M)
    rows, n = M.shape
    R = np.zeros((n, n), dtype=np.float32)
    qtb = np.zeros(n, dtype=np.float32)
    x = np.zeros(n)
    rc = lib().orc_householder_lstsq_f32(rows, n, _fp(M), n, _fp(_f32(rhs)), _fp(R), n, _fp(qtb), _dp(x))
    if rc == 1:
        raise ValueError("orc_householder_lstsq_f32: bad arguments")
    if rc >= 3:
        raise np.linalg.LinAlgError(f"rank deficient at column {rc - 3}")
    if rc:
        raise MemoryError("orc_householder_lstsq_f32")
    return x, R, qtb


def precond_f32(R, c):
    """R^{-1} R^{-T} c with FP32 R and FP32 solves on c scaled by a power of two (FP64 in/out)."""
    R = _f32(R)
    n = R.shape[0]
    d = np.zeros(n)
    lib().orc_precond_f32(n, _fp(R), R.shape[1], _dp(_f64(c)), _dp(d))
    return d


def normest_f32(R, g, steps: int) -> float:
    R = _f32(R)
    return float(lib().orc_normest_f32(R.shape[0], _fp(R), R.shape[1], _dp(_f64(g)), steps))


def condest_1_f32(R) -> float:
    R = _f32(R)
    return float(lib().orc_condest_1_f32(R.shape[0], _fp(R), R.shape[1]))


def mixed_start_steps(condest: float) -> int:
    """Refinement steps of the mixed-precision sketch-and-solve start for a given condest(R)."""
    return int(lib().orc_mixed_start_steps(condest))


def iterative_sketching_mixed(A, b, n: int, d: int, q: int, zeta: int = 8, seed: int = 0):
    """Mixed-precision Algorithm 2 with the fallback rule: (x, used, R32, rnorm2 of mixed steps)."""
    A, m, _, lda = _mat(A)
    x = np.zeros(n)
    R = np.zeros((n, n), dtype=np.float32)
    rn = np.zeros(max(q, 1))
    used = ctypes.c_int32(0)
    rc = lib().orc_iterative_sketching_mixed(m, n, _dp(A), lda, _dp(_f64(b)), d, zeta, seed, q,
                                             _dp(x), _fp(R), n, _dp(rn), ctypes.byref(used))
    if rc == 1:
        raise ValueError("orc_iterative_sketching_mixed: bad arguments")
    if rc >= 3:
        raise np.linalg.LinAlgError(f"sketch rank deficient at column {rc - 3}")
    if rc:
        raise MemoryError("orc_iterative_sketching_mixed")
    return x, used.value, R, rn[:q]
