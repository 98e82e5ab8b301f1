"""ctypes binding of libls (include/ls.h): argument marshalling only.

Every function takes torch tensors that live on the context's GPU and passes their device
pointers, leading dimensions and the current torch stream to the C ABI; all arithmetic runs in the
HIP kernels.  A missing libls.so is an error, never a fallback.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libls.so")

LS_OK, LS_ERR_ARG, LS_ERR_ALLOC, LS_ERR_DEVICE, LS_ERR_RANK, LS_ERR_NONFINITE, \
    LS_ERR_DIVERGED, LS_ERR_UNSUPPORTED, LS_ERR_TIMEOUT = range(9)
STATUS_NAMES = ["LS_OK", "LS_ERR_ARG", "LS_ERR_ALLOC", "LS_ERR_DEVICE", "LS_ERR_RANK",
                "LS_ERR_NONFINITE", "LS_ERR_DIVERGED", "LS_ERR_UNSUPPORTED", "LS_ERR_TIMEOUT"]
OPT_ZETA, OPT_SEED, OPT_UPDATE, OPT_ALPHA, OPT_BETA, OPT_PRECISION, OPT_PROFILE, OPT_QR_PANEL, \
    OPT_STOP, OPT_GAMMA, OPT_RHO, OPT_GATHER = 1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12
NORMEST_SEED_OFFSET = 0x632BE59BD9B4E019
PRECISION_FP64, PRECISION_MIXED, PRECISION_FELL_BACK_COND, PRECISION_FELL_BACK_GROWTH = 0, 1, 2, 3

EXPORTS = ["ls_create", "ls_destroy", "ls_last_error", "ls_limits", "ls_set_option",
           "ls_get_option", "ls_sketch_embedding", "ls_sketch_csr", "ls_sketch", "ls_qr_sketch",
           "ls_gradient", "ls_precond_solve", "ls_iterate", "ls_solve", "ls_sync", "ls_profile",
           "ls_solve_info", "ls_sketch_f32", "ls_qr_sketch_f32", "ls_precond_solve_f32",
           "ls_server_create", "ls_server_destroy", "ls_server_submit", "ls_server_wait",
           "ls_server_request_info", "ls_server_stats", "ls_server_last_error",
           "ls_gradient_noalloc", "ls_server_footprint", "ls_server_set_precision",
           "ls_server_request_precision"]

_lib = None
_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_i32 = ctypes.c_int32
_u64 = ctypes.c_uint64
_f64 = ctypes.c_double


class LSError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        self.status = status
        name = STATUS_NAMES[status] if 0 <= status < len(STATUS_NAMES) else str(status)
        super().__init__(f"{where}: {name}: {detail}")


def load():
    """Load libls.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libls.so not built at {LIB_PATH}; run __graft_entry__.build()")
    L = ctypes.CDLL(LIB_PATH)
    sig = {
        "ls_create": ([ctypes.c_int, ctypes.POINTER(_vp)], ctypes.c_int),
        "ls_destroy": ([_vp], None),
        "ls_last_error": ([_vp], ctypes.c_char_p),
        "ls_limits": ([ctypes.POINTER(_i32), ctypes.POINTER(_i32)], ctypes.c_int),
        "ls_set_option": ([_vp, ctypes.c_int, _i64, _f64], ctypes.c_int),
        "ls_get_option": ([_vp, ctypes.c_int, ctypes.POINTER(_i64), ctypes.POINTER(_f64)], ctypes.c_int),
        "ls_sketch_embedding": ([_vp, _vp, _i64, _i64, _i32, _u64, _vp, _vp], ctypes.c_int),
        "ls_sketch_csr": ([_vp, _vp, _i64, _i64, _i32, _u64, _vp, _vp], ctypes.c_int),
        "ls_sketch": ([_vp, _vp, _i64, _i64, _vp, _i64, _vp, _i64, _i32, _u64, _vp, _i64, _vp], ctypes.c_int),
        "ls_qr_sketch": ([_vp, _vp, _i64, _i64, _vp, _i64, _vp, _vp, _i64, _vp], ctypes.c_int),
        "ls_gradient": ([_vp, _vp, _i64, _i64, _vp, _i64, _vp, _vp, _vp, _vp], ctypes.c_int),
        "ls_gradient_noalloc": ([_vp, _vp, _i64, _i64, _vp, _i64, _vp, _vp, _vp, _vp], ctypes.c_int),
        "ls_precond_solve": ([_vp, _vp, _i64, _vp, _i64, _vp, _vp], ctypes.c_int),
        "ls_iterate": ([_vp, _vp, _i64, _i64, _vp, _i64, _vp, _vp, _i64, _vp, _i32, _vp], ctypes.c_int),
        "ls_solve": ([_vp, _vp, _i64, _i64, _vp, _i64, _vp, _i64, _i32, _vp], ctypes.c_int),
        "ls_sync": ([_vp, _vp], ctypes.c_int),
        "ls_profile": ([_vp, ctypes.POINTER(_f64), ctypes.POINTER(_i64), _i32], ctypes.c_int),
        "ls_solve_info": ([_vp, ctypes.POINTER(_i64), ctypes.POINTER(_i32), ctypes.POINTER(_f64),
                           ctypes.POINTER(_f64), ctypes.POINTER(_i32)], ctypes.c_int),
        "ls_sketch_f32": ([_vp, _vp, _i64, _i64, _vp, _i64, _vp, _i64, _i32, _u64, _vp, _i64, _vp], ctypes.c_int),
        "ls_qr_sketch_f32": ([_vp, _vp, _i64, _i64, _vp, _i64, _vp, _vp, _i64, _vp], ctypes.c_int),
        "ls_precond_solve_f32": ([_vp, _vp, _i64, _vp, _i64, _vp, _vp], ctypes.c_int),
        "ls_server_create": ([ctypes.c_int, _i64, _i32, ctypes.POINTER(_vp)], ctypes.c_int),
        "ls_server_destroy": ([_vp], None),
        "ls_server_submit": ([_vp, _i64, _i64, _vp, _i64, _vp, _i64, _i32, _u64, _vp,
                              ctypes.POINTER(_i64)], ctypes.c_int),
        "ls_server_wait": ([_vp, _i64, _f64, ctypes.POINTER(ctypes.c_int)], ctypes.c_int),
        "ls_server_request_info": ([_vp, _i64, ctypes.POINTER(_f64)], ctypes.c_int),
        "ls_server_stats": ([_vp, ctypes.POINTER(_i64)], ctypes.c_int),
        "ls_server_last_error": ([_vp], ctypes.c_char_p),
        "ls_server_footprint": ([_vp, _i64, _i64, _i64, ctypes.POINTER(_i64), ctypes.POINTER(_i64)], ctypes.c_int),
        "ls_server_set_precision": ([_vp, _i32], ctypes.c_int),
        "ls_server_request_precision": ([_vp, _i64, ctypes.POINTER(_i32)], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _lib = L
    return L


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _mat(t: torch.Tensor, name: str, dtype=torch.float64):
    if t.dim() != 2 or t.dtype != dtype or t.stride(1) != 1 or not t.is_cuda:
        raise ValueError(f"{name}: need a 2-D {dtype} CUDA tensor with unit column stride")
    return t.shape[0], t.shape[1], t.stride(0)


def _vec(t: torch.Tensor, name: str, dtype=torch.float64):
    if t.dtype != dtype or not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{name}: need a contiguous {dtype} CUDA tensor")
    return t


class Context:
    """One libls context bound to a GPU (device >= 0) or host-only (device = -1)."""

    def __init__(self, device: int = 0):
        self._L = load()
        h = _vp()
        st = self._L.ls_create(device, ctypes.byref(h))
        if st != LS_OK:
            raise LSError(st, "ls_create", f"device {device}")
        self.h = h
        self.device = device

    def close(self):
        if getattr(self, "h", None):
            self._L.ls_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st: int, where: str):
        if st != LS_OK:
            raise LSError(st, where, self._L.ls_last_error(self.h).decode())

    def _stream(self):
        return _vp(torch.cuda.current_stream().cuda_stream) if self.device >= 0 else _vp(0)

    # options
    def set_option(self, key: int, ival: int = 0, dval: float = 0.0):
        self._check(self._L.ls_set_option(self.h, key, ival, dval), "ls_set_option")

    def get_option(self, key: int):
        iv, dv = _i64(), _f64()
        self._check(self._L.ls_get_option(self.h, key, ctypes.byref(iv), ctypes.byref(dv)), "ls_get_option")
        return iv.value, dv.value

    # (a1) the embedding's nonzeros
    def sketch_embedding(self, m: int, d: int, zeta: int, seed: int):
        rows = torch.empty((m, zeta), dtype=torch.int32, device="cuda")
        signs = torch.empty((m, zeta), dtype=torch.int8, device="cuda")
        self._check(self._L.ls_sketch_embedding(self.h, self._stream(), m, d, zeta, seed,
                                                _ptr(rows), _ptr(signs)), "ls_sketch_embedding")
        return rows, signs

    # (a2) compressed rows of S
    def sketch_csr(self, m: int, d: int, zeta: int, seed: int):
        rowptr = torch.empty(d + 1, dtype=torch.int32, device="cuda")
        cols = torch.empty(m * zeta, dtype=torch.int32, device="cuda")
        self._check(self._L.ls_sketch_csr(self.h, self._stream(), m, d, zeta, seed, _ptr(rowptr),
                                          _ptr(cols)), "ls_sketch_csr")
        return rowptr, cols

    # (a3) B = S A, S b
    def sketch(self, A: torch.Tensor, b, d: int, zeta: int, seed: int, B=None, Sb=None):
        m, n, lda = _mat(A, "A")
        if B is None:
            B = torch.empty((d, n), dtype=torch.float64, device=A.device)
        _, _, ldb = _mat(B, "B")
        if b is not None and Sb is None:
            Sb = torch.empty(d, dtype=torch.float64, device=A.device)
        self._check(self._L.ls_sketch(self.h, self._stream(), m, n, _ptr(A), lda,
                                      _ptr(None if b is None else _vec(b, "b")), d, zeta, seed,
                                      _ptr(B), ldb, _ptr(Sb)), "ls_sketch")
        return B, Sb

    # (a4, a5) QR of [B | Sb], R and x0
    def qr_sketch(self, B: torch.Tensor, Sb: torch.Tensor, want_x0: bool = True):
        d, n, ldb = _mat(B, "B")
        R = torch.empty((n, n), dtype=torch.float64, device=B.device)
        x0 = torch.empty(n, dtype=torch.float64, device=B.device) if want_x0 else None
        self._check(self._L.ls_qr_sketch(self.h, self._stream(), d, n, _ptr(B), ldb,
                                         _ptr(_vec(Sb, "Sb")), _ptr(R), n, _ptr(x0)), "ls_qr_sketch")
        return R, x0

    # (a6, a7) c = A^T (b - A x), ||r||^2
    def gradient(self, A: torch.Tensor, b: torch.Tensor, x: torch.Tensor):
        m, n, lda = _mat(A, "A")
        c = torch.empty(n, dtype=torch.float64, device=A.device)
        rr = torch.empty(1, dtype=torch.float64, device=A.device)
        self._check(self._L.ls_gradient(self.h, self._stream(), m, n, _ptr(A), lda, _ptr(_vec(b, "b")),
                                        _ptr(_vec(x, "x")), _ptr(c), _ptr(rr)), "ls_gradient")
        return c, rr

    def gradient_noalloc(self, A: torch.Tensor, b: torch.Tensor, x: torch.Tensor, c: torch.Tensor,
                         rr: torch.Tensor | None = None):
        """ls_gradient_noalloc: the same c and ||r||^2 into caller-given buffers, with the library's
        fixed per-GPU scratch in place of its workspace."""
        m, n, lda = _mat(A, "A")
        if c.numel() != n:
            raise ValueError("c: need n entries")
        self._check(self._L.ls_gradient_noalloc(self.h, self._stream(), m, n, _ptr(A), lda,
                                                _ptr(_vec(b, "b")), _ptr(_vec(x, "x")),
                                                _ptr(_vec(c, "c")),
                                                _ptr(None if rr is None else _vec(rr, "rr"))),
                    "ls_gradient_noalloc")
        return c, rr

    # (a8) d = R^{-1} R^{-T} c
    def precond_solve(self, R: torch.Tensor, c: torch.Tensor):
        n, _, ldr = _mat(R, "R")
        d = torch.empty(n, dtype=torch.float64, device=R.device)
        self._check(self._L.ls_precond_solve(self.h, self._stream(), n, _ptr(R), ldr,
                                             _ptr(_vec(c, "c")), _ptr(d)), "ls_precond_solve")
        return d

    # (a6..a9) x <- x + R^{-1} R^{-T} A^T (b - A x), q times, in place
    def iterate(self, A: torch.Tensor, b: torch.Tensor, R: torch.Tensor, x: torch.Tensor, q: int,
                rnorm2: torch.Tensor | None = None):
        m, n, lda = _mat(A, "A")
        _, _, ldr = _mat(R, "R")
        self._check(self._L.ls_iterate(self.h, self._stream(), m, n, _ptr(A), lda, _ptr(_vec(b, "b")),
                                       _ptr(R), ldr, _ptr(_vec(x, "x")), q,
                                       _ptr(None if rnorm2 is None else _vec(rnorm2, "rnorm2"))),
                    "ls_iterate")
        return x

    # whole solve (Algorithm 2)
    def solve(self, A: torch.Tensor, b: torch.Tensor, d: int, q: int, x: torch.Tensor | None = None):
        m, n, lda = _mat(A, "A")
        if x is None:
            x = torch.empty(n, dtype=torch.float64, device=A.device)
        self._check(self._L.ls_solve(self.h, self._stream(), m, n, _ptr(A), lda, _ptr(_vec(b, "b")),
                                     d, q, _ptr(_vec(x, "x"))), "ls_solve")
        return x

    def sync(self):
        self._check(self._L.ls_sync(self.h, self._stream()), "ls_sync")

    def solve_info(self):
        """(d used, refinement steps made, normest, condest, precision used) of the last solve."""
        d, q, ne, ce, pr = _i64(), _i32(), _f64(), _f64(), _i32()
        self._check(self._L.ls_solve_info(self.h, ctypes.byref(d), ctypes.byref(q), ctypes.byref(ne),
                                          ctypes.byref(ce), ctypes.byref(pr)), "ls_solve_info")
        return d.value, q.value, ne.value, ce.value, pr.value

    # mixed-precision pieces (FP32 sketch, QR and R-solves)
    def sketch_f32(self, A: torch.Tensor, b, d: int, zeta: int, seed: int):
        m, n, lda = _mat(A, "A")
        B = torch.empty((d, n), dtype=torch.float32, device=A.device)
        Sb = torch.empty(d, dtype=torch.float32, device=A.device) if b is not None else None
        self._check(self._L.ls_sketch_f32(self.h, self._stream(), m, n, _ptr(A), lda,
                                          _ptr(None if b is None else _vec(b, "b")), d, zeta, seed,
                                          _ptr(B), n, _ptr(Sb)), "ls_sketch_f32")
        return B, Sb

    def qr_sketch_f32(self, B: torch.Tensor, Sb: torch.Tensor, want_x0: bool = True):
        d, n, ldb = _mat(B, "B", torch.float32)
        R = torch.empty((n, n), dtype=torch.float32, device=B.device)
        x0 = torch.empty(n, dtype=torch.float64, device=B.device) if want_x0 else None
        self._check(self._L.ls_qr_sketch_f32(self.h, self._stream(), d, n, _ptr(B), ldb,
                                             _ptr(_vec(Sb, "Sb", torch.float32)), _ptr(R), n, _ptr(x0)),
                    "ls_qr_sketch_f32")
        return R, x0

    def precond_solve_f32(self, R: torch.Tensor, c: torch.Tensor):
        n, _, ldr = _mat(R, "R", torch.float32)
        d = torch.empty(n, dtype=torch.float64, device=R.device)
        self._check(self._L.ls_precond_solve_f32(self.h, self._stream(), n, _ptr(R), ldr,
                                                 _ptr(_vec(c, "c")), _ptr(d)), "ls_precond_solve_f32")
        return d

    def profile(self, reset: bool = True):
        """(summed fused-pass kernel ms, launches) since the last reset (needs OPT_PROFILE = 1)."""
        ms, cnt = _f64(), _i64()
        self._check(self._L.ls_profile(self.h, ctypes.byref(ms), ctypes.byref(cnt), int(reset)), "ls_profile")
        return ms.value, cnt.value


class Server:
    """A served stream of solves on one GPU (ls_server_*), FP64 or mixed precision (set_precision).
    submit() returns a ticket at once; the tensors stay referenced here until wait() has seen the
    request finish."""

    def __init__(self, device: int = 0, budget_bytes: int = 64 << 30, max_active: int = 1024):
        self._L = load()
        h = _vp()
        st = self._L.ls_server_create(device, budget_bytes, max_active, ctypes.byref(h))
        if st != LS_OK:
            raise LSError(st, "ls_server_create", f"device {device}")
        self.h = h
        self.device = device
        self._keep = {}

    def close(self):
        if getattr(self, "h", None):
            self._L.ls_server_destroy(self.h)
            self.h = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st: int, where: str):
        if st != LS_OK:
            raise LSError(st, where, self._L.ls_server_last_error(self.h).decode())

    def submit(self, A: torch.Tensor, b: torch.Tensor, d: int, q: int, seed: int,
               x: torch.Tensor | None = None):
        m, n, lda = _mat(A, "A")
        if x is None:
            x = torch.empty(n, dtype=torch.float64, device=A.device)
        # the server's streams run apart from torch's: the inputs must be complete on the device
        torch.cuda.current_stream().synchronize()
        t = _i64()
        self._check(self._L.ls_server_submit(self.h, m, n, _ptr(A), lda, _ptr(_vec(b, "b")), d, q,
                                             seed, _ptr(_vec(x, "x")), ctypes.byref(t)),
                    "ls_server_submit")
        self._keep[t.value] = (A, b, x)
        return t.value, x

    def wait(self, ticket: int, timeout: float = -1.0) -> int:
        """Waits for the request; returns its status (LS_OK or that problem's deferred error)."""
        res = ctypes.c_int(0)
        self._check(self._L.ls_server_wait(self.h, ticket, timeout, ctypes.byref(res)), "ls_server_wait")
        self._keep.pop(ticket, None)
        return res.value

    def set_precision(self, precision: int):
        """Arithmetic of later submissions: PRECISION_FP64 or PRECISION_MIXED."""
        self._check(self._L.ls_server_set_precision(self.h, precision), "ls_server_set_precision")

    def precision(self, ticket: int) -> int:
        """The precision the request's result comes from (PRECISION_*)."""
        u = _i32()
        self._check(self._L.ls_server_request_precision(self.h, ticket, ctypes.byref(u)),
                    "ls_server_request_precision")
        return u.value

    def times(self, ticket: int):
        """(submitted, admitted, first round, finished), seconds since the server was created."""
        t = (_f64 * 4)()
        self._check(self._L.ls_server_request_info(self.h, ticket, t), "ls_server_request_info")
        return tuple(t)

    def stats(self):
        s = (_i64 * 8)()
        self._check(self._L.ls_server_stats(self.h, s), "ls_server_stats")
        keys = ["submitted", "finished", "queued", "admitted", "footprint", "footprint_peak", "rounds",
                "setup_workspace"]
        return dict(zip(keys, list(s)))

    def footprint(self, m: int, n: int, d: int):
        """(resident bytes, setup-lane workspace bytes) admission charges for a problem of this shape."""
        res, su = _i64(), _i64()
        self._check(self._L.ls_server_footprint(self.h, m, n, d, ctypes.byref(res), ctypes.byref(su)),
                    "ls_server_footprint")
        return res.value, su.value


def limits():
    L = load()
    z, n = _i32(), _i32()
    L.ls_limits(ctypes.byref(z), ctypes.byref(n))
    return z.value, n.value
