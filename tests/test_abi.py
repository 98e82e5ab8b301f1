"""Host-side checks of the C ABI: the library loads, exports what include/ls.h declares, validates
arguments synchronously (through a host-only context, so no GPU is needed), and keeps its options.
No compute call reaches a device here."""
import ctypes
import os
import re
import subprocess

import pytest

from paper_2311_04362_amd import ls

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ls.h")

# Fake, 8-byte aligned, never dereferenced: validation runs before any device work.
P = ctypes.c_void_p(0x10000)
NUL = ctypes.c_void_p(0)
S0 = ctypes.c_void_p(0)


def declared_symbols():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^(?:ls_status|void|const char \*)\s*\*?\s*(ls_\w+)\s*\(", text, re.M)))


@pytest.fixture(scope="module")
def L():
    return ls.load()


@pytest.fixture()
def hctx(L):
    h = ctypes.c_void_p()
    assert L.ls_create(-1, ctypes.byref(h)) == ls.LS_OK
    yield h
    L.ls_destroy(h)


def test_exports_match_header(L):
    decl = declared_symbols()
    assert len(decl) >= 15
    out = subprocess.run(["nm", "-D", "--defined-only", ls.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\sT\s(ls_\w+)$", out, re.M))
    assert set(decl) <= exported, set(decl) - exported
    assert sorted(ls.EXPORTS) == decl


def test_library_does_not_link_oracle():
    out = subprocess.run(["ldd", ls.LIB_PATH], capture_output=True, text=True).stdout
    assert "oracle" not in out
    pkg = os.path.join(ROOT, "paper_2311_04362_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".cpp", ".h")):
                src = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in src and "ls_oracle" not in src and "orc_" not in src, f


def test_limits(L):
    z, n = ctypes.c_int32(), ctypes.c_int32()
    assert L.ls_limits(ctypes.byref(z), ctypes.byref(n)) == ls.LS_OK
    assert z.value == 32 and n.value == 2048


def test_null_context(L):
    assert L.ls_last_error(None) == b"null context"
    assert L.ls_sync(None, S0) == ls.LS_ERR_ARG
    assert L.ls_set_option(None, ls.OPT_ZETA, 8, 0.0) == ls.LS_ERR_ARG
    assert L.ls_create(-1, None) == ls.LS_ERR_ARG
    L.ls_destroy(None)


def test_options_roundtrip(L, hctx):
    iv, dv = ctypes.c_int64(), ctypes.c_double()
    assert L.ls_get_option(hctx, ls.OPT_ZETA, ctypes.byref(iv), ctypes.byref(dv)) == ls.LS_OK
    assert iv.value == 8
    assert L.ls_set_option(hctx, ls.OPT_ZETA, 4, 0.0) == ls.LS_OK
    L.ls_get_option(hctx, ls.OPT_ZETA, ctypes.byref(iv), ctypes.byref(dv))
    assert iv.value == 4
    assert L.ls_set_option(hctx, ls.OPT_ZETA, 0, 0.0) == ls.LS_ERR_ARG
    assert L.ls_set_option(hctx, ls.OPT_ZETA, 33, 0.0) == ls.LS_ERR_ARG
    assert L.ls_set_option(hctx, ls.OPT_SEED, 12345, 0.0) == ls.LS_OK
    L.ls_get_option(hctx, ls.OPT_SEED, ctypes.byref(iv), ctypes.byref(dv))
    assert iv.value == 12345
    assert L.ls_set_option(hctx, ls.OPT_UPDATE, 3, 0.0) == ls.LS_ERR_ARG
    assert L.ls_set_option(hctx, ls.OPT_ALPHA, 0, float("nan")) == ls.LS_ERR_ARG
    assert L.ls_get_option(hctx, ls.OPT_GATHER, ctypes.byref(iv), ctypes.byref(dv)) == ls.LS_OK
    assert iv.value == 0
    assert L.ls_set_option(hctx, ls.OPT_GATHER, 1, 0.0) == ls.LS_OK
    L.ls_get_option(hctx, ls.OPT_GATHER, ctypes.byref(iv), ctypes.byref(dv))
    assert iv.value == 1
    assert L.ls_set_option(hctx, ls.OPT_GATHER, 2, 0.0) == ls.LS_ERR_ARG
    assert L.ls_set_option(hctx, ls.OPT_GATHER, 0, 0.0) == ls.LS_OK
    assert L.ls_set_option(hctx, 999, 0, 0.0) == ls.LS_ERR_ARG
    assert b"unknown" in L.ls_last_error(hctx)


def test_sketch_argument_errors(L, hctx):
    ok = dict(m=100, n=10, A=P, lda=16, b=P, d=50, zeta=8, seed=1, B=P, ldb=10, Sb=P)

    def call(**kw):
        a = dict(ok, **kw)
        return L.ls_sketch(hctx, S0, a["m"], a["n"], a["A"], a["lda"], a["b"], a["d"], a["zeta"],
                           a["seed"], a["B"], a["ldb"], a["Sb"])
    assert call() == ls.LS_ERR_DEVICE                 # valid: stops at "no device"
    assert call(A=NUL) == ls.LS_ERR_ARG
    assert call(A=ctypes.c_void_p(0x10004)) == ls.LS_ERR_ARG   # misaligned
    assert call(lda=9) == ls.LS_ERR_ARG
    assert call(ldb=9) == ls.LS_ERR_ARG
    assert call(n=0) == ls.LS_ERR_ARG
    assert call(m=0) == ls.LS_ERR_ARG
    assert call(d=0) == ls.LS_ERR_ARG
    assert call(zeta=0) == ls.LS_ERR_ARG
    assert call(zeta=51, d=50) == ls.LS_ERR_ARG        # zeta > d
    assert call(zeta=33, d=100) == ls.LS_ERR_ARG       # zeta > LS_MAX_ZETA
    assert call(b=NUL) == ls.LS_ERR_ARG                # b without Sb
    assert call(b=NUL, Sb=NUL) == ls.LS_ERR_DEVICE     # both NULL is allowed
    assert call(n=4096, lda=4096, ldb=4096) == ls.LS_ERR_UNSUPPORTED
    assert call(m=1 << 28, zeta=8) == ls.LS_ERR_UNSUPPORTED   # m*zeta >= 2^31


def test_embedding_and_csr_argument_errors(L, hctx):
    assert L.ls_sketch_embedding(hctx, S0, 10, 20, 8, 0, P, P) == ls.LS_ERR_DEVICE
    assert L.ls_sketch_embedding(hctx, S0, 10, 20, 8, 0, NUL, P) == ls.LS_ERR_ARG
    assert L.ls_sketch_embedding(hctx, S0, 10, 4, 8, 0, P, P) == ls.LS_ERR_ARG
    assert L.ls_sketch_csr(hctx, S0, 10, 20, 8, 0, P, P) == ls.LS_ERR_DEVICE
    assert L.ls_sketch_csr(hctx, S0, 10, 20, 8, 0, P, NUL) == ls.LS_ERR_ARG
    assert L.ls_sketch_csr(hctx, S0, 0, 20, 8, 0, P, P) == ls.LS_ERR_ARG


def test_qr_gradient_solve_argument_errors(L, hctx):
    assert L.ls_qr_sketch(hctx, S0, 100, 10, P, 10, P, P, 10, P) == ls.LS_ERR_DEVICE
    assert L.ls_qr_sketch(hctx, S0, 100, 10, P, 10, P, P, 10, NUL) == ls.LS_ERR_DEVICE  # x0 optional
    assert L.ls_qr_sketch(hctx, S0, 9, 10, P, 10, P, P, 10, P) == ls.LS_ERR_ARG    # d < n
    assert L.ls_qr_sketch(hctx, S0, 100, 10, P, 10, P, P, 9, P) == ls.LS_ERR_ARG   # ldr < n
    assert L.ls_qr_sketch(hctx, S0, 100, 10, P, 10, NUL, P, 10, P) == ls.LS_ERR_ARG
    assert L.ls_gradient(hctx, S0, 100, 10, P, 10, P, P, P, NUL) == ls.LS_ERR_DEVICE
    assert L.ls_gradient(hctx, S0, 0, 10, P, 10, P, P, P, NUL) == ls.LS_ERR_ARG
    assert L.ls_gradient(hctx, S0, 100, 10, P, 10, P, NUL, P, NUL) == ls.LS_ERR_ARG
    # the allocation-free form validates alike, then needs a device
    assert L.ls_gradient_noalloc(hctx, S0, 100, 10, P, 10, P, P, P, NUL) == ls.LS_ERR_DEVICE
    assert L.ls_gradient_noalloc(hctx, S0, 0, 10, P, 10, P, P, P, NUL) == ls.LS_ERR_ARG
    assert L.ls_gradient_noalloc(hctx, S0, 100, 10, P, 9, P, P, P, NUL) == ls.LS_ERR_ARG
    assert L.ls_gradient_noalloc(hctx, S0, 100, 4096, P, 4096, P, P, P, NUL) == ls.LS_ERR_UNSUPPORTED
    assert L.ls_precond_solve(hctx, S0, 10, P, 10, P, P) == ls.LS_ERR_DEVICE
    assert L.ls_precond_solve(hctx, S0, 10, P, 5, P, P) == ls.LS_ERR_ARG
    assert L.ls_iterate(hctx, S0, 100, 10, P, 10, P, P, 10, P, 3, NUL) == ls.LS_ERR_DEVICE
    assert L.ls_iterate(hctx, S0, 100, 10, P, 10, P, P, 10, P, -1, NUL) == ls.LS_ERR_ARG
    assert L.ls_solve(hctx, S0, 100, 10, P, 10, P, 200, 5, P) == ls.LS_ERR_DEVICE
    assert L.ls_solve(hctx, S0, 100, 10, P, 10, P, 0, 5, P) == ls.LS_ERR_DEVICE   # d <= 0: 20 n
    assert L.ls_solve(hctx, S0, 9, 10, P, 10, P, 200, 5, P) == ls.LS_ERR_ARG      # m < n
    assert L.ls_solve(hctx, S0, 100, 10, P, 10, P, 5, 5, P) == ls.LS_ERR_ARG      # d < n
    assert L.ls_solve(hctx, S0, 100, 10, P, 10, P, 200, -2, P) == ls.LS_ERR_ARG   # q < 0
    assert L.ls_sync(hctx, S0) == ls.LS_ERR_DEVICE


def test_iterate_damping_needs_parameters(L, hctx):
    assert L.ls_set_option(hctx, ls.OPT_UPDATE, 2, 0.0) == ls.LS_OK
    assert L.ls_iterate(hctx, S0, 100, 10, P, 10, P, P, 10, P, 3, NUL) == ls.LS_ERR_ARG
    assert L.ls_set_option(hctx, ls.OPT_ALPHA, 0, 0.9) == ls.LS_OK
    assert L.ls_set_option(hctx, ls.OPT_BETA, 0, 0.05) == ls.LS_OK
    assert L.ls_iterate(hctx, S0, 100, 10, P, 10, P, P, 10, P, 3, NUL) == ls.LS_ERR_DEVICE


def test_precision_option_and_f32_argument_errors(L, hctx):
    iv, dv = ctypes.c_int64(), ctypes.c_double()
    assert L.ls_set_option(hctx, ls.OPT_PRECISION, 1, 0.0) == ls.LS_OK
    L.ls_get_option(hctx, ls.OPT_PRECISION, ctypes.byref(iv), ctypes.byref(dv))
    assert iv.value == 1
    assert L.ls_set_option(hctx, ls.OPT_PRECISION, 2, 0.0) == ls.LS_ERR_ARG
    P4 = ctypes.c_void_p(0x10004)                       # 4-byte aligned: fine for FP32 arrays
    assert L.ls_sketch_f32(hctx, S0, 100, 10, P, 10, P, 50, 8, 1, P4, 10, P4) == ls.LS_ERR_DEVICE
    assert L.ls_sketch_f32(hctx, S0, 100, 10, P4, 10, P, 50, 8, 1, P4, 10, P4) == ls.LS_ERR_ARG  # A is FP64
    assert L.ls_sketch_f32(hctx, S0, 100, 10, P, 10, P, 50, 8, 1, ctypes.c_void_p(0x10002), 10, P4) == ls.LS_ERR_ARG
    assert L.ls_sketch_f32(hctx, S0, 100, 10, P, 10, NUL, 50, 8, 1, P4, 10, P4) == ls.LS_ERR_ARG  # b without Sb
    assert L.ls_qr_sketch_f32(hctx, S0, 100, 10, P4, 10, P4, P4, 10, P) == ls.LS_ERR_DEVICE
    assert L.ls_qr_sketch_f32(hctx, S0, 100, 10, P4, 10, P4, P4, 10, P4) == ls.LS_ERR_ARG    # x0 is FP64
    assert L.ls_qr_sketch_f32(hctx, S0, 9, 10, P4, 10, P4, P4, 10, NUL) == ls.LS_ERR_ARG     # d < n
    assert L.ls_precond_solve_f32(hctx, S0, 10, P4, 10, P, P) == ls.LS_ERR_DEVICE
    assert L.ls_precond_solve_f32(hctx, S0, 10, P4, 9, P, P) == ls.LS_ERR_ARG
    assert L.ls_solve(hctx, S0, 100, 10, P, 10, P, 200, 5, P) == ls.LS_ERR_DEVICE


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    monkeypatch.setattr(ls, "_lib", None)
    monkeypatch.setattr(ls, "LIB_PATH", str(tmp_path / "libls.so"))
    with pytest.raises(RuntimeError, match="not built"):
        ls.load()


def test_stop_options(L, hctx):
    iv, dv = ctypes.c_int64(), ctypes.c_double()
    assert L.ls_set_option(hctx, ls.OPT_STOP, 1, 0.0) == ls.LS_OK
    assert L.ls_set_option(hctx, ls.OPT_STOP, 2, 0.0) == ls.LS_ERR_ARG
    assert L.ls_set_option(hctx, ls.OPT_GAMMA, 0, 2.0) == ls.LS_OK
    assert L.ls_set_option(hctx, ls.OPT_RHO, 0, -1.0) == ls.LS_ERR_ARG
    L.ls_get_option(hctx, ls.OPT_GAMMA, ctypes.byref(iv), ctypes.byref(dv))
    assert dv.value == 2.0
    L.ls_get_option(hctx, ls.OPT_RHO, ctypes.byref(iv), ctypes.byref(dv))
    assert dv.value == 0.04
    d, q = ctypes.c_int64(), ctypes.c_int32()
    pr = ctypes.c_int32(-1)
    assert L.ls_solve_info(hctx, ctypes.byref(d), ctypes.byref(q), None, None, ctypes.byref(pr)) == ls.LS_OK
    assert pr.value == ls.PRECISION_FP64


def test_server_argument_errors(L):
    h = ctypes.c_void_p()
    assert L.ls_server_create(-1, 0, 16, ctypes.byref(h)) == ls.LS_ERR_ARG        # no budget
    assert L.ls_server_create(-1, 1 << 30, 0, ctypes.byref(h)) == ls.LS_ERR_ARG    # no slots
    assert L.ls_server_create(-1, 1 << 30, 16, ctypes.byref(h)) == ls.LS_OK
    t = ctypes.c_int64()
    try:
        def sub(m=100, n=10, A=P, lda=10, b=P, d=200, q=5, x=P):
            return L.ls_server_submit(h, m, n, A, lda, b, d, q, 0, x, ctypes.byref(t))
        assert sub() == ls.LS_ERR_DEVICE                  # valid: stops at "no device"
        assert sub(m=9) == ls.LS_ERR_ARG
        assert sub(d=9) == ls.LS_ERR_ARG
        assert sub(q=-1) == ls.LS_ERR_ARG
        assert sub(lda=9) == ls.LS_ERR_ARG
        assert sub(A=NUL) == ls.LS_ERR_ARG
        assert sub(x=ctypes.c_void_p(0x10004)) == ls.LS_ERR_ARG
        assert sub(n=4096, lda=4096, m=10000, d=100000) == ls.LS_ERR_UNSUPPORTED
        assert sub(m=1 << 26, n=2000, lda=2000, d=40000) == ls.LS_ERR_ALLOC          # over budget
        assert b"budget" in L.ls_server_last_error(h)
        res = ctypes.c_int()
        assert L.ls_server_wait(h, 12345, 0.0, ctypes.byref(res)) == ls.LS_ERR_ARG   # unknown ticket
        st = (ctypes.c_int64 * 8)()
        assert L.ls_server_stats(h, st) == ls.LS_OK and st[0] == 0 and st[7] == 0
        res_b, su_b = ctypes.c_int64(), ctypes.c_int64()
        assert L.ls_server_footprint(h, 1000, 10, 200, ctypes.byref(res_b), ctypes.byref(su_b)) == ls.LS_OK
        # host-only: A and b; the setup workspace holds at least the QR work matrix and the embedding
        assert res_b.value == 8 * 1000 * 10 + 8 * 1000
        assert su_b.value >= 8 * 200 * 11 + 4 * 8 * 1000
        assert L.ls_server_footprint(h, 1000, 10, 9, ctypes.byref(res_b), ctypes.byref(su_b)) == ls.LS_ERR_ARG
        assert L.ls_server_footprint(h, 1000, 10, 200, None, ctypes.byref(su_b)) == ls.LS_ERR_ARG
        # mixed precision: the setup lane also holds the FP32 work matrix, S b and the start's buffers
        assert L.ls_server_set_precision(h, 2) == ls.LS_ERR_ARG
        assert L.ls_server_set_precision(None, 1) == ls.LS_ERR_ARG
        assert L.ls_server_set_precision(h, ls.PRECISION_MIXED) == ls.LS_OK
        su_m = ctypes.c_int64()
        assert L.ls_server_footprint(h, 1000, 10, 200, ctypes.byref(res_b), ctypes.byref(su_m)) == ls.LS_OK
        assert su_m.value >= su_b.value + 4 * 200 * 11 + 8 * 200
        assert sub() == ls.LS_ERR_DEVICE
        assert L.ls_server_set_precision(h, ls.PRECISION_FP64) == ls.LS_OK
        assert L.ls_server_footprint(h, 1000, 10, 200, ctypes.byref(res_b), ctypes.byref(su_m)) == ls.LS_OK
        assert su_m.value == su_b.value
        used = ctypes.c_int32()
        assert L.ls_server_request_precision(h, 12345, ctypes.byref(used)) == ls.LS_ERR_ARG
        assert L.ls_server_request_precision(h, 12345, None) == ls.LS_ERR_ARG
    finally:
        L.ls_server_destroy(h)
