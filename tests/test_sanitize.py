"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only, no device work).

* The oracle (oracle/ls_oracle.c) built with gcc and both sanitizers, every entry point called once
  on small inputs (tests/sanitize/oracle_driver.c).
* The host side of libls -- argument checks of every C-ABI entry point, the arena sizing of every
  workspace carve, the served stream's admission bookkeeping -- built with hipcc, the sanitizers on
  the host code only (the device code is compiled as usual), driven through host-only contexts and
  servers (tests/sanitize/host_driver.cpp).
Any out-of-bounds access, use after free, leak or undefined operation fails the run."""
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
CSRC = os.path.join(ROOT, "paper_2311_04362_amd", "csrc")
INCLUDE = os.path.join(ROOT, "include")
HIPCC = "/opt/rocm/bin/hipcc"
CLANG = "/opt/rocm/llvm/bin/clang++"
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="halt_on_error=1")


def run(cmd, **kw):
    return subprocess.run(cmd, capture_output=True, text=True, **kw)


def test_oracle_under_sanitizers(tmp_path):
    if not shutil.which("gcc"):
        pytest.skip("gcc not found")
    exe = str(tmp_path / "oracle_asan")
    r = run(["gcc", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
             "-fno-omit-frame-pointer", "-fopenmp", "-std=c11", os.path.join(ROOT, "oracle", "ls_oracle.c"),
             os.path.join(HERE, "oracle_driver.c"), "-o", exe, "-lm"])
    assert r.returncode == 0, r.stderr
    r = run([exe], env=ENV, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "all calls clean" in r.stdout


@pytest.mark.slow
def test_library_host_code_under_sanitizers(tmp_path):
    if not (os.path.exists(HIPCC) and os.path.exists(CLANG)):
        pytest.skip("ROCm compilers not found")
    # the sanitizers apply to the host code only: each -fsanitize= is preceded by -Xarch_host
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-omit-frame-pointer"]
    srcs = sorted(f for f in os.listdir(CSRC) if f.endswith(".hip"))

    def compile_one(f):
        obj = str(tmp_path / (f + ".o"))
        r = run([HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", *san,
                 "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                 "-I", INCLUDE, "-I", CSRC, "-c", os.path.join(CSRC, f), "-o", obj])
        assert r.returncode == 0, r.stderr[-4000:]
        return obj

    with ThreadPoolExecutor(max_workers=min(6, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(compile_one, srcs))
    drv = str(tmp_path / "driver.o")
    r = run([CLANG, "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
             "-I", INCLUDE, "-c", os.path.join(HERE, "host_driver.cpp"), "-o", drv])
    assert r.returncode == 0, r.stderr
    exe = str(tmp_path / "host_asan")
    r = run([HIPCC, "--offload-arch=gfx950", "-g", *san[:4], drv, *objs, "-o", exe,
             "-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx"])
    assert r.returncode == 0, r.stderr[-4000:]
    r = run([exe], env=ENV, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr[-4000:]
    assert "all calls clean" in r.stdout
