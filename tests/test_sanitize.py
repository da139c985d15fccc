"""Sanitizer builds of the host code (CPU only): the oracle's C source and
libnbreg's host-side argument handling, each compiled with AddressSanitizer
and UndefinedBehaviorSanitizer and driven through every function on small
and edge-case inputs.  Any invalid memory access, leak or undefined
operation aborts the driver and fails the test.  GPU code is not
instrumented (the device code of libnbreg is built as usual)."""
import glob
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests")
CLANG = "/opt/rocm/llvm/bin/clang"
HIPCC = "/opt/rocm/bin/hipcc"
SAN_ENV = dict(os.environ, ASAN_OPTIONS="abort_on_error=1:detect_leaks=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", OMP_NUM_THREADS="2")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout}\n{r.stderr[-4000:]}"
    return r


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_address_and_ub_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_san")
    _run(["gcc", "-O1", "-g", "-std=c11", "-fopenmp", "-ffp-contract=off",
          "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
          "-fno-sanitize-recover=all", "-o", exe,
          os.path.join(ROOT, "oracle", "oracle.c"),
          os.path.join(HERE, "sanitize_oracle_driver.c"), "-lm"])
    r = _run([exe], env=SAN_ENV)
    assert "ok" in r.stdout


@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANG)),
                    reason="ROCm toolchain not available")
def test_library_host_code_under_address_and_ub_sanitizers(tmp_path):
    """Host code instrumented, device code as usual: every sanitizer flag is
    given to the host compilation only."""
    san_host = ["-Xarch_host", "-fsanitize=address",
                "-Xarch_host", "-fsanitize=undefined",
                "-Xarch_host", "-fno-sanitize-recover=all",
                "-Xarch_host", "-fno-omit-frame-pointer"]
    flags = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-ffp-contract=off",
             "-fno-gpu-rdc", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-I", os.path.join(ROOT, "include")]
    srcs = sorted(glob.glob(os.path.join(ROOT, "paper_1504_03687_amd", "csrc", "*.hip")))

    def comp(src):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        _run([HIPCC, *flags, *san_host, "-c", src, "-o", obj])
        return obj

    with ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(comp, srcs))
    lib = str(tmp_path / "libnbreg_san.so")
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", lib, *objs])
    exe = str(tmp_path / "abi_san")
    _run([CLANG, "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
          "-fno-sanitize-recover=all", "-I", os.path.join(ROOT, "include"),
          os.path.join(HERE, "sanitize_abi_driver.c"), "-o", exe, lib,
          f"-Wl,-rpath,{tmp_path}", "-Wl,-rpath,/opt/rocm/lib"])
    r = _run([exe], env=SAN_ENV)
    assert "ok" in r.stdout
