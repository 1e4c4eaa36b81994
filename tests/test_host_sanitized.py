"""CPU: the library's host code built with AddressSanitizer and UndefinedBehaviorSanitizer
(device code as usual) passes the C ABI checks: symbol exports, argument validation and
error reporting run without a sanitizer report.  No GPU is touched."""

import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _asan_runtime():
    libs = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return libs[-1] if libs else None


@pytest.mark.skipif(_asan_runtime() is None, reason="needs the ROCm clang ASan runtime")
def test_abi_checks_under_host_asan_ubsan():
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    import host_sanitize_build

    lib = host_sanitize_build.build()
    env = dict(os.environ)
    env.update({
        "LD_PRELOAD": _asan_runtime(),
        "ASAN_OPTIONS": "detect_leaks=0:halt_on_error=1:abort_on_error=1",
        "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1",
        "TPM_LIBRARY": lib,
    })
    code = ("import sys; sys.path.insert(0, %r); from paper_2001_07158_amd import tpm; "
            "assert tpm._lib._name == %r, tpm._lib._name" % (ROOT, lib))
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr[-3000:]
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_lib_abi.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert r.returncode == 0 and " passed" in out, out[-3000:]
