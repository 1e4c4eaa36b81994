"""CPU: the oracle's pins run again against an AddressSanitizer + UndefinedBehaviorSanitizer
build of the C oracle (out-of-bounds accesses, use after free, signed overflow, shifts
out of range and misaligned loads abort the run)."""

import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_pins_under_asan_ubsan():
    sys.path.insert(0, ROOT)
    from oracle import build

    build.build_sanitized()
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True,
                          text=True).stdout.strip()
    ubsan = subprocess.run(["gcc", "-print-file-name=libubsan.so"], capture_output=True,
                           text=True).stdout.strip()
    assert os.path.isabs(asan) and os.path.exists(asan), asan
    env = dict(os.environ)
    env.update({
        "LD_PRELOAD": ":".join(p for p in (asan, ubsan) if os.path.isabs(p)),
        # the interpreter's own allocations are not the oracle's: no leak report
        "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1:halt_on_error=1",
        "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1",
        "TPM_ORACLE_SANITIZED": "1",
        "OMP_NUM_THREADS": "2",
    })
    tests = [os.path.join(ROOT, "tests", f) for f in ("test_oracle_field_hash.py", "test_oracle_pins.py")]
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        "-m", "not gpu and not slow", *tests],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    assert " passed" in out, out[-2000:]
