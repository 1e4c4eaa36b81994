"""Builds the library with AddressSanitizer and UndefinedBehaviorSanitizer on its host
code (device code as usual) into paper_2001_07158_amd/_build_san/libtpm_san.so, for the
CPU test that reruns the ABI checks against it.  Host code only: every sanitizer flag
is passed through -Xarch_host."""

from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, ROOT)
from paper_2001_07158_amd import build as lib_build  # noqa: E402

OUT = os.path.join(ROOT, "paper_2001_07158_amd", "_build_san")
LIB = os.path.join(OUT, "libtpm_san.so")
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=all"]


def build() -> str:
    os.makedirs(OUT, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(lib_build.CSRC, "*.hip")))

    def one(src):
        obj = os.path.join(OUT, os.path.basename(src) + ".o")
        cmd = [lib_build.HIPCC, *lib_build.COMMON, *HOST_SAN, "-c", src, "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode:
            raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr[-3000:]}")
        return obj

    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(one, srcs))
    cmd = [lib_build.HIPCC, f"--offload-arch={lib_build.ARCH}", "-shared", "-fPIC", *HOST_SAN,
           "-Xarch_host", "-shared-libasan", *objs, "-o", LIB]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode:
        raise RuntimeError(f"link failed:\n{r.stderr[-3000:]}")
    return LIB


if __name__ == "__main__":
    print(build())
