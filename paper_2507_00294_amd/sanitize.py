"""Host-side sanitizer run of the CPU test suite.

    python -m paper_2507_00294_amd.sanitize [pytest arguments]

Builds the library's host code and the CPU oracle with AddressSanitizer and
UndefinedBehaviorSanitizer (clang of ROCm for both, so that one runtime
serves the process), then runs ``pytest -m "not gpu"`` with those builds
(DD_LIBRARY, DDO_LIBRARY) and the sanitizer runtime preloaded into the
uninstrumented Python.  Any report aborts the run.  Device code is not
instrumented (no GPU sanitizer is used)."""
from __future__ import annotations

import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CLANG = "/opt/rocm/llvm/bin/clang"


def runtime() -> str:
    libs = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not libs:
        raise RuntimeError("no clang AddressSanitizer runtime found")
    return libs[-1]


def build_oracle() -> str:
    out = os.path.join(HERE, "_build", "san", "libddo.so")
    os.makedirs(os.path.dirname(out), exist_ok=True)
    src = os.path.join(ROOT, "oracle", "ddo.c")
    # quadmath.h ships with gcc's own headers
    gcc_inc = subprocess.check_output(["gcc", "-print-file-name=include"], text=True).strip()
    subprocess.check_call([CLANG, "-O1", "-g", "-std=c99", "-D_POSIX_C_SOURCE=200809L", "-fPIC",
                           "-idirafter", gcc_inc,
                           "-shared", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                           "-fno-omit-frame-pointer", "-o", out, src, "-lquadmath", "-lm",
                           "-lpthread"])
    return out


def main(argv) -> int:
    from . import build

    lib = build.build(sanitize=True)
    ora = build_oracle()
    env = dict(os.environ, DD_LIBRARY=lib, DDO_LIBRARY=ora, LD_PRELOAD=runtime(),
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    cmd = [sys.executable, "-m", "pytest", "-q", "-x", "-m", "not gpu", "-p", "no:cacheprovider",
           *argv]
    return subprocess.call(cmd, cwd=ROOT, env=env)


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
