"""Build libdd.so (HIP, gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libdd.so")
SOURCES = ["dd_kernels.hip", "dd_batch.hip", "unet_kernels.hip", "unet_conv.hip", "dd_host.cpp",
           "dd_queries.cpp", "dd_tune.cpp", "unet.cpp", "dd_visits.hip", "dd_visits_host.cpp", "dd_noalloc.hip",
           "dd_render.hip"]
FLAGS = ["-O3", "--offload-arch=gfx950", "-std=c++17", "-fPIC", "-Wall",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


# Host-side AddressSanitizer and UndefinedBehaviorSanitizer (device code is
# not instrumented); the runtime is preloaded into the process that loads
# the library (see sanitize.py).
SAN_FLAGS = ["-g", "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=all"]


def build(verbose: bool = False, sanitize: bool = False) -> str:
    """Compile every source for gfx950 and link libdd.so; always rebuilds.
    With sanitize, the host code is instrumented and the library goes to
    _build/san/libdd.so instead."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    objdir = os.path.join(HERE, "_build", "san" if sanitize else "")
    os.makedirs(objdir, exist_ok=True)
    procs = []
    objs = []
    for src in SOURCES:
        obj = os.path.join(objdir, src.rsplit(".", 1)[0] + ".o")
        objs.append(obj)
        cmd = [hipcc, *FLAGS, *(SAN_FLAGS if sanitize else []), "-c", os.path.join(CSRC, src),
               "-o", obj]
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
    failed = []
    for src, p in procs:
        out, _ = p.communicate()
        text = "\n".join(l for l in out.decode(errors="replace").splitlines()
                         if "packed-fp32-ops" not in l)
        if p.returncode != 0:
            failed.append((src, text))
        elif verbose and text.strip():
            print(text)
    if failed:
        raise RuntimeError("libdd build failed:\n" + "\n".join(f"[{s}]\n{t}" for s, t in failed))
    lib = os.path.join(objdir, "libdd.so") if sanitize else LIB
    tmp = lib + ".tmp%d" % os.getpid()
    subprocess.check_call([hipcc, "-shared", "-fPIC", "--offload-arch=gfx950", *objs, "-o", tmp])
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
