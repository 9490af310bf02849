"""Builds libctcalign.so for gfx950 in-tree with hipcc.

    python -m paper_2310_17864_amd.build        # or build() from Python
"""
from __future__ import annotations

import os
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libctcalign.so")
SOURCES = ["kernels.hip", "api.cpp", "server.cpp"]
HEADERS = ["engine.hpp", "internal.hpp", "kernels.hpp", "tune.hpp", "ctx.hpp", "sched.hpp",
           os.path.join("..", "..", "include", "ctcalign.h")]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("CTCALIGN_ARCH", "gfx950")
DEVICE_FLAGS = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC",
                # no packed fp32 instructions in the generated code
                "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("build failed: " + " ".join(cmd))
    return r


def build(verbose: bool = False) -> str:
    """Compile every source and link libctcalign.so (always rebuilds)."""
    with tempfile.TemporaryDirectory() as tmp:
        objs = []
        for src in SOURCES:
            obj = os.path.join(tmp, src + ".o")
            lang = ["-x", "hip"] if src.endswith(".cpp") else []
            cmd = [HIPCC] + DEVICE_FLAGS + lang + ["-I", os.path.join(ROOT, "include"),
                                                  "-c", os.path.join(CSRC, src), "-o", obj]
            if verbose:
                print(" ".join(cmd))
            _run(cmd)
            objs.append(obj)
        out_tmp = LIB + ".tmp%d" % os.getpid()
        cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", out_tmp] + objs
        if verbose:
            print(" ".join(cmd))
        _run(cmd)
        os.replace(out_tmp, LIB)
    return LIB


def stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    for f in SOURCES + HEADERS:
        if os.path.getmtime(os.path.join(CSRC, f)) > t:
            return True
    return False


if __name__ == "__main__":
    print(build(verbose=True))
