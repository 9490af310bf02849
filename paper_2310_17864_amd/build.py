"""Builds libctcalign.so for gfx950 in-tree with hipcc.

    python -m paper_2310_17864_amd.build        # or build() from Python

Every source compiles in its own hipcc process (in parallel), then one link.
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
SOURCES = ["k_one.hip", "k_batch.hip", "k_multi.hip", "k_serve.hip", "k_misc.hip",
           "api.cpp", "server.cpp", "noalloc.hip", "k_ckpt.hip", "k_beam.hip"]
HEADERS = ["engine.hpp", "internal.hpp", "kernels.hpp", "kernels_common.hpp", "tune.hpp", "ctx.hpp",
           "sched.hpp", os.path.join("..", "..", "include", "ctcalign.h")]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("CTCALIGN_ARCH", "gfx950")
DEVICE_FLAGS = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC",
                # no packed fp32 instructions in the generated code
                "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _compile_cmd(src: str, obj: str):
    lang = ["-x", "hip"] if src.endswith(".cpp") else []
    return [HIPCC] + DEVICE_FLAGS + lang + ["-I", os.path.join(ROOT, "include"),
                                           "-c", os.path.join(CSRC, src), "-o", obj]


def build(verbose: bool = False, jobs: int = 0) -> str:
    """Compile every source and link libctcalign.so (always rebuilds)."""
    jobs = jobs or max(1, min(len(SOURCES), os.cpu_count() or 1, 16))
    with tempfile.TemporaryDirectory() as tmp:
        objs = [os.path.join(tmp, src + ".o") for src in SOURCES]
        todo = list(zip(SOURCES, objs))
        running = []
        failed = []
        while todo or running:
            while todo and len(running) < jobs:
                src, obj = todo.pop(0)
                cmd = _compile_cmd(src, obj)
                if verbose:
                    print(" ".join(cmd))
                running.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE,
                                                      stderr=subprocess.STDOUT, text=True)))
            cmd, pr = running.pop(0)
            out, _ = pr.communicate()
            if pr.returncode != 0:
                failed.append((cmd, out))
        if failed:
            for cmd, out in failed:
                sys.stderr.write(out)
            raise RuntimeError("build failed: " + " ".join(failed[0][0]))
        out_tmp = LIB + ".tmp%d" % os.getpid()
        cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", out_tmp] + objs
        if verbose:
            print(" ".join(cmd))
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            sys.stderr.write(r.stdout + r.stderr)
            raise RuntimeError("link failed: " + " ".join(cmd))
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
