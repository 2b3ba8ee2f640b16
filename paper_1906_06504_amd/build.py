"""Build libgheap.so (HIP, gfx950) in-tree with hipcc.

Usage: python -m paper_1906_06504_amd.build [--trace]   (or call build()).
Each supported node capacity k and entry width (8 or 16 bytes) gets its own
objects of gh_kernels.hip, gh_serve.hip, gh_bu.hip and gh_private.hip, so they
compile in parallel.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libgheap.so")
LIB_TRACE = os.path.join(HERE, "libgheap_trace.so")
KS = (32, 64, 128, 256, 512, 1024)
ARCH = os.environ.get("GHEAP_ARCH", "gfx950")

HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
COMMON = [
    "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def _run(cmd):
    p = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in p.stdout.splitlines()
                    if "packed-fp32-ops" not in l and l.strip())
    if p.returncode != 0:
        raise RuntimeError("command failed: %s\n%s" % (" ".join(cmd), out))
    return out


def build(jobs: int | None = None, verbose: bool = False, trace: bool = False) -> str:
    """Compile every object and link libgheap.so; with trace, the tracing
    build libgheap_trace.so instead (every object with -DGH_PHASE_TRACE: the
    whole-root kernels time-stamp their root phases, include/gheap_trace.h)."""
    build_dir = BUILD + ("_trace" if trace else "")
    lib = LIB_TRACE if trace else LIB
    flags = COMMON + (["-DGH_PHASE_TRACE"] if trace else [])
    os.makedirs(build_dir, exist_ok=True)
    jobs = jobs or min(8, os.cpu_count() or 4)
    tasks = []
    for k in KS:
        for eb in (8, 16):
            for name in ("gh_kernels", "gh_serve", "gh_bu", "gh_private"):
                obj = os.path.join(build_dir, "%s_k%d_e%d.o" % (name, k, eb))
                tasks.append([HIPCC] + flags + ["-DGH_K=%d" % k, "-DGH_ENT_BYTES=%d" % eb, "-c",
                                                os.path.join(CSRC, name + ".hip"), "-o", obj])
    for name in ("gh_setup", "gh_filter"):
        tasks.append([HIPCC] + flags + ["-c", os.path.join(CSRC, name + ".hip"),
                                        "-o", os.path.join(build_dir, name + ".o")])
    tasks.append([HIPCC] + flags + ["-x", "hip", "-c", os.path.join(CSRC, "gheap_api.cpp"),
                                    "-o", os.path.join(build_dir, "gheap_api.o")])
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        outs = list(ex.map(_run, tasks))
    if verbose:
        for o in outs:
            if o:
                print(o)
    objs = [t[t.index("-o") + 1] for t in tasks]
    tmp = lib + ".tmp%d" % os.getpid()
    _run([HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs)
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, trace="--trace" in sys.argv))
