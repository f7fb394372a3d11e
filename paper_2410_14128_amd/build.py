"""Compile the HIP library libhvf.so for gfx950 (in-tree).

Flags: -O3; -ffp-contract=off (plane times are two separately rounded fp32 operations);
packed-fp32 instructions disabled for device code; hipcc's default correctly rounded
fp32 division is kept (no fast-math).
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
SO = os.path.join(HERE, "libhvf.so")
SOURCES = ["hvf_build.cpp", "hvf_paper.cpp", "hvf_api.hip", "hvf_trace.hip", "hvf_batch.hip", "hvf_server.hip", "hvf_devbuild.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"


def flags():
    return ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wno-unused-command-line-argument",
            "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def build(verbose: bool = False) -> str:
    """Always recompiles (this is the does-it-build check); returns the library path. The
    sources compile concurrently (at most 4 compiler processes)."""
    from concurrent.futures import ThreadPoolExecutor

    objs = []
    cmds = []
    builddir = os.path.join(HERE, "_build")
    os.makedirs(builddir, exist_ok=True)
    for src in SOURCES:
        obj = os.path.join(builddir, os.path.splitext(src)[0] + ".o")
        lang = ["-x", "hip"] if src.endswith(".hip") else []
        cmds.append([HIPCC] + flags() + lang + ["-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    # Longest compiles first, so the pool finishes together.
    order = sorted(range(len(cmds)), key=lambda i: SOURCES[i] not in ("hvf_trace.hip", "hvf_devbuild.hip"))
    with ThreadPoolExecutor(max_workers=min(4, os.cpu_count() or 1)) as pool:
        futs = []
        for i in order:
            if verbose:
                print(" ".join(cmds[i]), flush=True)
            futs.append(pool.submit(subprocess.check_call, cmds[i]))
        for f in futs:
            f.result()
    tmp = SO + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, SO)
    return SO


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(SO)
