"""Compile the gfx950 HIP sources into ``libih.so`` next to this file.

Usage: ``python -m paper_1711_01656_amd.build`` (or ``build()`` from Python).
hipcc cross-compiles without a GPU present.
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libih.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = [
    "--offload-arch=" + ARCH,
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    # packed FP32 instructions are disabled for every kernel of this library
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
]


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    msgs = [l for l in (res.stdout + res.stderr).splitlines() if "packed-fp32-ops" not in l]
    if res.returncode != 0:
        raise RuntimeError("hipcc failed (%d):\n%s" % (res.returncode, "\n".join(msgs)))
    if verbose and msgs:
        print("\n".join(msgs))


def build(verbose: bool = False, jobs: int = 0) -> str:
    """Compile every HIP source (always, even when a library exists): one
    object per source, compiled in parallel, then linked into libih.so."""
    import tempfile
    from concurrent.futures import ThreadPoolExecutor

    tmp = LIB + ".tmp%d" % os.getpid()
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    cflags = [f for f in FLAGS if f != "-shared"]
    srcs = sources()
    jobs = jobs or min(len(srcs), max(1, min(16, os.cpu_count() or 1)))
    with tempfile.TemporaryDirectory(prefix="ihbuild") as d:
        objs = [os.path.join(d, os.path.basename(s) + ".o") for s in srcs]
        with ThreadPoolExecutor(jobs) as ex:
            for f in [ex.submit(_run, [HIPCC] + cflags + inc + ["-c", s, "-o", o], verbose)
                      for s, o in zip(srcs, objs)]:
                f.result()
        _run([HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs, verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
