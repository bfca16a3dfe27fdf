"""Builds libbbc.so (HIP, gfx950) in-tree.

Each source is compiled to an object in parallel, then the objects are
linked into the shared library (every translation unit keeps its own device
code, so this equals one hipcc call over all sources).

Usage: python -m paper_2601_17707_amd.build  (or build() from Python).
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libbbc.so")
SOURCES = ["api.hip", "build.hip", "dense.hip", "dynamic.hip", "planner.hip", "primitives.hip", "wedge.hip"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-Wall",
    # no packed fp32 instructions in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]
LINK_FLAGS = [
    "--offload-arch=gfx950",
    "-shared",
    "-Wl,-z,defs",  # no undefined symbols in the shared library
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False, out: str = LIB, defines: tuple = ()) -> str:
    """Compiles every source and links `out`; `defines` are extra -D flags."""
    cc = hipcc()
    jobs = max(1, min(len(SOURCES), os.cpu_count() or 1, 16))
    with tempfile.TemporaryDirectory(prefix="bbc_build_") as tmpdir:
        objs = [os.path.join(tmpdir, os.path.splitext(s)[0] + ".o") for s in SOURCES]
        cmds = [[cc, *HIPCC_FLAGS, *[f"-D{d}" for d in defines], "-c", "-o", o, os.path.join(CSRC, s)]
                for s, o in zip(SOURCES, objs)]

        def run(cmd):
            if verbose:
                print(" ".join(cmd), flush=True)
            return subprocess.run(cmd, cwd=CSRC).returncode

        with ThreadPoolExecutor(jobs) as ex:
            rcs = list(ex.map(run, cmds))
        if any(rcs):
            raise subprocess.CalledProcessError(max(rcs), "hipcc")
        tmp = out + ".tmp"
        link = [cc, *LINK_FLAGS, "-o", tmp, *objs]
        if verbose:
            print(" ".join(link), flush=True)
        subprocess.check_call(link, cwd=CSRC)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
