"""Build the b3d HIP library (libb3d.so) for gfx950 with hipcc, in-tree.

Usage: python -m paper_2312_08715_amd.build   (or build() from Python)
"""

from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB_DIR = os.path.join(HERE, "_lib")
LIB_PATH = os.path.join(LIB_DIR, "libb3d.so")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")

SOURCES = ["api.cpp", "mesh.cpp", "smc.cpp", "k_render.hip", "k_score.hip", "k_fused.hip", "k_sample.hip", "k_track.hip",
           "c2f_noalloc.hip"]
# microbenchmarks of the chip's peaks: a library of their own, loaded by the benchmark only
PROBE_SOURCES = ["k_probe.hip"]
PROBE_LIB_PATH = os.path.join(LIB_DIR, "libb3d_probe.so")

HIPCC_FLAGS = [
    "-O3",
    "-std=c++17",
    "--offload-arch=gfx950",
    "-fPIC",
    "-Wall",
    "-Wno-unused-function",
    # keep the compiler from forming packed fp32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False, jobs: int = 8) -> str:
    """Compile every source and link libb3d.so (always rebuilds)."""
    os.makedirs(LIB_DIR, exist_ok=True)
    cc = hipcc()
    objs = []
    tmpdir = tempfile.mkdtemp(prefix="b3d_build_")
    procs = []
    try:
        for src in SOURCES + PROBE_SOURCES:
            obj = os.path.join(tmpdir, os.path.splitext(src)[0] + ".o")
            lang = ["-x", "hip"] if src.endswith(".hip") else []
            cmd = [cc, *HIPCC_FLAGS, "-I", INCLUDE, "-I", CSRC, *lang, "-c", os.path.join(CSRC, src), "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
            objs.append(obj)
            if len([p for _, p in procs if p.poll() is None]) >= jobs:
                procs[0][1].wait()
        for src, p in procs:
            out, _ = p.communicate()
            if p.returncode != 0:
                raise RuntimeError(f"hipcc failed on {src}:\n{out.decode(errors='replace')}")
            if verbose and out:
                print(out.decode(errors="replace"))
        nmain = len(SOURCES)
        for path, part in ((LIB_PATH, objs[:nmain]), (PROBE_LIB_PATH, objs[nmain:])):
            tmp_lib = path + ".tmp"
            subprocess.check_call([cc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp_lib, *part])
            os.replace(tmp_lib, path)
    finally:
        shutil.rmtree(tmpdir, ignore_errors=True)
    return LIB_PATH


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
