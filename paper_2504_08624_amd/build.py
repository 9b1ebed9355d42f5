"""Build libtfx.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_2504_08624_amd.build

Every HIP source is compiled for gfx950 only, with packed-FP32 instruction
selection disabled (``-target-feature -packed-fp32-ops``) and matrix-core
accumulators in ordinary vector registers (``-amdgpu-mfma-vgpr-form``: the
fused Toeplitz FIR's accumulators then share registers with the cascade's
working set instead of adding accumulator registers), then linked into
``paper_2504_08624_amd/libtfx.so`` next to this file.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libtfx.so")

ARCH = "gfx950"
HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-mllvm", "-amdgpu-mfma-vgpr-form=1",
             "-Wno-unused-command-line-argument"]
CXX_FLAGS = ["-x", "c++", "-O2", "-std=c++17", "-fPIC", "-I", "/opt/rocm/include"]


def sources():
    hip = sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))
    cpp = sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".cpp"))
    return hip, cpp


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False) -> str:
    """Compile every HIP/C++ source and link libtfx.so; returns its path."""
    hip, cpp = sources()
    cc = hipcc()
    with tempfile.TemporaryDirectory(prefix="tfx_build_") as tmp:
        cmds, objs = [], []
        for src in hip + cpp:
            obj = os.path.join(tmp, os.path.basename(src) + ".o")
            if src.endswith(".hip"):
                cmd = [cc, "-x", "hip", *HIP_FLAGS, "-I", INCLUDE, "-I", CSRC, "-c", src, "-o", obj]
            else:
                cmd = [cc, *CXX_FLAGS, "-D__HIP_PLATFORM_AMD__", "-I", INCLUDE, "-I", CSRC, "-c", src, "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            cmds.append(cmd)
            objs.append(obj)
        # one compiler process per source, at most as many as the CPUs this
        # process may use (and never more than 16)
        jobs = max(1, min(16, len(os.sched_getaffinity(0)), len(cmds)))
        with ThreadPoolExecutor(jobs) as pool:
            for r in list(pool.map(lambda c: subprocess.run(c, check=True), cmds)):
                pass
        tmp_lib = LIB + ".tmp%d" % os.getpid()
        cmd = [cc, "-shared", f"--offload-arch={ARCH}", "-o", tmp_lib, *objs]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        os.replace(tmp_lib, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
