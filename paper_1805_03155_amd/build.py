"""Build libspstd.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_1805_03155_amd.build
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libspstd.so")
SOURCES = ["kernels.hip", "mixed.hip", "resident.hip", "probes.hip", "planes.hip", "fourstep.hip", "engine.cpp", "batch.cpp",
           "spectrum.cpp"]
ARCH = os.environ.get("SPSTD_OFFLOAD_ARCH", "gfx950")

# Packed FP32 instructions are kept out of the generated code.
HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wall", "-Wno-unused-function", f"-I{os.path.join(ROOT, 'include')}",
             f"-I{CSRC}"]


def _hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False, jobs: int = 3) -> str:
    hipcc = _hipcc()
    tmp = tempfile.mkdtemp(prefix="spstd_build_")
    try:
        objs, procs = [], []
        for src in SOURCES:
            obj = os.path.join(tmp, src + ".o")
            lang = ["-x", "hip"]
            cmd = [hipcc, *HIP_FLAGS, *lang, "-c", os.path.join(CSRC, src), "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            procs.append((subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT), src))
            objs.append(obj)
            if len(procs) >= jobs:
                _drain(procs)
        _drain(procs)
        out_tmp = LIB + ".tmp"
        link = [hipcc, "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", out_tmp]
        subprocess.run(link, check=True)
        os.replace(out_tmp, LIB)
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
    return LIB


def _drain(procs):
    while procs:
        p, src = procs.pop(0)
        out, _ = p.communicate()
        if p.returncode != 0:
            sys.stderr.write(out.decode(errors="replace"))
            raise RuntimeError(f"hipcc failed on {src}")
        elif out.strip():
            sys.stderr.write(out.decode(errors="replace"))


if __name__ == "__main__":
    print(build(verbose=True))
