"""Builds libhoqri.so (the HIP library behind include/hoqri.h) for gfx950,
and libhoqri_gather.so (include/hoqri_gather.h), the gather-only measurement
aid built from measure/*.hip.

Each csrc/*.hip file is compiled separately with hipcc and linked into
paper_2510_16930_amd/libhoqri.so. Packed float32 instructions are disabled
(-packed-fp32-ops) for every HIP translation unit, and matrix-core
accumulators are kept in ordinary vector registers (-amdgpu-mfma-vgpr-form):
in the segment passes, whose accumulators are reset at slice ends, the
accumulator-register form copies every accumulator out and back in each step.
The segment passes are also compiled with regions of wave-uniform branches
left unstructured (-structurizecfg-skip-uniform-regions): their block loops
branch on wave-uniform slice bounds only, and structurizing those regions
puts copies of the accumulators and of undefined scalar values on the path
of every 16-nonzero block.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OUT = os.path.join(PKG, "libhoqri.so")
MEASURE = os.path.join(PKG, "measure")
GATHER_OUT = os.path.join(PKG, "libhoqri_gather.so")
BUILD_DIR = os.path.join(ROOT, "_build")

ARCH = os.environ.get("HOQRI_ARCH", "gfx950")
HIPCC = os.environ.get("HIPCC", shutil.which("hipcc") or "/opt/rocm/bin/hipcc")
FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-fPIC", "-std=c++17", "-Wall",
    "-Wno-unused-function", "-Wno-unused-variable",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-mllvm", "-amdgpu-mfma-vgpr-form",
    "-I", os.path.join(ROOT, "include"),
]


def sources(folder: str = CSRC):
    return sorted(os.path.join(folder, f) for f in os.listdir(folder) if f.endswith(".hip"))


# extra flags per translation unit
FILE_FLAGS = {"segpass.hip": ["-mllvm", "-structurizecfg-skip-uniform-regions=true"]}


def _compile(src: str) -> str:
    obj = os.path.join(BUILD_DIR, os.path.basename(src)[:-4] + ".o")
    cmd = [HIPCC, *FLAGS, *FILE_FLAGS.get(os.path.basename(src), []), "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


def _link(objs, out: str) -> None:
    tmp = out + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, out)


def build(verbose: bool = False, jobs: int = 4) -> str:
    """Compiles every HIP source, links libhoqri.so and libhoqri_gather.so;
    returns the path of libhoqri.so."""
    os.makedirs(BUILD_DIR, exist_ok=True)
    srcs, msrcs = sources(), sources(MEASURE)
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(_compile, srcs + msrcs))
    _link(objs[:len(srcs)], OUT)
    _link(objs[len(srcs):], GATHER_OUT)
    if verbose:
        print(f"built {OUT} from {len(srcs)} sources, {GATHER_OUT} from {len(msrcs)}")
    return OUT


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
