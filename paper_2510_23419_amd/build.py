"""Build libpbit.so (HIP for gfx950) in-tree with hipcc.

Every source is compiled for gfx950 only, with packed-FP32 instructions
disabled and no floating-point contraction (the host builds the FP64
threshold table, which must not depend on the compiler's choice of FMA).
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor
from pathlib import Path

PKG = Path(__file__).resolve().parent
CSRC = PKG / "csrc"
ROOT = PKG.parent
BUILD = ROOT / "_build" / "pbit"
LIB = PKG / "libpbit.so"

SOURCES = ["host.cpp", "runtime.cpp", "serve.cpp", "ea_kernels.hip", "ea_mfma.hip", "bq_kernels.hip", "bq_slab.hip", "batch_kernels.hip", "graph_kernels.hip", "misc_kernels.hip", "noalloc.cpp", "probe_kernels.hip"]

ARCH = "gfx950"
FLAGS = [
    "--offload-arch=" + ARCH, "-O3", "-fPIC", "-std=c++17", "-Wall", "-Wno-unused-result",
    "-ffp-contract=off", "-fno-fast-math",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + str(ROOT / "include"), "-I" + str(CSRC),
]


def hipcc() -> str:
    exe = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not Path(exe).exists():
        raise RuntimeError("hipcc not found: the HIP library cannot be built")
    return exe


# Per-source flags: the matrix-core cube kernel keeps its MFMA accumulators in
# ordinary VGPRs (no copies out of the accumulation registers before the decisions).
EXTRA = {"ea_mfma.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"]}


def _compile(src: str) -> Path:
    obj = BUILD / (src + ".o")
    cmd = [hipcc(), "-x", "hip", "-c", str(CSRC / src), "-o", str(obj)] + FLAGS + EXTRA.get(src, [])
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed on %s:\n%s\n%s" % (src, r.stdout, r.stderr))
    return obj


def build(verbose: bool = False) -> Path:
    BUILD.mkdir(parents=True, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(len(SOURCES), 8)) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB.with_suffix(".so.tmp%d" % os.getpid())
    # -z defs: a kernel template that the host pass failed to instantiate shows up
    # as an undefined symbol here instead of at load time
    cmd = [hipcc(), "-shared", "-fPIC", "--offload-arch=" + ARCH, "-Wl,-z,defs", "-o", str(tmp)] + [str(o) for o in objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s\n%s" % (r.stdout, r.stderr))
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
