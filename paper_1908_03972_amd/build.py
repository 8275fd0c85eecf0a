"""Build libpmgfr.so for gfx950 in-tree with hipcc (no GPU needed to compile).

Every source is compiled to its own object in parallel (the kernels of one source are launched
only from that source, so no relocatable device code is needed), then the objects are linked.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libpmgfr.so")
OBJ = os.path.join(HERE, "_build")
ARCH = os.environ.get("PMGFR_ARCH", "gfx950")

SOURCES = ["api.cpp", "hex_geometry.cpp", "fr_kernels.hip", "fr3_kernels.hip", "jac3_kernels.hip", "jac_kernels.hip",
           "transfer_kernels.hip", "krylov_kernels.hip", "line_kernels.hip", "noalloc.hip"]

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    # keep the compiler from forming packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-munsafe-fp-atomics", "-Wall", "-Wno-unused-result",
]


def hipcc() -> str:
    path = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(path):
        raise RuntimeError("hipcc not found; ROCm is required to build libpmgfr.so")
    return path


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    proc = subprocess.run(cmd, capture_output=True, text=True)
    if proc.returncode != 0:
        sys.stderr.write(proc.stdout + proc.stderr)
        raise RuntimeError(f"hipcc failed with exit code {proc.returncode}: {' '.join(cmd[-3:])}")
    return proc


def build(verbose: bool = False, jobs: int | None = None) -> str:
    os.makedirs(OBJ, exist_ok=True)
    cc = hipcc()
    objs, cmds = [], []
    for s in SOURCES:
        o = os.path.join(OBJ, os.path.splitext(s)[0] + ".o")
        objs.append(o)
        cmds.append([cc, *FLAGS, "-c", "-o", o, os.path.join(CSRC, s)])
    jobs = jobs or max(1, min(len(cmds), os.cpu_count() or 1, 16))
    with cf.ThreadPoolExecutor(jobs) as ex:
        for f in [ex.submit(_run, c, verbose) for c in cmds]:
            f.result()
    tmp = LIB + ".tmp"
    _run([cc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs], verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
