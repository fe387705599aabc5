"""Build liblbm.so (gfx950) in-tree with hipcc.

    python -m paper_1410_2569_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblbm.so")
SOURCES = ["lbm_kernels.hip", "lbm_adjoint.hip", "lbm_batch.hip", "lbm_api.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # keep the compiler from forming packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
]


def build(verbose: bool = False) -> str:
    """Compile every HIP source of the library (in parallel) and link liblbm.so. Always
    recompiles."""
    from concurrent.futures import ThreadPoolExecutor

    os.makedirs(os.path.join(HERE, "_build"), exist_ok=True)
    cmds, objs = [], []
    for src in SOURCES:
        obj = os.path.join(HERE, "_build", src.replace(".hip", ".o"))
        cmds.append([HIPCC, *FLAGS, "-I", os.path.join(os.path.dirname(HERE), "include"), "-c",
                     os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    for cmd in cmds:
        if verbose:
            print(" ".join(cmd), flush=True)
    with ThreadPoolExecutor(max_workers=len(cmds)) as pool:
        for f in [pool.submit(subprocess.check_call, cmd) for cmd in cmds]:
            f.result()
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
