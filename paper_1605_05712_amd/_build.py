"""Build libahom.so (HIP for gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libahom.so")

# (source, extra defines): the power-of-two kernels are compiled in parts
SOURCES = [("ahom_plan.cpp", []), ("ahom_kernels.hip", []), ("ahom_api.hip", []), ("ahom_batch.hip", []), ("ahom_learn.hip", []), ("ahom_cg.hip", []),
           ("ahom_fast.hip", [])] + [
    ("ahom_fast.hip", [f"-DAHOM_FAST_PART={k}"]) for k in range(12)
]

HIP_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def build(verbose: bool = False) -> str:
    from concurrent.futures import ThreadPoolExecutor

    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    cmds, objs = [], []
    for n, (src, defs) in enumerate(SOURCES):
        path = os.path.join(CSRC, src)
        obj = os.path.join(CSRC, f"_obj_{n}_" + os.path.splitext(src)[0] + ".o")
        if src.endswith(".hip"):
            cmd = [hipcc, *HIP_FLAGS, *defs, "-x", "hip", "-c", path, "-o", obj]
        else:
            cmd = [hipcc, "-O2", "-std=c++17", "-fPIC", "-c", path, "-o", obj]
        cmds.append(cmd)
        objs.append(obj)
    workers = max(1, min(len(cmds), os.cpu_count() or 1, 16))

    def run(cmd):
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)

    with ThreadPoolExecutor(max_workers=workers) as ex:
        list(ex.map(run, cmds))
    tmp = LIB + ".tmp"
    cmd = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp,
           "-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx", "-Wl,-rpath,/opt/rocm/lib"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    for o in objs:
        os.remove(o)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    print(LIB)
    sys.exit(0)
