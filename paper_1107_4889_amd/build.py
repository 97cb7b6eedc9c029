"""Build the HIP library ``liblbrbc.so`` for gfx950 with hipcc (in-tree)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblbrbc.so")
SOURCES = ["lb_kernels.hip", "rbc_kernels.hip", "lbrbc_api.hip"]

# Packed FP32 instructions are disabled for every HIP translation unit. Multiply-adds are
# contracted only within one source expression (-ffp-contract=on), so a device function
# rounds identically wherever it is inlined: the per-context and the fused multi-context
# kernels of a step give bitwise-equal results.
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=on",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-command-line-argument"]


def _torch_hip_dir() -> str:
    import importlib.util

    spec = importlib.util.find_spec("torch")
    if spec is None or spec.origin is None:
        raise RuntimeError("PyTorch (ROCm) is required: it provides the HIP runtime")
    d = os.path.join(os.path.dirname(spec.origin), "lib")
    if not os.path.exists(os.path.join(d, "libamdhip64.so")):
        raise RuntimeError(f"no libamdhip64.so in {d}")
    return d


def build(verbose: bool = False) -> str:
    objs = []
    os.makedirs(os.path.join(HERE, "_build"), exist_ok=True)
    procs = []
    for src in SOURCES:
        obj = os.path.join(HERE, "_build", src.replace(".hip", ".o"))
        cmd = ["hipcc", *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((subprocess.Popen(cmd), cmd))
        objs.append(obj)
    for p, cmd in procs:
        if p.wait() != 0:
            raise RuntimeError("hipcc failed: " + " ".join(cmd))
    tmp = LIB + ".tmp"
    # Link against the HIP runtime that PyTorch loads, so that the process holds a single
    # HIP/HSA runtime (a second one cannot open the device). torch's libamdhip64.so carries
    # no soname, so the dependency is recorded by file name and found through the rpath.
    hiplib = _torch_hip_dir()
    cmd = ["g++", "-shared", "-fPIC", "-o", tmp, *objs, "-L" + hiplib, "-l:libamdhip64.so",
           "-Wl,-rpath," + hiplib, "-Wl,--no-undefined"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
