"""Build the HIP library libphipm.so in-tree for gfx950."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = [os.path.join(HERE, "csrc", f) for f in ("phipm_api.hip", "batch.hip", "mlp.hip")]
LIB = os.path.join(HERE, "libphipm.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    "-Wall",
    "-Werror=return-type",
    # keep packed-FP32 instructions out of the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # per-lane LDS atomics (pivot search) stay per-lane instead of becoming a
    # scalar loop over the active lanes
    "-mllvm", "-amdgpu-atomic-optimizer-strategy=None",
    # callers assume the calling convention's clobbers instead of the callee's
    # actual register use: the persistent solver's register allocation (and
    # speed) then does not shift with every change inside its out-of-line
    # phases (the step decision, the proposer)
    "-mllvm", "-enable-ipra=false",
    "-I", os.path.join(ROOT, "include"),
]


def build(verbose: bool = False) -> str:
    """Compile every source to an object in parallel, then link."""
    objdir = os.path.join(ROOT, "_build")
    os.makedirs(objdir, exist_ok=True)
    compile_flags = [f for f in FLAGS if f != "-shared"]
    procs, objs = [], []
    for src in SRC:
        obj = os.path.join(objdir, os.path.basename(src) + ".o")
        cmd = [HIPCC, *compile_flags, "-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((subprocess.Popen(cmd), cmd))
        objs.append(obj)
    for proc, cmd in procs:
        if proc.wait() != 0:
            raise subprocess.CalledProcessError(proc.returncode, cmd)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
