"""Build the HIP library ``libbte.so`` for gfx950 in-tree.

    python -m paper_1401_6047_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libbte.so")
SOURCES = [os.path.join(HERE, "csrc", f) for f in ("bte_kernels.hip", "bte_solver.hip", "bte_tune.hip", "bte_batch.hip",
                                                     "bte_mlp.hip", "bte_reconstruct.hip")]
ARCH = os.environ.get("BTE_OFFLOAD_ARCH", "gfx950")

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    # every product and sum rounds as written (explicit fma() calls stay fused),
    # so all kernel forms and launch shapes produce identical bits
    "-ffp-contract=off",
    "-Wall", "-Wno-unused-result",
    # never let the compiler form packed FP32 arithmetic
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
]


# Per-source additions.  The reconstruction kernel keeps its FP64 matrix
# accumulators in ordinary VGPRs: with the accumulator-register form the
# compiler copied all of them between the two register files on every loop
# iteration.
EXTRA_FLAGS = {
    "bte_reconstruct.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"],
}
OBJ_DIR = os.path.join(ROOT, "_build")


def build(verbose: bool = False) -> str:
    """Compile every source to an object (in parallel), then link the shared
    library; every call compiles afresh."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    os.makedirs(OBJ_DIR, exist_ok=True)
    procs, objs = [], []
    for src in SOURCES:
        name = os.path.basename(src)
        obj = os.path.join(OBJ_DIR, name + ".o")
        cmd = [hipcc, *HIPCC_FLAGS, *EXTRA_FLAGS.get(name, []), "-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((subprocess.Popen(cmd), cmd))
        objs.append(obj)
    failed = [cmd for p, cmd in procs if p.wait() != 0]
    if failed:
        raise subprocess.CalledProcessError(1, failed[0])
    tmp = LIB + ".tmp"
    cmd = [hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
