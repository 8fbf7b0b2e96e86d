"""Build the gfx950 HIP library libhww.so in-tree (hipcc, no JIT)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libhww.so")
SOURCES = ["hww_runtime.hip", "hww_sweep.hip", "hww_losm.hip", "hww_adjoint.hip", "hww_comb.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # Bit-reproducible flight arithmetic: no FMA contraction of a*b+c.
    "-ffp-contract=off",
    # Hardware FP64 atomics on coarse-grained device memory.
    "-munsafe-fp-atomics",
    # No packed FP32 instructions.
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # Atomics stay single instructions: the compiler's wave-level rewrite of
    # uniform-address atomics (a loop over the active lanes) costs the sweep
    # more than it saves, since its uniform-address updates already come
    # from one lane (1.6 % of the launch).
    "-mllvm", "-amdgpu-atomic-optimizer-strategy=None",
    "-Wall", "-Wno-unused-result",
    "-I", os.path.join(ROOT, "include"),
]


def build(verbose: bool = False) -> str:
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    tmp = LIB + ".tmp"
    cmd = [HIPCC, *FLAGS, "-o", tmp, *srcs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
