"""Compile the HIP planner library ``libtwa.so`` for gfx950 (in-tree)."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = [os.path.join(HERE, "csrc", "twa.hip"), os.path.join(HERE, "csrc", "adjoint.hip")]
LIB = os.path.join(HERE, "libtwa.so")
ARCH = os.environ.get("TWA_OFFLOAD_ARCH", "gfx950")


def build(verbose: bool = False) -> str:
    # -ffp-contract=on: a*b+c is fused only within one source expression, so
    # every kernel that inlines a device function (plain, dense, batched)
    # rounds it identically and their results stay bitwise equal.
    cmd = ["hipcc", f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=on",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I", os.path.join(ROOT, "include"), "-o", LIB + ".tmp"] + SRC
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
