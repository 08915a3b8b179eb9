"""Build the HIP library (gfx950) of the batched physics step in-tree.

    python -m paper_2207_03530_amd.build

produces paper_2207_03530_amd/libvmas.so from csrc/*.hip with hipcc. FP32
contraction is off (every fused multiply-add is explicit in the source) and
packed FP32 instructions are disabled.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libvmas.so")
SOURCES = ["vmas_runtime.hip", "vmas_kernels.hip", "vmas_backward.hip", "vmas_mlp.hip",
           "vmas_mlp_api.hip", "vmas_surrogate.hip"]
ARCH = os.environ.get("VMAS_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for c in (os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc"), "hipcc"):
        if os.path.sep not in c or os.path.exists(c):
            return c
    return "hipcc"


def build(verbose: bool = False) -> str:
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
           "-ffp-contract=off", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Wall", "-Wno-unused-function", "-I", os.path.join(HERE, "..", "include"),
           "-o", LIB + ".tmp"] + [os.path.join(CSRC, s) for s in SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
