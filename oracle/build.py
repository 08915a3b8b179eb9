"""Build the FP64 CPU oracle (test infrastructure) into oracle/liboracle.so.

The oracle is plain C++17 (FP64) compiled by the host compiler with
floating-point contraction and fast-math switched off, so every operation is
the IEEE double-precision operation written in the source.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "vmas_oracle.cpp")
LIB = os.path.join(HERE, "liboracle.so")
# AddressSanitizer + UndefinedBehaviorSanitizer build (python oracle/build.py
# --sanitize); the tests load it when VMAS_ORACLE_LIB names it
LIB_SAN = os.path.join(HERE, "liboracle_san.so")
SAN_FLAGS = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
             "-fno-sanitize-recover=all"]


def build(verbose: bool = False, sanitize: bool = False) -> str:
    out = LIB_SAN if sanitize else LIB
    opt = SAN_FLAGS if sanitize else ["-O2"]
    cmd = ["g++"] + opt + ["-std=c++17", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
                           "-shared", "-Wall", "-o", out + ".tmp", SRC, "-lpthread"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    build(verbose=True, sanitize="--sanitize" in sys.argv[1:])
    sys.exit(0)
