"""Build the HIP library (gfx950) of the batched physics step in-tree.

    python -m paper_2207_03530_amd.build [--incremental]

produces paper_2207_03530_amd/libvmas.so from csrc/*.hip with hipcc: every
source is compiled to an object file in parallel, then the objects are
linked. FP32 contraction is off (every fused multiply-add is explicit in the
source) and packed FP32 instructions are disabled. --incremental recompiles
only the sources whose object is older than the source or a header.
"""
import concurrent.futures
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.normpath(os.path.join(HERE, "..", "include"))
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libvmas.so")
# Host-side AddressSanitizer + UndefinedBehaviorSanitizer build of the C
# boundary (argument validation, plan building): --sanitize. Device code is
# built as usual (each -fsanitize= applies to the host pass only).
LIB_SAN = os.path.join(HERE, "libvmas_san.so")
SAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer",
             "-g"]
SOURCES = ["vmas_runtime.hip", "vmas_kernels.hip", "vmas_backward.hip", "vmas_mlp.hip",
           "vmas_mlp_api.hip", "vmas_surrogate.hip"]
ARCH = os.environ.get("VMAS_OFFLOAD_ARCH", "gfx950")
FLAGS = [f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wall",
         "-Wno-unused-function", "-I", INCLUDE]


def hipcc() -> str:
    for c in (os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc"), "hipcc"):
        if os.path.sep not in c or os.path.exists(c):
            return c
    return "hipcc"


def _headers():
    hs = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".h")]
    hs += [os.path.join(INCLUDE, f) for f in os.listdir(INCLUDE) if f.endswith(".h")]
    return hs


def _compile(src: str, verbose: bool, sanitize: bool = False) -> str:
    obj = os.path.join(OBJ, os.path.splitext(src)[0] + (".san.o" if sanitize else ".o"))
    cmd = [hipcc()] + FLAGS + (SAN_FLAGS if sanitize else []) + ["-c", "-o", obj + ".tmp",
                                                                 os.path.join(CSRC, src)]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(obj + ".tmp", obj)
    return obj


def build_sanitized(verbose: bool = False) -> str:
    """libvmas_san.so: the host code of the C boundary under ASan and UBSan
    (the runtime source; the kernel sources are linked from the plain
    build's objects, which build() must have made)."""
    os.makedirs(OBJ, exist_ok=True)
    san = _compile("vmas_runtime.hip", verbose, sanitize=True)
    objs = [san] + [os.path.join(OBJ, os.path.splitext(s)[0] + ".o") for s in SOURCES[1:]]
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-Xarch_host",
           "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined", "-o", LIB_SAN + ".tmp"] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB_SAN + ".tmp", LIB_SAN)
    return LIB_SAN


def build(verbose: bool = False, incremental: bool = False) -> str:
    os.makedirs(OBJ, exist_ok=True)
    newest_header = max(os.path.getmtime(h) for h in _headers())
    todo = []
    for src in SOURCES:
        obj = os.path.join(OBJ, os.path.splitext(src)[0] + ".o")
        if incremental and os.path.exists(obj):
            t = os.path.getmtime(obj)
            if t >= os.path.getmtime(os.path.join(CSRC, src)) and t >= newest_header:
                continue
        todo.append(src)
    workers = max(1, min(len(todo), os.cpu_count() or 1, 8))
    with concurrent.futures.ThreadPoolExecutor(workers) as ex:
        list(ex.map(lambda s: _compile(s, verbose), todo))
    objs = [os.path.join(OBJ, os.path.splitext(s)[0] + ".o") for s in SOURCES]
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", LIB + ".tmp"] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    if "--sanitize" in sys.argv[1:]:
        build_sanitized(verbose=True)
    else:
        build(verbose=True, incremental="--incremental" in sys.argv[1:])
    sys.exit(0)
