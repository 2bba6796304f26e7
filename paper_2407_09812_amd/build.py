"""Build libmppi.so (HIP, gfx950) in-tree with hipcc.

Packed FP32 instructions are disabled (-packed-fp32-ops); everything else is
plain -O3 HIP for one target, gfx950.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
SOURCES = [os.path.join(CSRC, f) for f in ("kernels.hip", "batch.hip", "api.hip", "batch_api.hip",
                                           "server.hip")]
HEADERS = [os.path.join(CSRC, f) for f in ("kernels.h", "model.h", "stages.h", "batch.h",
                                           "context.h")] + [
    os.path.join(ROOT, "include", "mppi.h")]
LIB = os.path.join(HERE, "libmppi.so")
ARCH = os.environ.get("MPPI_OFFLOAD_ARCH", "gfx950")


def hipcc_flags():
    return ["-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-Wno-unused-result", "-I", os.path.join(ROOT, "include")]


def build(verbose: bool = False) -> str:
    """Compile every source to an object (in parallel; each translation unit carries
    its own device code), then link the shared library."""
    obj_dir = os.path.join(ROOT, "_build", "mppi")
    os.makedirs(obj_dir, exist_ok=True)
    objs, procs = [], []
    for src in SOURCES:
        obj = os.path.join(obj_dir, os.path.basename(src) + ".o")
        cmd = ["hipcc", *hipcc_flags(), "-pthread", "-c", "-o", obj, src]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((subprocess.Popen(cmd), cmd))
        objs.append(obj)
    failed = [cmd for p, cmd in procs if p.wait() != 0]
    if failed:
        raise subprocess.CalledProcessError(1, failed[0])
    tmp = LIB + ".tmp"
    cmd = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-pthread", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


def is_stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(f) > t for f in SOURCES + HEADERS)


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
