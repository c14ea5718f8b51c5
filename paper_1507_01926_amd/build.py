"""Build libmaxflow.so (the HIP library) in-tree with hipcc for gfx950.

Each translation unit is compiled to an object in parallel, then the objects
are linked into the shared library."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SOURCES = ["csrc/kernels.hip", "csrc/persistent.hip", "csrc/solver.hip", "csrc/server.hip"]
TARGET = os.path.join(HERE, "libmaxflow.so")
OBJDIR = os.path.join(HERE, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # no packed FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def build(verbose: bool = False) -> str:
    os.makedirs(OBJDIR, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include")]
    procs, objs = [], []
    for src in SOURCES:
        obj = os.path.join(OBJDIR, os.path.basename(src).replace(".hip", ".o"))
        cmd = [HIPCC] + FLAGS + inc + ["-c", "-o", obj, os.path.join(HERE, src)]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((subprocess.Popen(cmd), src))
        objs.append(obj)
    failed = [src for p, src in procs if p.wait() != 0]
    if failed:
        raise subprocess.CalledProcessError(1, f"hipcc {' '.join(failed)}")
    link = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", TARGET + ".tmp"] + objs
    if verbose:
        print(" ".join(link), flush=True)
    subprocess.run(link, check=True)
    os.replace(TARGET + ".tmp", TARGET)
    return TARGET


if __name__ == "__main__":
    print(build(verbose="-q" not in sys.argv))
