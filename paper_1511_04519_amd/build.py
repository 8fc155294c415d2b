"""Build libmatex.so (HIP for gfx950 + host C++) in-tree with hipcc."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmatex.so")
OBJ = os.path.join(HERE, "_build")

HIP_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
SOURCES = [("kernels.hip", True), ("batched.hip", True), ("matex.cpp", True),
           ("factor.cpp", False), ("schedule.cpp", False)]


def build(verbose: bool = False) -> str:
    os.makedirs(OBJ, exist_ok=True)
    objs = []
    for src, hip in SOURCES:
        obj = os.path.join(OBJ, src + ".o")
        if hip:
            cmd = ["hipcc", *HIP_FLAGS, "-x", "hip" if src.endswith(".hip") else "hip",
                   "-c", os.path.join(CSRC, src), "-o", obj]
        else:
            cmd = ["g++", "-O3", "-std=c++17", "-fPIC", "-march=x86-64-v2", "-c",
                   os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            sys.stderr.write(r.stdout + r.stderr)
            raise RuntimeError(f"compiling {src} failed")
        objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = ["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs, "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("linking libmatex.so failed")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
