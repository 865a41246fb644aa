"""Builds libucns.so (HIP for gfx950 + host mesh build) in-tree."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libucns.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# Packed FP32 instructions are kept out of the device code.
DEVICE_FLAGS = ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def build(verbose: bool = False) -> str:
    obj_dir = os.path.join(HERE, "_build")
    os.makedirs(obj_dir, exist_ok=True)
    mesh_o = os.path.join(obj_dir, "mesh_build.o")
    kern_o = os.path.join(obj_dir, "ucns_kernels.o")
    cmds = [
        ["g++", "-std=c++17", "-O2", "-fPIC", "-pthread", "-c", os.path.join(CSRC, "mesh_build.cpp"), "-o", mesh_o],
        [HIPCC, "-std=c++17", "-O3", "-fPIC", *DEVICE_FLAGS, "-c", os.path.join(CSRC, "ucns_kernels.hip"), "-o", kern_o],
        [HIPCC, "-shared", "-fPIC", *DEVICE_FLAGS, "-o", LIB + ".tmp", kern_o, mesh_o, "-pthread"],
    ]
    for cmd in cmds:
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            sys.stderr.write(r.stdout + r.stderr)
            raise RuntimeError("libucns build failed: " + " ".join(cmd[:2]))
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
