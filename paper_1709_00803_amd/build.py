"""Builds paper_1709_00803_amd/libigks.so (HIP, gfx950) in-tree with hipcc."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libigks.so")
ARCH = os.environ.get("IGKS_OFFLOAD_ARCH", "gfx950")

# packed FP32 instructions stay disabled for all device code
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def build(verbose: bool = False) -> str:
    bdir = os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)
    common = ["hipcc", f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-Wall"]
    kobj = os.path.join(bdir, "igks_kernels.o")
    hobj = os.path.join(bdir, "igks_host.o")
    _run(common + DEVICE_FLAGS + ["-c", os.path.join(CSRC, "igks_kernels.hip"), "-o", kobj], verbose)
    _run(common + ["-x", "hip", "-c", os.path.join(CSRC, "igks_host.cpp"), "-o", hobj], verbose)
    _run(["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", LIB + ".tmp", kobj, hobj], verbose)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
