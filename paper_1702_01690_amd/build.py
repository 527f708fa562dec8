"""Build the gfx950 HIP library ``libolb.so`` and the measurement program
``olb_probes`` in-tree with hipcc."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libolb.so")
PROBES = os.path.join(HERE, "olb_probes")
SOURCES = ["olb_kernels.hip", "olb_runtime.hip", "olb_closure.hip"]
ARCH = os.environ.get("OLB_OFFLOAD_ARCH", "gfx950")

FLAGS = ["-O3", "-std=c++17", "-fPIC", "-shared", f"--offload-arch={ARCH}",
         # packed FP32 instructions are disabled for all device code
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         # the stage kernel's population loop must unroll fully (its accumulators
         # are indexed by population); the default size limit left the FP32
         # specular-x instantiations rolled, with the accumulators in scratch
         "-mllvm", "-pragma-unroll-threshold=100000",
         "-Wall", "-Wno-unused-function",
         "-I", os.path.join(ROOT, "include")]


def build(verbose: bool = False) -> str:
    cmd = ["hipcc"] + FLAGS + [os.path.join(CSRC, s) for s in SOURCES] + ["-o", LIB + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    build_probes(verbose)
    return LIB


def build_probes(verbose: bool = False) -> str:
    """The roofline probes (instruction issue costs, the stage kernel's memory
    pattern without its arithmetic): a program of their own."""
    flags = [f for f in FLAGS if f not in ("-fPIC", "-shared")]
    cmd = ["hipcc"] + flags + [os.path.join(CSRC, "olb_probes.hip"), "-o", PROBES + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(PROBES + ".tmp", PROBES)
    return PROBES


if __name__ == "__main__":
    print(build(verbose=True))
    sys.exit(0)
