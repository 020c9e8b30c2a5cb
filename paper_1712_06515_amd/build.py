"""Build the gfx950 shared library ``libccr.so`` in-tree with hipcc."""

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libccr.so")
SOURCES = [os.path.join(CSRC, "ccr_host.cpp"), os.path.join(CSRC, "ccr_kernels.hip")]
ARCH = os.environ.get("CCR_OFFLOAD_ARCH", "gfx950")

# Packed FP32 instructions are disabled for all device code (hipcc -O3 would form them from
# float2 arithmetic).
HIP_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def build(out=LIB, extra=(), quiet=True):
    cmd = ["hipcc", f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
           "-Wall", "-Wno-unused-function", *HIP_FLAGS, "-I", INCLUDE, "-I", CSRC,
           *extra, *SOURCES, "-o", out + ".tmp"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc build of libccr.so failed")
    if not quiet:
        sys.stderr.write(r.stderr)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    print(build(quiet=False))
