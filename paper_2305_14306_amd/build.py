"""Build libhav.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_2305_14306_amd.build

Exact binary32 arithmetic is part of the library's contract, so the flags pin it:
no FMA contraction, correctly rounded fp32 division, fp32 denormals kept, and no
packed-fp32 instructions.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SOURCES = [os.path.join(HERE, "csrc", "hav.hip"), os.path.join(HERE, "csrc", "compare.hip"),
           os.path.join(HERE, "csrc", "metrics.hip")]
DEPS = [os.path.join(HERE, "csrc", "hav_device.hpp"), os.path.join(ROOT, "include", "hav.h")]
LIB = os.path.join(HERE, "libhav.so")
ARCH = os.environ.get("HAV_OFFLOAD_ARCH", "gfx950")

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared",
    f"--offload-arch={ARCH}",
    "-ffp-contract=off",
    "-fno-fast-math",
    "-fhip-fp32-correctly-rounded-divide-sqrt",
    "-fno-gpu-flush-denormals-to-zero",
    # no packed fp32 instructions in device code; hipcc hands these cc1 flags to the host
    # pass too, whose target has no such feature: it says so once per function, and
    # build() drops exactly that line (HOST_NOISE) from the output
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
    "-I", os.path.join(ROOT, "include"),
]


HOST_NOISE = "'-packed-fp32-ops' is not a recognized feature for this target (ignoring feature)"


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = LIB + ".tmp"
    cmd = [hipcc] + HIPCC_FLAGS + ["-o", tmp] + SOURCES
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "".join(line for line in r.stdout.splitlines(keepends=True) if line.strip() != HOST_NOISE)
    if out:
        sys.stderr.write(out)
    if r.returncode != 0:
        raise subprocess.CalledProcessError(r.returncode, cmd, out)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
