"""Build the HIP library ``libvlbm.so`` (gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRCS = [os.path.join(HERE, "csrc", "vlbm.hip"), os.path.join(HERE, "csrc", "closure.hip")]
OUT = os.path.join(HERE, "libvlbm.so")
# the VALU issue-rate probe: a measurement program beside the library
PROBE_SRC = os.path.join(HERE, "csrc", "valu_probe.hip")
PROBE_OUT = os.path.join(HERE, "valu_probe")

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # packed FP32 instructions are kept out of the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = OUT + ".tmp"
    cmd = [hipcc, *HIPCC_FLAGS, "-o", tmp, *SRCS]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, OUT)
    probe = [hipcc, *[f for f in HIPCC_FLAGS if f not in ("-fPIC", "-shared")], "-o", PROBE_OUT + ".tmp", PROBE_SRC]
    if verbose:
        print(" ".join(probe), flush=True)
    subprocess.check_call(probe)
    os.replace(PROBE_OUT + ".tmp", PROBE_OUT)
    return OUT


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
