"""Compile the HIP library ``libbpida.so`` for gfx950, in-tree.

    python -m paper_1705_02843_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libbpida.so")
SOURCES = ["bpida_kernels.hip", "bpida_batch.hip", "bpida_lb.hip", "bpida_path.hip", "bpida_host.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # no packed-FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
    # the split's level-size table is computed at compile time
    "-fconstexpr-steps=16777216",
    "-I" + os.path.join(ROOT, "include"),
]


# The VALU issue-rate probe the benchmark states its roofline peak with (not
# part of the search library).
PROBE_LIB = os.path.join(HERE, "libvalu_probe.so")
PROBE_SOURCES = ["valu_probe.hip"]


def _compile(sources, out, verbose):
    tmp = out + ".tmp%d" % os.getpid()
    cmd = [HIPCC] + FLAGS + [os.path.join(CSRC, s) for s in sources] + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, out)


def build(verbose: bool = False) -> str:
    _compile(SOURCES, LIB, verbose)
    _compile(PROBE_SOURCES, PROBE_LIB, verbose)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
    sys.exit(0)
