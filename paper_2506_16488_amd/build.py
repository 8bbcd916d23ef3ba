"""Builds the gfx950 HIP library libppsp.so in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
SO = os.path.join(HERE, "libppsp.so")
SOURCES = ["engine.hip", "kernels.hip", "mlp.hip", "randbench.hip"]
ARCH = "gfx950"


def hipcc_command(out: str) -> list:
    return [
        os.environ.get("HIPCC", "/opt/rocm/bin/hipcc"),
        "--offload-arch=" + ARCH,
        "-O3", "-std=c++17", "-fPIC", "-shared",
        # no packed-FP32 instructions in device code
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-I", os.path.join(ROOT, "include"),
        "-o", out,
    ] + [os.path.join(CSRC, s) for s in SOURCES]


def build(verbose: bool = False) -> str:
    tmp = SO + ".tmp%d" % os.getpid()
    cmd = hipcc_command(tmp)
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, SO)
    return SO


if __name__ == "__main__":
    build(verbose=True)
    print(SO)
    sys.exit(0)
