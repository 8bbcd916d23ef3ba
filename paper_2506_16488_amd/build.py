"""Builds the gfx950 HIP libraries in-tree with hipcc: libppsp.so (the
search library behind include/ppsp.h) and libppsp_probe.so (the benchmark's
scattered-access probe, outside the search library's interface)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
SO = os.path.join(HERE, "libppsp.so")
SOURCES = ["engine.hip", "kernels.hip", "mlp.hip"]
PROBE_SO = os.path.join(HERE, "libppsp_probe.so")
PROBE_SOURCES = ["randbench.hip"]
ARCH = "gfx950"


def hipcc_command(out: str, sources=None) -> list:
    return [
        os.environ.get("HIPCC", "/opt/rocm/bin/hipcc"),
        "--offload-arch=" + ARCH,
        "-O3", "-std=c++17", "-fPIC", "-shared",
        # no packed-FP32 instructions in device code
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-I", os.path.join(ROOT, "include"),
        "-o", out,
    ] + [os.path.join(CSRC, s) for s in (SOURCES if sources is None else sources)]


def build(verbose: bool = False) -> str:
    for so, sources in ((SO, SOURCES), (PROBE_SO, PROBE_SOURCES)):
        tmp = so + ".tmp%d" % os.getpid()
        cmd = hipcc_command(tmp, sources)
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        os.replace(tmp, so)
    return SO


if __name__ == "__main__":
    build(verbose=True)
    print(SO)
    sys.exit(0)
