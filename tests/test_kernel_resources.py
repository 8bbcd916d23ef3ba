"""Register budget of the round and hub-list kernels (CPU: hipcc
cross-compiles gfx950).

Both kernels run 20 single-wave workgroups per CU, which are resident
at once only at 5 waves per SIMD (at most 96 registers per lane). At 4, a
fifth of the workgroups start only when others finish and the static chunk
stride leaves them a tail (1.5x the launch time on the 2048^2 lattice), so
every instantiation must keep 5, and the default one (no pull pass, memo,
transpose or dense frontiers) must do so without spilling."""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.fixture(scope="module")
def usage(tmp_path_factory):
    if not os.path.exists(HIPCC) and shutil.which("hipcc") is None:
        pytest.skip("no hipcc")
    out = tmp_path_factory.mktemp("ru") / "k.o"
    r = subprocess.run([HIPCC, "--offload-arch=gfx950", "-O3", "-std=c++17", "-c", "--cuda-device-only",
                        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                        "-Rpass-analysis=kernel-resource-usage", "-I", os.path.join(ROOT, "include"),
                        os.path.join(ROOT, "paper_2506_16488_amd", "csrc", "kernels.hip"), "-o", str(out)],
                       capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-2000:]
    kernels, cur = {}, None
    for line in r.stderr.splitlines():
        m = re.search(r"Function Name: (\S+)", line)
        if m:
            cur = kernels.setdefault(m.group(1), {})
            continue
        m = re.search(r"remark:\s+([A-Za-z ]+?)(?: \[[^\]]*\])?: (\d+)", line)
        if m and cur is not None:
            cur[m.group(1).strip()] = int(m.group(2))
    return kernels


def test_round_kernel_keeps_five_waves_per_simd(usage):
    rounds = {k: v for k, v in usage.items() if "7k_round" in k or "7k_heavy" in k}
    assert len(rounds) >= 10, list(usage)
    for name, u in rounds.items():
        assert u["Occupancy"] >= 5, (name, u)
    default = [v for k, v in rounds.items() if k.startswith("_ZN4ppsp7k_roundILb0ELb0ELb0ELb0E")]
    assert default and default[0]["VGPRs Spill"] == 0 and default[0]["ScratchSize"] == 0, default
