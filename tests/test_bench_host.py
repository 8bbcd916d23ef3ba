"""Host logic of bench.py (no GPU): the one-GPU rule, the kernel-source hash
that ties the committed counter profile to the round kernel it measured, and
the fields of that profile."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_kernel_hash_ignores_comments_only(tmp_path):
    srcs = []
    for f in bench.KERNEL_SOURCES:
        dst = tmp_path / os.path.basename(f)
        dst.write_text(open(f).read())
        srcs.append(str(dst))
    saved = bench.KERNEL_SOURCES
    try:
        bench.KERNEL_SOURCES = srcs
        h0 = bench.kernel_source_hash()
        k = tmp_path / "kernels.hip"
        k.write_text("// a new comment line\n" + k.read_text().replace("{\n", "{  /* note */\n", 1) + "\n\n")
        assert bench.kernel_source_hash() == h0
        k.write_text(k.read_text().replace("CARRY_CHECK 2", "CARRY_CHECK 4"))
        assert bench.kernel_source_hash() != h0
    finally:
        bench.KERNEL_SOURCES = saved


def test_traffic_profile_fields():
    t = json.load(open(bench.TRAFFIC_FILE))
    for key in ("kernel", "kernel_source_hash", "fetch_kib_per_launch", "write_kib_per_launch", "fetch_scale",
                "write_scale", "traffic_bytes_per_launch"):
        assert key in t
    assert t["kernel"] == "k_round" and t["traffic_bytes_per_launch"] > 0
    expect = (t["fetch_kib_per_launch"] * t["fetch_scale"] + t["write_kib_per_launch"] * t["write_scale"]) * 1024
    assert abs(expect - t["traffic_bytes_per_launch"]) <= 1024
    # reported only while the kernel source matches the one the counters measured
    assert bench.measured_traffic() in (None, int(t["traffic_bytes_per_launch"]))
