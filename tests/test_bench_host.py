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
    """Every committed counter summary (per workload and kernel) holds the
    scaled FETCH_SIZE + WRITE_SIZE bytes it reports, and is reported only while
    the kernel source matches the one it measured."""
    if not os.path.exists(bench.TRAFFIC_FILE):
        assert bench.measured_traffic("rmat24", "k_round") is None
        return
    t = json.load(open(bench.TRAFFIC_FILE))
    assert t
    for workload, kernels in t.items():
        for kernel, e in kernels.items():
            for key in ("kernel_source_hash", "fetch_kib_per_launch", "write_kib_per_launch", "fetch_scale",
                        "write_scale", "traffic_bytes_per_launch", "command"):
                assert key in e, (workload, kernel, key)
            assert e["traffic_bytes_per_launch"] > 0
            expect = (e["fetch_kib_per_launch"] * e["fetch_scale"] + e["write_kib_per_launch"] * e["write_scale"]) * 1024
            # the stored figures are rounded (0.1 KiB, scales to 4 decimals)
            assert abs(expect - e["traffic_bytes_per_launch"]) <= max(1024, 1e-4 * e["traffic_bytes_per_launch"])
            assert bench.measured_traffic(workload, kernel) in (None, int(e["traffic_bytes_per_launch"]))
    assert bench.measured_traffic("no-such-workload", "k_round") is None


def test_rooflines_from_counters():
    """The per-kernel rooflines: algorithmic bytes per launch from the
    counters (24 B per scanned vertex and per arc, the hub arcs to the hub-list
    kernel), achieved = bytes / sampled launch time, the dominant kernel is
    the one with the longer launches."""
    agg = {"relax_launches": 10, "relax_timed": 5, "relax_kernel_ms": 5.0, "heavy_kernel_ms": 10.0,
           "scanned_vertices": 1000, "scanned_arcs": 10000, "heavy_arcs": 6000, "heavy_chunks": 10,
           "relax_success": 500, "heavy_success": 200}
    dom, r = bench.kernel_rooflines(agg, "none")
    assert dom == "k_heavy"
    kr, kh = r["k_round"], r["k_heavy"]
    assert kr["alg_bytes_per_launch"] == int((24 * 1000 + 24 * 4000 + 32 * 10) / 10)
    assert kh["alg_bytes_per_launch"] == int((24 * 6000 + 32 * 10) / 10)
    assert abs(kr["avg_launch_us"] - 1000.0) < 1e-6 and abs(kh["avg_launch_us"] - 2000.0) < 1e-6
    assert abs(kr["achieved"] - kr["alg_bytes_per_launch"] / 1e-3 / 1e9) < 0.01
    assert kr["frac"] == round(kr["achieved"] / 8000.0, 5)
    ra = bench.random_access_roofline((1e10, 1e9), 3000, 100, 10.0)
    assert abs(ra["floor_us"] - 1e6 * (3000 / 1e10 + 100 / 1e9)) < 0.01
