#!/usr/bin/env python3
"""Throughput benchmark of the exact point-to-point shortest-path path on one MI355X.

Workload (one step): the road-like jittered 2048 x 2048 lattice (4,194,304
vertices, ~17.2M arcs, weights ceil(1000 * Euclidean length), fixed-point
coordinates) with its 1,000 seeded uniform s-t pairs, answered as one batch
(Plain*: every query with its own forward and backward search in the same
launches) with bidirectional A*. Inputs are resident on the GPU before timing.

Printed: one JSON line with queries/s (whole job), GTEPS over the arcs the
searches actually relaxed, the roofline of the dominant kernel (the round
kernel, timed with HIP events on the library's stream), single-query
p50/p99 latency, and the CPU oracle (binary-heap Dijkstra on the host cores)
timed on a bounded sample of the same pairs.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_round_traffic.json")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2506_16488_amd", "csrc", f) for f in ("kernels.hip", "ppsp_dev.h")]


def kernel_source_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per round-kernel launch from the committed rocprofv3 counter
    summary, or None when the kernel source changed since it was taken."""
    try:
        t = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_hash") != kernel_source_hash():
        return None
    return int(t["traffic_bytes_per_launch"])


def copy_kernel():
    """Calibration target for the FETCH_SIZE / WRITE_SIZE counters: three
    device copies of 1 GiB (torch), 1 GiB read + 1 GiB written each."""
    import torch
    torch.cuda.set_device(0)
    x = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print("copied 3 x 1 GiB", flush=True)


BYTES_PER_SCANNED_VERTEX = 24  # row_ptr 8 + own state 8 + frontier entry read/write 8
BYTES_PER_SCANNED_ARC = 24     # arc (neighbour, weight) 8 + neighbour state read-modify-write 16


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--algo", default="bidastar")
    ap.add_argument("--batch", default="plainstar")
    ap.add_argument("--delta", type=int, default=0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=64)
    ap.add_argument("--latency-sample", type=int, default=40)
    ap.add_argument("--copy-kernel", action="store_true", help="run the 1 GiB copy used to calibrate counters")
    args = ap.parse_args()
    if args.copy_kernel:
        copy_kernel()
        return
    if args.gpus != 1:
        print("bench.py: this build measures one GPU only (queries shard across GPUs with no exchange; "
              "see DESIGN.md); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import gen
    import paper_2506_16488_amd as P

    torch.cuda.set_device(0)
    t0 = time.time()
    g = gen.config_graph(2)
    pairs = gen.config_pairs(2, g)
    G = P.Graph.from_host(g, device=0)
    G.set_option("timeout_ms", 300000)
    print("# graph n=%d m=%d built+uploaded in %.1fs" % (g.n, g.m, time.time() - t0), file=sys.stderr, flush=True)
    delta = args.delta

    for w in range(args.warmup):
        G.batch_query(pairs, algo=args.algo, batch=args.batch, delta=delta)
        print("# warmup %d done" % w, file=sys.stderr, flush=True)

    # timed region: K full steps with round-kernel timing on the library stream
    G.set_option("profile", 1)
    agg = {"scanned_vertices": 0, "scanned_arcs": 0, "relax_kernel_ms": 0.0, "relax_launches": 0, "rounds": 0,
           "relax_success": 0, "entries": 0}
    dist0 = None
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for k in range(args.steps):
        d = G.batch_query(pairs, algo=args.algo, batch=args.batch, delta=delta)
        st = G.stats()
        for key in agg:
            agg[key] += st[key]
        if dist0 is None:
            dist0 = d
        print("# step %d: %.1f ms, rounds %d" % (k, st["wall_ms"], st["rounds"]), file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    G.set_option("profile", 0)

    K = args.steps
    q = pairs.shape[0]
    ms_per_step = 1000.0 * elapsed / K
    qps = q * K / elapsed
    gteps = agg["scanned_arcs"] / elapsed / 1e9
    alg_bytes = BYTES_PER_SCANNED_VERTEX * agg["scanned_vertices"] + BYTES_PER_SCANNED_ARC * agg["scanned_arcs"]
    launches = max(1, agg["relax_launches"])
    kern_s = agg["relax_kernel_ms"] / 1000.0
    achieved = alg_bytes / kern_s / 1e9 if kern_s > 0 else 0.0

    # single-query latency (each query alone through ppsp_query)
    lat = []
    for i in range(min(args.latency_sample, q)):
        s, t = int(pairs[i, 0]), int(pairs[i, 1])
        a = time.perf_counter()
        dd = G.query(s, t, algo=args.algo, delta=delta)
        lat.append(1000.0 * (time.perf_counter() - a))
        assert dd == int(dist0[i]), "single query disagrees with the batch"
    lat = np.array(lat)

    out = {
        "metric": "exact s-t queries/sec",
        "value": round(qps, 2),
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {
            "workload": "road-like jittered lattice 2048x2048 (4,194,304 vertices, %d arcs, w=ceil(1000*len)), "
                        "1,000 uniform s-t pairs per step, %s, %s batch" % (g.m, args.algo, args.batch),
            "queries_per_step": int(q),
            "delta": int(G.get_option("default_delta") if delta == 0 else delta),
        },
        "gteps": round(gteps, 4),
        "scanned_arcs_per_query": int(agg["scanned_arcs"] / (K * q)),
        "rounds_per_step": int(agg["rounds"] / K),
        "single_query_p50_ms": round(float(np.percentile(lat, 50)), 3),
        "single_query_p99_ms": round(float(np.percentile(lat, 99)), 3),
        "roofline": {
            "bound": "hbm",
            "kernel": "k_round",
            "achieved": round(achieved, 2),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 5),
            "traffic": measured_traffic(),
            "avg_launch_us": round(1000.0 * agg["relax_kernel_ms"] / launches, 3),
            "alg_bytes_per_launch": int(alg_bytes / launches),
            "launches": int(launches),
        },
    }

    if not args.no_cpu:
        import oracle
        threads = min(16, os.cpu_count() or 1)
        sample = pairs[: args.cpu_sample]
        a = time.perf_counter()
        exp = oracle.pp_batch(g.n, g.row_ptr, g.col, g.w, sample, nthreads=threads)
        cpu_s = time.perf_counter() - a
        assert np.array_equal(exp, dist0[: args.cpu_sample]), "GPU and oracle disagree on the CPU sample"
        out["cpu_baseline"] = {
            "value": round(sample.shape[0] / cpu_s, 3),
            "unit": "queries/s",
            "cores": threads,
            "kind": "oracle",
            "sample": "first %d of the 1,000 pairs, one binary-heap Dijkstra per pair (stops at t), "
                      "%d host threads, %.1f s wall" % (sample.shape[0], threads, cpu_s),
        }
    G.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
