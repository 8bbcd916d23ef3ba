#!/usr/bin/env python3
"""Throughput benchmark of the exact point-to-point shortest-path path on one MI355X.

Workload (one step): the road-like jittered 2048 x 2048 lattice (4,194,304
vertices, ~17.2M arcs, weights ceil(1000 * Euclidean length), fixed-point
coordinates) with its 1,000 seeded uniform s-t pairs, answered as one batch
(Plain*: every query with its own forward and backward search in the same
launches) with bidirectional A*. The graph is created with PPSP_REORDER (the
device copy in Morton order of the coordinates; ids at the interface are the
caller's). Inputs are resident on the GPU before timing.

Printed: one JSON line with queries/s (whole job), GTEPS over the arcs the
searches actually relaxed, the roofline of the dominant kernel (the round
kernel: every 4th launch of the timed steps carries HIP events, on the library stream), single-query
p50/p99 latency, and the CPU oracle (binary-heap Dijkstra on the host cores)
timed on a bounded sample of the same pairs.
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_round_traffic.json")
# the round kernel and the engine whose defaults shape its launches
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2506_16488_amd", "csrc", f) for f in ("kernels.hip", "ppsp_dev.h", "engine.hip")]


def kernel_source_hash():
    """Hash of the round kernel's sources with comments and blank lines
    removed (a comment edit does not invalidate the counters)."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        src = open(f).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        src = re.sub(r"//[^\n]*", "", src)
        h.update("\n".join(l.rstrip() for l in src.splitlines() if l.strip()).encode())
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


# The round kernel's duration: every PROFILE_EVERY-th launch of the timed steps
# carries HIP events (a uniform sample; timing every launch costs about 2%).
PROFILE_EVERY = 4
BYTES_PER_SCANNED_VERTEX = 24  # row_ptr 8 + own state 8 + frontier entry read/write 8
BYTES_PER_SCANNED_ARC = 24     # arc (neighbour, weight) 8 + neighbour state read-modify-write 16
# Scattered accesses of the round kernel: per scanned vertex its own state,
# its row_ptr pair and the first line of its arcs; per scanned arc the head's
# state pair; per successful relaxation one 64-bit atomic minimum.
LOADS_PER_SCANNED_VERTEX = 3
RANDBENCH_WORDS = 1 << 33      # 64 GiB table, about the size of the workload's search state
RANDBENCH_OPS = 1 << 28


def random_access_roofline(P, agg, launches, avg_launch_us):
    """Second roofline for the round kernel: its scattered loads and atomics
    per launch priced at the device's measured rates for such accesses
    (the probe library's scattered-access kernel, taken now on this GPU). frac = that floor / the launch
    time; atomics are counted from successful relaxations, a lower bound."""
    from paper_2506_16488_amd import probe
    load_ms = probe.randbench(RANDBENCH_WORDS, RANDBENCH_OPS, 0)
    atom_ms = probe.randbench(RANDBENCH_WORDS, RANDBENCH_OPS, 1)
    load_rate = RANDBENCH_OPS / (load_ms * 1e-3)
    atom_rate = RANDBENCH_OPS / (atom_ms * 1e-3)
    loads = (LOADS_PER_SCANNED_VERTEX * agg["scanned_vertices"] + agg["scanned_arcs"]) / launches
    atomics = agg["relax_success"] / launches
    floor_us = 1e6 * (loads / load_rate + atomics / atom_rate)
    return {
        "bound": "scattered 16-byte loads + 64-bit atomics",
        "loads_per_launch": int(loads),
        "atomics_per_launch": int(atomics),
        "load_rate_gops": round(load_rate / 1e9, 2),
        "atomic_rate_gops": round(atom_rate / 1e9, 2),
        "table_gib": RANDBENCH_WORDS * 8 >> 30,
        "floor_us": round(floor_us, 2),
        "avg_launch_us": avg_launch_us,
        "frac": round(floor_us / avg_launch_us, 4) if avg_launch_us > 0 else None,
    }


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
    ap.add_argument("--workload", default="lattice2048", choices=["lattice2048", "lattice4096hub", "rmat24", "serve", "ranks"],
                    help="lattice2048: the headline line; the others are the further measured workloads")
    args = ap.parse_args()
    if args.copy_kernel:
        copy_kernel()
        return
    if args.gpus != 1:
        print("bench.py: one GPU only (queries shard across GPUs with no exchange, so a multi-GPU run "
              "is N independent copies of this one); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.workload != "lattice2048":
        OTHER_WORKLOADS[args.workload](args)
        return

    import numpy as np
    import torch
    import gen
    import paper_2506_16488_amd as P

    torch.cuda.set_device(0)
    t0 = time.time()
    g = gen.workload_graph("lattice2048")
    pairs = gen.workload_pairs("lattice2048", g)
    G = P.Graph.from_host(g, device=0, reorder=True)
    G.set_option("timeout_ms", 300000)
    print("# graph n=%d m=%d built+uploaded in %.1fs" % (g.n, g.m, time.time() - t0), file=sys.stderr, flush=True)
    delta = args.delta
    # pairs and results resident on the GPU (PPSP_DEVICE_IO), used on torch's current stream
    pairs_dev = torch.from_numpy(pairs.astype(np.int32)).cuda()
    dist_dev = torch.empty(pairs.shape[0], dtype=torch.int64, device="cuda")
    torch.cuda.synchronize()

    def step():
        G.batch_query_device(pairs_dev, dist_dev, algo=args.algo, batch=args.batch, delta=delta)

    for w in range(args.warmup):
        step()
        print("# warmup %d done" % w, file=sys.stderr, flush=True)

    # timed region: K full steps with round-kernel timing on the library stream
    G.set_option("profile", PROFILE_EVERY)
    agg = {"scanned_vertices": 0, "scanned_arcs": 0, "relax_kernel_ms": 0.0, "relax_launches": 0, "relax_timed": 0,
           "rounds": 0,
           "relax_success": 0, "entries": 0}
    step_ms = []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for k in range(args.steps):
        a = time.perf_counter()
        step()
        step_ms.append(1000.0 * (time.perf_counter() - a))
        st = G.stats()
        for key in agg:
            agg[key] += st[key]
        print("# step %d: %.1f ms, rounds %d" % (k, step_ms[-1], st["rounds"]), file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    G.set_option("profile", 0)
    dist0 = dist_dev.cpu().numpy().view(np.uint64)

    K = args.steps
    q = pairs.shape[0]
    ms_per_step = 1000.0 * elapsed / K
    qps = q * K / elapsed
    gteps = agg["scanned_arcs"] / elapsed / 1e9
    alg_bytes = BYTES_PER_SCANNED_VERTEX * agg["scanned_vertices"] + BYTES_PER_SCANNED_ARC * agg["scanned_arcs"]
    launches = max(1, agg["relax_launches"])
    avg_launch_s = agg["relax_kernel_ms"] / 1000.0 / max(1, agg["relax_timed"])
    achieved = alg_bytes / launches / avg_launch_s / 1e9 if avg_launch_s > 0 else 0.0

    # single-query latency (each query alone through ppsp_query)
    lat = []
    for i in range(min(args.latency_sample, q)):
        s, t = int(pairs[i, 0]), int(pairs[i, 1])
        a = time.perf_counter()
        dd = G.query(s, t, algo=args.algo, delta=delta)
        lat.append(1000.0 * (time.perf_counter() - a))
        assert dd == int(dist0[i]), "single query disagrees with the batch"
    lat = np.array(lat) if lat else None

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
        "ms_per_step_median": round(float(np.median(step_ms)), 3),
        "gteps": round(gteps, 4),
        "sssp_equivalent_gteps": round(g.m * qps / 1e9, 3),
        "scanned_arcs_per_query": int(agg["scanned_arcs"] / (K * q)),
        "rounds_per_step": int(agg["rounds"] / K),
        "single_query_p50_ms": None if lat is None else round(float(np.percentile(lat, 50)), 3),
        "single_query_p99_ms": None if lat is None else round(float(np.percentile(lat, 99)), 3),
        "roofline": {
            "bound": "hbm",
            "kernel": "k_round",
            "achieved": round(achieved, 2),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 5),
            "traffic": measured_traffic(),
            "traffic_gbs": None if measured_traffic() is None else round(measured_traffic() / avg_launch_s / 1e9, 1),
            "avg_launch_us": round(1e6 * avg_launch_s, 3),
            "alg_bytes_per_launch": int(alg_bytes / launches),
            "launches": int(launches),
            "timed_launches": int(agg["relax_timed"]),
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
        a = time.perf_counter()
        one = oracle.pp_batch(g.n, g.row_ptr, g.col, g.w, pairs[:4], nthreads=1)
        one_ms = 1000.0 * (time.perf_counter() - a) / 4
        assert np.array_equal(one, dist0[:4])
        out["cpu_baseline"] = {
            "value": round(sample.shape[0] / cpu_s, 3),
            "unit": "queries/s",
            "cores": threads,
            "kind": "oracle",
            "sample": "first %d of the 1,000 pairs, one binary-heap Dijkstra per pair (stops at t), "
                      "%d host threads, %.1f s wall" % (sample.shape[0], threads, cpu_s),
            "single_thread_ms_per_query": round(one_ms, 2),
            "host_cpu": _cpu_model(),
        }
    G.close()
    out["random_access"] = random_access_roofline(P, agg, launches, out["roofline"]["avg_launch_us"])
    print(json.dumps(out), flush=True)


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


# ---- further workloads (one JSON line each; not the headline) -----------------

def _timed(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    a = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - a) / steps


def _cpu_baseline(g, sample, label):
    import oracle
    threads = min(16, os.cpu_count() or 1)
    a = time.perf_counter()
    exp = oracle.pp_batch(g.n, g.row_ptr, g.col, g.w, sample, nthreads=threads)
    cpu_s = time.perf_counter() - a
    return exp, {"value": round(sample.shape[0] / cpu_s, 3), "unit": "queries/s", "cores": threads, "kind": "oracle",
                 "sample": "%d pairs of %s, one binary-heap Dijkstra per pair (stops at t), %d host threads, %.1f s"
                           % (sample.shape[0], label, threads, cpu_s)}


def _line(args, workload, value, ms, dtype="u32", **extra):
    out = {"metric": "exact s-t queries/sec", "value": round(value, 2), "unit": "queries/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 3), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": dtype, "data": "synthetic",
           "config": {"workload": workload}}
    out.update(extra)
    print(json.dumps(out), flush=True)


def workload_lattice4096hub(args):
    """4096 x 4096 jittered lattice; batches of 1,024 pairs, half from 32
    hubs (Multi-BiDS shares one search per hub), half uniform."""
    import numpy as np
    import torch
    import gen
    import paper_2506_16488_amd as P
    torch.cuda.set_device(0)
    g = gen.workload_graph("lattice4096")
    G = P.Graph.from_host(g, device=0, reorder=True)
    G.set_option("timeout_ms", 600000)
    batches = [gen.workload_pairs("lattice4096", g, batch=b) for b in range(args.steps + args.warmup)]
    it = iter(batches)
    res = {}
    dist = None
    for algo, batch in [("bids", "multi"), ("bidastar", "plainstar"), ("bids", "plainstar")]:
        n = args.steps if (algo, batch) == ("bids", "multi") else 1
        bb = batches[args.warmup:args.warmup + n]
        G.batch_query(batches[0], algo=algo, batch=batch)
        torch.cuda.synchronize()
        a = time.perf_counter()
        for p in bb:
            d = G.batch_query(p, algo=algo, batch=batch)
        torch.cuda.synchronize()
        t = (time.perf_counter() - a) / n
        st = G.stats()
        res["%s_%s" % (algo, batch)] = {"queries_per_s": round(1024 / t, 2), "ms_per_batch": round(1000 * t, 1),
                                        "searches": st["searches"], "waves": st["waves"], "rounds": st["rounds"]}
        if dist is None:
            dist = (bb[-1], d)
        else:
            assert np.array_equal(G.batch_query(dist[0], algo=algo, batch=batch), dist[1])
        print("# %s %s: %.1f q/s" % (algo, batch, 1024 / t), file=sys.stderr, flush=True)
    best = max(res, key=lambda k: res[k]["queries_per_s"])
    main_ = res[best]
    extra = {"strategies": res, "best_strategy": best}
    if not args.no_cpu:
        exp, cb = _cpu_baseline(g, dist[0][:8], "the last timed batch")
        assert np.array_equal(exp, dist[1][:8])
        extra["cpu_baseline"] = cb
    G.close()
    _line(args, "jittered lattice 4096x4096 (16,777,216 vertices, %d arcs), batches of 1,024 pairs "
                "(512 from 32 hubs, 512 uniform); value = the fastest of Multi-BiDS, Plain* BiD-A* and Plain* BiDS"
                % g.m,
          main_["queries_per_s"], main_["ms_per_batch"], **extra)


def workload_rmat24(args):
    """R-MAT scale 24, edge factor 16, weights U[1, 65535]: 256 pairs from the
    largest component, BiDS Plain*, with the graph's default Delta, the
    autotuned setting and the learned schedule."""
    import numpy as np
    import torch
    import gen
    import paper_2506_16488_amd as P
    torch.cuda.set_device(0)
    g = gen.workload_graph("rmat24")
    lcc = gen.lcc(g)
    pairs = gen.workload_pairs("rmat24", g, cand=lcc)
    G = P.Graph.from_host(g, device=0, reorder=True)
    G.set_option("timeout_ms", 900000)
    print("# graph built: n=%d m=%d" % (g.n, g.m), file=sys.stderr, flush=True)
    res = {}
    t = _timed(lambda: G.batch_query(pairs, algo="bids"), 1, 1)
    res["fixed_default_delta"] = {"queries_per_s": round(len(pairs) / t, 2), "delta": G.get_option("default_delta"),
                                  "scanned_arcs_per_query": int(G.stats()["scanned_arcs"] / len(pairs))}
    print("# fixed: %.2f q/s" % (len(pairs) / t), file=sys.stderr, flush=True)
    print("# tuning on 32 pairs", file=sys.stderr, flush=True)
    tr = G.tune(pairs[:32], algo="bids", batch="plainstar")
    print("# tuned: %s" % tr, file=sys.stderr, flush=True)
    t = _timed(lambda: G.batch_query(pairs, algo="bids", sched="autotuned"), max(1, args.steps), 0)
    res["autotuned"] = {"queries_per_s": round(len(pairs) / t, 2), "tune": {k: (round(v, 3) if isinstance(v, float) else v)
                                                                              for k, v in tr.items()},
                        "scanned_arcs_per_query": int(G.stats()["scanned_arcs"] / len(pairs))}
    d_auto = G.batch_query(pairs, algo="bids", sched="autotuned")
    print("# autotuned: %.2f q/s" % (len(pairs) / t), file=sys.stderr, flush=True)
    train = gen.pairs_uniform(lcc, 16, seed=1104)
    print("# fitting the learned schedule on 16 pairs", file=sys.stderr, flush=True)
    params, rep = G.mlp_fit(train, gen.mlp_init(4), algo="bids", epochs=20, seed=4, delta=int(tr["delta"]))
    t = _timed(lambda: G.batch_query(pairs, algo="bids", sched="learned", delta=int(tr["delta"])), 1, 0)
    assert np.array_equal(G.batch_query(pairs[:32], algo="bids", sched="learned", delta=int(tr["delta"])), d_auto[:32])
    res["learned"] = {"queries_per_s": round(len(pairs) / t, 2), "fit": {k: (round(v, 3) if isinstance(v, float) else v)
                                                                          for k, v in rep.items()}}
    print("# learned: %.2f q/s" % (len(pairs) / t), file=sys.stderr, flush=True)
    extra = {"schedules": res}
    if not args.no_cpu:
        exp, cb = _cpu_baseline(g, pairs[:8], "the 256")
        assert np.array_equal(exp, d_auto[:8])
        extra["cpu_baseline"] = cb
    G.close()
    best = max(v["queries_per_s"] for v in res.values())
    _line(args, "R-MAT scale 24 (16,777,216 vertices, %d arcs, weights U[1,65535]), 256 pairs from the largest "
                "component, BiDS Plain*; value = best of default-Delta, autotuned and learned schedules" % g.m,
          best, 1000.0 * len(pairs) / best, **extra)


def workload_serve(args):
    """Serving: the 4096^2 lattice (BiD-A*) and R-MAT 24 (BiDS) resident in one
    server; requests of log-uniform size in [1, 64] pairs on either graph
    (50/50), Poisson arrivals at 50% and 80% of the measured saturation rate."""
    import numpy as np
    import torch
    import gen
    import paper_2506_16488_amd as P
    torch.cuda.set_device(0)
    hosts = [gen.workload_graph("lattice4096"), gen.workload_graph("rmat24")]
    lcc = gen.lcc(hosts[1])
    print("# graphs built", file=sys.stderr, flush=True)
    Gs = [P.Graph.from_host(h, device=0, reorder=True) for h in hosts]
    # the R-MAT graph runs with its autotuned Delta
    tr = Gs[1].tune(gen.workload_pairs("rmat24", hosts[1], cand=lcc)[:16], algo="bids", batch="plainstar")
    rng = np.random.default_rng(105)

    def make_requests(k, seed):
        r = np.random.default_rng(seed)
        out = []
        for j in range(k):
            gi = int(r.integers(0, 2))
            size = int(np.floor(np.exp(r.uniform(0, np.log(65)))))
            size = max(1, min(64, size))
            cand = None if gi == 0 else lcc
            p = gen.pairs_uniform(hosts[gi].n if cand is None else cand, size, seed=seed * 1000 + j)
            out.append((gi, p))
        return out

    S = P.Server(Gs, algo=["bidastar", "bids"], delta=[0, int(tr["delta"])], state_budget_bytes=48 << 30)
    # saturation: everything submitted at once
    reqs = make_requests(60, 1)
    a = time.perf_counter()
    ids = [S.submit(gi, p) for gi, p in reqs]
    for r in ids:
        S.wait(r, timeout_ms=600000)
    sat_s = time.perf_counter() - a
    nq = sum(p.shape[0] for _, p in reqs)
    sat_rps = len(reqs) / sat_s
    print("# saturation: %.1f requests/s, %.1f queries/s" % (sat_rps, nq / sat_s), file=sys.stderr, flush=True)
    out = {"saturation_requests_per_s": round(sat_rps, 2), "saturation_queries_per_s": round(nq / sat_s, 2),
           "slots": S.stats()["slots"]}
    check = None
    for frac in (0.5, 0.8):
        lam = frac * sat_rps
        reqs = make_requests(120, 2 if frac == 0.5 else 3)
        gaps = rng.exponential(1.0 / lam, len(reqs))
        a = time.perf_counter()
        t_next = a
        ids = []
        for (gi, p), gap in zip(reqs, gaps):
            t_next += gap
            while time.perf_counter() < t_next:
                time.sleep(0.0005)
            ids.append(S.submit(gi, p))
        lats = []
        res = []
        for r in ids:
            d, lat = S.wait(r, timeout_ms=600000)
            lats.append(lat)
            res.append(d)
        wall = time.perf_counter() - a
        lats = np.array(lats)
        q = sum(p.shape[0] for _, p in reqs)
        out["load_%d" % int(frac * 100)] = {"offered_requests_per_s": round(lam, 2), "queries_per_s": round(q / wall, 2),
                                             "p50_ms": round(float(np.percentile(lats, 50)), 2),
                                             "p99_ms": round(float(np.percentile(lats, 99)), 2), "requests": len(reqs)}
        print("# load %.0f%%: p50 %.1f ms p99 %.1f ms" % (100 * frac, np.percentile(lats, 50), np.percentile(lats, 99)),
              file=sys.stderr, flush=True)
        check = (reqs, res)
    S.close()
    # results in the mix equal each request run alone
    for (gi, p), d in list(zip(*check))[:10]:
        alone = Gs[gi].batch_query(p, algo="bidastar" if gi == 0 else "bids",
                                   delta=0 if gi == 0 else int(tr["delta"]))
        assert np.array_equal(alone, d)
    for G in Gs:
        G.close()
    _line(args, "serving: lattice 4096x4096 (BiD-A*) + R-MAT 24 (BiDS, autotuned Delta) resident together, requests "
                "of log-uniform 1..64 pairs on either graph, Poisson arrivals at 50% and 80% of saturation",
          out["load_80"]["queries_per_s"], out["load_80"]["p50_ms"], serving=out)


def workload_ranks(args):
    """The distance-rank study of Section 6 on the 2048 x 2048 lattice: from
    4 seeded sources, targets at distance ranks 10, 20, 40, ... up to the
    farthest vertex (ranks from the library's own single-source distances),
    each query answered alone by ET, A*, BiDS and BiD-A*; per rank the median
    milliseconds over the sources, and the single-source search for scale."""
    import numpy as np
    import torch
    import gen
    import paper_2506_16488_amd as P
    torch.cuda.set_device(0)
    g = gen.workload_graph("lattice2048")
    G = P.Graph.from_host(g, device=0, reorder=True)
    G.set_option("timeout_ms", 300000)
    sources = gen.pairs_uniform(g.n, 4, seed=2026)[:, 0]
    algos = ["et", "astar", "bids", "bidastar"]
    per_rank = {}
    sssp_ms = []
    ladder_pairs = []
    G.query(int(sources[0]), int(sources[1]), algo="bidastar")          # warm-up
    for s in sources.tolist():
        a = time.perf_counter()
        d = G.sssp(s)
        sssp_ms.append(1000 * (time.perf_counter() - a))
        reach = int(np.sum(d != P.INF)) - 1
        ranks = gen.rank_ladder(reach)
        targets = gen.targets_by_rank(d, s, ranks)
        for r, t in zip(ranks, targets.tolist()):
            ladder_pairs.append((s, t, int(d[t])))
            for algo in algos:
                a = time.perf_counter()
                got = G.query(s, t, algo=algo)
                ms = 1000 * (time.perf_counter() - a)
                assert got == d[t], (s, t, algo)
                per_rank.setdefault("farthest" if r == reach else r, {}).setdefault(algo, []).append(ms)
        print("# source %d: %d ranks" % (s, len(ranks)), file=sys.stderr, flush=True)
    by_rank = {str(r): {a: round(float(np.median(v)), 3) for a, v in m.items()} for r, m in per_rank.items()}
    bida = [ms for m in per_rank.values() for ms in m["bidastar"]]
    extra = {"by_rank_median_ms": by_rank, "sssp_median_ms": round(float(np.median(sssp_ms)), 2),
             "queries": len(ladder_pairs) * len(algos)}
    if not args.no_cpu:
        first = [p for p in ladder_pairs if p[0] == int(sources[0])]
        sample = np.array([[s, t] for s, t, _ in first], np.uint32)
        exp, cb = _cpu_baseline(g, sample, "the first source's whole ladder (ranks 10 to the farthest vertex)")
        assert exp.tolist() == [dd for _, _, dd in first]
        extra["cpu_baseline"] = cb
    G.close()
    mean_ms = float(np.mean(bida))
    _line(args, "distance-rank ladder on the jittered 2048x2048 lattice (4 sources, targets at ranks 10, 20, 40, ... "
                "to the farthest vertex), single queries; value = BiD-A* queries/s over the ladder",
          1000.0 / mean_ms, mean_ms, **extra)


OTHER_WORKLOADS = {"lattice4096hub": workload_lattice4096hub, "rmat24": workload_rmat24, "serve": workload_serve,
                   "ranks": workload_ranks}


if __name__ == "__main__":
    main()
