#!/usr/bin/env python3
"""Throughput benchmark of the exact point-to-point shortest-path path on one MI355X.

Default workload (one step = one batch): the power-law graph R-MAT scale 24
(16,777,216 vertices, edge factor 16, (a, b, c, d) = (0.57, 0.19, 0.19,
0.05), symmetrised, deduplicated, weights uniform in [1, 65535]) with its
256 seeded s-t pairs from the largest connected component, answered as one
BiDS Plain* batch (every query with its own forward and backward search in
the same launches). Three threshold schedules run on the same graph and
pairs in the same run:
  - fixed Delta*-stepping: the i-th threshold is i * Delta (Section 2), with
    Delta chosen by the doubling sweep of the experiments (Section 6.1) on
    128 held-out sample pairs;
  - autotuned: ppsp_tune on the same sample (threshold rule, Delta, hub
    window, launch shape, dense frontiers); this is also the best fixed
    Delta under the threshold rule the learned schedule uses;
  - learned: the step network trained by ppsp_mlp_fit on counterfactual
    replays of 32 of the sample pairs (held out from the 256), with the
    tuned setting as its base; `value` is its queries/s over the timed steps.
Inputs are resident on the GPU (graph in HBM, pairs handed over at the
interface) before timing; every schedule gives the same distances, checked
against each other and, on a sample, against the CPU oracle.

Printed: one JSON line with queries/s (whole job), GTEPS over the arcs the
searches relaxed, the rooflines of the round kernel and of the hub-list
kernel (every 4th round of the timed steps carries HIP events in both
launches, on the library stream) with the dominant one as `roofline`, and
the CPU oracle (binary-heap Dijkstra on the host cores) on a bounded sample.
`--workload` selects the other measured workloads (one JSON line each).
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
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
# the kernels and the engine whose defaults shape their launches
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2506_16488_amd", "csrc", f) for f in ("kernels.hip", "ppsp_dev.h", "engine.hip")]


def kernel_source_hash():
    """Hash of the kernels' sources with comments and blank lines removed
    (a comment edit does not invalidate the counters)."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        src = open(f).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        src = re.sub(r"//[^\n]*", "", src)
        h.update("\n".join(l.rstrip() for l in src.splitlines() if l.strip()).encode())
    return h.hexdigest()[:16]


def measured_traffic(workload, kernel):
    """HBM bytes per launch of `kernel` on `workload` from the committed
    rocprofv3 counter summary, or None when the kernels changed since."""
    try:
        t = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    e = t.get(workload, {}).get(kernel)
    if not e or e.get("kernel_source_hash") != kernel_source_hash():
        return None
    return int(e["traffic_bytes_per_launch"])


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


# Kernel durations: every PROFILE_EVERY-th round of the timed steps carries
# HIP events in its round-kernel and hub-list-kernel launches (a uniform
# sample; timing every launch costs about 2%).
PROFILE_EVERY = 4
BYTES_PER_SCANNED_VERTEX = 24  # row_ptr 8 + own state 8 + frontier entry read/write 8
BYTES_PER_SCANNED_ARC = 24     # arc (neighbour, weight) 8 + neighbour state read-modify-write 16
BYTES_PER_HEAVY_CHUNK = 64     # a hub-list record, written by the round kernel and read by the hub-list kernel
# Scattered accesses: per scanned vertex its own state, its row_ptr pair and
# the first line of its arcs; per relaxed arc the head's state pair; per
# successful relaxation one 64-bit atomic minimum.
LOADS_PER_SCANNED_VERTEX = 3
RANDBENCH_WORDS = 1 << 33      # 64 GiB table, the size of the workloads' search state
RANDBENCH_OPS = 1 << 28


def cpu_threads():
    """Host threads the oracle runs on: every CPU this process may use."""
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def random_access_rates():
    """The device's measured rates of scattered 16-byte loads and 64-bit
    atomics over a 64 GiB table (the probe library's kernel, run now)."""
    from paper_2506_16488_amd import probe
    load_ms = probe.randbench(RANDBENCH_WORDS, RANDBENCH_OPS, 0)
    atom_ms = probe.randbench(RANDBENCH_WORDS, RANDBENCH_OPS, 1)
    return RANDBENCH_OPS / (load_ms * 1e-3), RANDBENCH_OPS / (atom_ms * 1e-3)


def random_access_roofline(rates, loads, atomics, avg_launch_us):
    """Second roofline of a kernel: its scattered loads and atomics per launch
    priced at the device's measured rates; frac = that floor / the launch
    time (atomics counted from successful relaxations, a lower bound)."""
    load_rate, atom_rate = rates
    floor_us = 1e6 * (loads / load_rate + atomics / atom_rate)
    return {
        "bound": "scattered 16-byte loads + 64-bit atomics",
        "loads_per_launch": int(loads),
        "atomics_per_launch": int(atomics),
        "load_rate_gops": round(load_rate / 1e9, 2),
        "atomic_rate_gops": round(atom_rate / 1e9, 2),
        "table_gib": RANDBENCH_WORDS * 8 >> 30,
        "floor_us": round(floor_us, 2),
        "avg_launch_us": round(avg_launch_us, 3),
        "frac": round(floor_us / avg_launch_us, 4) if avg_launch_us > 0 else None,
    }


def hbm_roofline(kernel, alg_bytes_per_launch, avg_launch_s, launches, timed, traffic):
    achieved = alg_bytes_per_launch / avg_launch_s / 1e9 if avg_launch_s > 0 else 0.0
    return {
        "bound": "hbm",
        "kernel": kernel,
        "achieved": round(achieved, 2),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 5),
        "traffic": traffic,
        "traffic_gbs": None if traffic is None or avg_launch_s <= 0 else round(traffic / avg_launch_s / 1e9, 1),
        "avg_launch_us": round(1e6 * avg_launch_s, 3),
        "alg_bytes_per_launch": int(alg_bytes_per_launch),
        "launches": int(launches),
        "timed_launches": int(timed),
    }


def _log(msg):
    print("# " + msg, file=sys.stderr, flush=True)


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def _cpu_baseline(g, sample, label, threads=None):
    """The oracle as it stands, one binary-heap Dijkstra per pair, timed on
    the host threads."""
    import oracle
    threads = threads or cpu_threads()
    a = time.perf_counter()
    exp = oracle.pp_batch(g.n, g.row_ptr, g.col, g.w, sample, nthreads=threads)
    cpu_s = time.perf_counter() - a
    return exp, {"value": round(sample.shape[0] / cpu_s, 3), "unit": "queries/s", "cores": threads, "kind": "oracle",
                 "sample": "%d pairs of %s, one binary-heap Dijkstra per pair (stops at t), %d host threads, %.1f s"
                           % (sample.shape[0], label, threads, cpu_s), "host_cpu": _cpu_model()}


def _line(args, workload, value, ms, dtype="u32", metric="exact s-t queries/sec", **extra):
    out = {"metric": metric, "value": round(value, 2), "unit": "queries/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 3), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": dtype, "data": "synthetic",
           "config": {"workload": workload}}
    out.update(extra)
    print(json.dumps(out), flush=True)


def _agg_stats(G, agg, keys):
    st = G.stats()
    for k in keys:
        agg[k] = agg.get(k, 0) + st[k]
    return st


STAT_KEYS = ("rounds", "entries", "scanned_vertices", "scanned_arcs", "relax_success", "carried", "relax_kernel_ms",
             "relax_launches", "relax_timed", "heavy_kernel_ms", "heavy_arcs", "heavy_chunks", "heavy_success")


def kernel_rooflines(agg, workload, rates=None):
    """Rooflines of the round kernel and the hub-list kernel from the timed
    steps' counters and sampled launch durations; the dominant one (more
    measured time per launch x launches) first."""
    launches = max(1, agg["relax_launches"])
    timed = max(1, agg["relax_timed"])
    k_round_s = agg["relax_kernel_ms"] / 1000.0 / timed
    k_heavy_s = agg["heavy_kernel_ms"] / 1000.0 / timed
    light_arcs = agg["scanned_arcs"] - agg["heavy_arcs"]
    rb = (BYTES_PER_SCANNED_VERTEX * agg["scanned_vertices"] + BYTES_PER_SCANNED_ARC * light_arcs
          + BYTES_PER_HEAVY_CHUNK / 2 * agg["heavy_chunks"]) / launches
    hb = (BYTES_PER_SCANNED_ARC * agg["heavy_arcs"] + BYTES_PER_HEAVY_CHUNK / 2 * agg["heavy_chunks"]) / launches
    out = {"k_round": hbm_roofline("k_round", rb, k_round_s, launches, agg["relax_timed"],
                                   measured_traffic(workload, "k_round"))}
    if agg["heavy_kernel_ms"] > 0:
        out["k_heavy"] = hbm_roofline("k_heavy", hb, k_heavy_s, launches, agg["relax_timed"],
                                      measured_traffic(workload, "k_heavy"))
    if rates is not None:
        heavy_succ = agg["heavy_success"]
        out["k_round"]["random_access"] = random_access_roofline(
            rates, (LOADS_PER_SCANNED_VERTEX * agg["scanned_vertices"] + light_arcs) / launches,
            (agg["relax_success"] - heavy_succ) / launches, 1e6 * k_round_s)
        if "k_heavy" in out:
            out["k_heavy"]["random_access"] = random_access_roofline(
                rates, agg["heavy_arcs"] / launches, heavy_succ / launches, 1e6 * k_heavy_s)
    dom = "k_heavy" if "k_heavy" in out and k_heavy_s > k_round_s else "k_round"
    return dom, out


# ---- the headline: R-MAT scale 24, three schedules -----------------------------

def workload_rmat24(args):
    import numpy as np
    import torch
    import gen
    import paper_2506_16488_amd as P

    torch.cuda.set_device(0)
    t0 = time.time()
    g = gen.workload_graph("rmat24")
    lcc = gen.lcc(g)
    pairs = gen.workload_pairs("rmat24", g, cand=lcc)          # the 256 pairs of every step
    tsample = gen.pairs_uniform(lcc, 128, seed=1104)           # held-out pairs: Delta sweep and autotuner
    sample = tsample[:32]                                      # held-out pairs: training the schedule
    assert not (set(map(tuple, tsample.tolist())) & set(map(tuple, pairs.tolist())))
    G = P.Graph.from_host(g, device=0, reorder=True)
    G.set_option("timeout_ms", 900000)
    _log("graph n=%d m=%d (largest component %d) built+uploaded in %.1fs" % (g.n, g.m, lcc.size, time.time() - t0))
    K = pairs.shape[0]
    sched = {}

    def time_batch(p, reps, **kw):
        """Wall ms of each of `reps` batches of pairs p (after the caller's warm-up)."""
        ms = []
        for _ in range(reps):
            torch.cuda.synchronize()
            a = time.perf_counter()
            d = G.batch_query(p, algo="bids", **kw)
            ms.append(1000.0 * (time.perf_counter() - a))
        return d, ms

    def summary(name, ms, st, **extra):
        m = float(np.median(ms))
        sched[name] = dict({"queries_per_s": round(1000.0 * K / m, 2), "ms_per_batch_median": round(m, 1),
                            "batches_timed": len(ms), "rounds": int(st["rounds"]),
                            "scanned_arcs_per_query": int(st["scanned_arcs"] / K),
                            "gteps": round(st["scanned_arcs"] / (m / 1000.0) / 1e9, 3)}, **extra)
        _log("%s: %.2f q/s (%.0f ms per batch, %d rounds)" % (name, 1000.0 * K / m, m, st["rounds"]))

    # 1. fixed Delta*-stepping (the i-th threshold is i * Delta, Section 2);
    #    Delta by doubling while the sample batch gets faster (Section 6.1)
    G.set_option("theta_mode", 0)
    d0 = max(int(g.w.min()), 256)
    G.batch_query(tsample, algo="bids", delta=d0)              # warm-up: buffers
    sweep, best = [], None
    d = d0
    while d <= (1 << 20):
        _, ms = time_batch(tsample, 1, delta=d)
        sweep.append([d, round(ms[0], 1)])
        if best is None or ms[0] < best[1]:
            best = (d, ms[0])
        else:
            break
        d *= 2
    d_star = best[0]
    G.batch_query(pairs, algo="bids", delta=d_star)
    d_fixed, ms = time_batch(pairs, args.cmp_steps, delta=d_star)
    summary("fixed_delta_star", ms, G.stats(), delta=d_star, theta_rule="i-th threshold = i * Delta",
            doubling_sweep_on_sample_ms=sweep)
    G.set_option("theta_mode", 2)

    # 2. autotuned on the same sample
    tr = G.tune(tsample, algo="bids", batch="plainstar")
    _log("tuned: %s" % {k: (round(v, 2) if isinstance(v, float) else v) for k, v in tr.items()})
    G.batch_query(pairs, algo="bids", sched="autotuned")
    d_auto, ms = time_batch(pairs, args.cmp_steps, sched="autotuned")
    rule = {0: "i * Delta", 1: "end of the smallest key's Delta bucket", 2: "smallest key + Delta - 1"}
    summary("autotuned", ms, G.stats(), delta=int(tr["delta"]), theta_rule=rule.get(int(tr["theta_mode"])),
            heavy_window=int(tr["heavy_window"]), grid_blocks=int(tr["grid_blocks"]), dense_min=int(tr["dense_min"]),
            dense_ring=int(tr["dense_ring"]), trials=int(tr["trials"]))
    assert np.array_equal(d_auto, d_fixed), "schedules disagree"

    # 3. learned: trained on the sample with the tuned setting as its base
    #    (Delta, threshold rule, hub window and launch shape), so the tuned
    #    fixed run above is the same-rule comparison
    G.set_option("theta_mode", int(tr["theta_mode"]))
    G.set_option("heavy_window", int(tr["heavy_window"]))
    G.set_option("grid_blocks", int(tr["grid_blocks"]))
    G.set_option("dense_min", int(tr["dense_min"]))
    G.set_option("dense_ring", int(tr["dense_ring"]))
    dl = int(tr["delta"])
    a = time.perf_counter()
    params, rep = G.mlp_fit(sample, gen.mlp_init(4), algo="bids", epochs=args.epochs, seed=4, delta=dl,
                            labels="counterfactual")
    fit_s = time.perf_counter() - a
    _log("fit in %.1fs: %s" % (fit_s, {k: (round(v, 3) if isinstance(v, float) else v) for k, v in rep.items()}))
    if args.save_schedule:
        # the trained schedule and its base setting, for counter runs of the same batch (--workload profile)
        np.savez(args.save_schedule, params=params, delta=dl, theta_mode=int(tr["theta_mode"]),
                 heavy_window=int(tr["heavy_window"]), grid_blocks=int(tr["grid_blocks"]),
                 dense_min=int(tr["dense_min"]), dense_ring=int(tr["dense_ring"]),
                 plain_fallback=int(rep["plain_fallback"]))

    def step():
        return G.batch_query(pairs, algo="bids", sched="learned", delta=dl)

    for w in range(args.warmup):
        step()
        _log("warmup %d done" % w)
    G.set_option("profile", PROFILE_EVERY)
    agg = {}
    step_ms = []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for k in range(args.steps):
        a = time.perf_counter()
        d_learned = step()
        step_ms.append(1000.0 * (time.perf_counter() - a))
        st = _agg_stats(G, agg, STAT_KEYS)
        _log("step %d: %.1f ms, rounds %d" % (k, step_ms[-1], st["rounds"]))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    G.set_option("profile", 0)
    assert np.array_equal(d_learned, d_auto), "the learned schedule disagrees with the fixed ones"
    steps = args.steps
    qps = K * steps / elapsed
    summary("learned", step_ms, {k: v / steps for k, v in agg.items()}, fit_seconds=round(fit_s, 1),
            fit={k: (round(v, 4) if isinstance(v, float) else v) for k, v in rep.items()})

    rates = None if args.no_randbench else random_access_rates()
    dom, roofs = kernel_rooflines(agg, "rmat24", rates)
    out = {
        "metric": "exact s-t queries/sec, learned schedule (vs fixed Delta*-stepping and autotuned, same run)",
        "value": round(qps, 2),
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": round(1000.0 * elapsed / steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {
            "workload": "R-MAT scale 24 (16,777,216 vertices, %d arcs after symmetrising and deduplication, "
                        "weights U[1,65535]), 256 pairs from the largest component per step, BiDS Plain*, "
                        "learned step schedule" % g.m,
            "queries_per_step": int(K),
        },
        "gteps": round(agg["scanned_arcs"] / elapsed / 1e9, 4),
        "sssp_equivalent_gteps": round(g.m * qps / 1e9, 3),
        "learned_vs_fixed_delta_star": round(qps / sched["fixed_delta_star"]["queries_per_s"], 4),
        "learned_vs_same_rule_fixed": round(qps / sched["autotuned"]["queries_per_s"], 4),
        "batch_ms_p50": round(float(np.percentile(step_ms, 50)), 1),
        "batch_ms_p99": round(float(np.percentile(step_ms, 99)), 1),
        "schedules": sched,
        "roofline": {k: v for k, v in roofs[dom].items() if k != "random_access"},
        "rooflines": roofs,
    }
    if not args.no_cpu:
        threads = cpu_threads()
        n_cpu = min(K, max(args.cpu_sample, threads))
        exp, cb = _cpu_baseline(g, pairs[:n_cpu], "the 256 (the first %d)" % n_cpu, threads)
        assert np.array_equal(exp, d_learned[:n_cpu]), "GPU and oracle disagree on the CPU sample"
        out["cpu_baseline"] = cb
    G.close()
    print(json.dumps(out), flush=True)


# ---- the road-like lattice: 1,000 BiD-A* queries per batch -----------------------

def workload_lattice2048(args):
    """The jittered 2048 x 2048 lattice (4,194,304 vertices, ~17.2M arcs,
    weights ceil(1000 * Euclidean length), fixed-point coordinates) with its
    1,000 seeded uniform pairs as one Plain* BiD-A* batch per step; the graph
    is stored in Morton order of the coordinates (PPSP_REORDER). Pairs and
    distances sit in device memory at the interface (PPSP_DEVICE_IO; the
    library plans the batch on the host, so it stages them through host
    memory inside the timed call). All 1,000 distances of the last step are
    checked against the oracle, and every pair is also answered alone for
    the single-query p50/p99."""
    import numpy as np
    import torch
    import gen
    import oracle
    import paper_2506_16488_amd as P

    torch.cuda.set_device(0)
    t0 = time.time()
    g = gen.workload_graph("lattice2048")
    pairs = gen.workload_pairs("lattice2048", g)
    G = P.Graph.from_host(g, device=0, reorder=True)
    G.set_option("timeout_ms", 300000)
    _log("graph n=%d m=%d built+uploaded in %.1fs" % (g.n, g.m, time.time() - t0))
    pairs_dev = torch.from_numpy(pairs.astype(np.int32)).cuda()
    dist_dev = torch.empty(pairs.shape[0], dtype=torch.int64, device="cuda")
    torch.cuda.synchronize()

    def step():
        G.batch_query_device(pairs_dev, dist_dev, algo=args.algo, batch=args.batch, delta=args.delta)

    for w in range(args.warmup):
        step()
        _log("warmup %d done" % w)
    G.set_option("profile", PROFILE_EVERY)
    agg = {}
    step_ms = []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for k in range(args.steps):
        a = time.perf_counter()
        step()
        step_ms.append(1000.0 * (time.perf_counter() - a))
        st = _agg_stats(G, agg, STAT_KEYS)
        _log("step %d: %.1f ms, rounds %d" % (k, step_ms[-1], st["rounds"]))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    G.set_option("profile", 0)
    dist0 = dist_dev.cpu().numpy().view(np.uint64)
    K, q = args.steps, pairs.shape[0]
    qps = q * K / elapsed

    # every distance of the last step against the oracle (not part of any timing)
    exp = oracle.pp_batch(g.n, g.row_ptr, g.col, g.w, pairs, nthreads=cpu_threads())
    assert np.array_equal(exp, dist0), "GPU and oracle disagree"
    # single-query latency: every pair alone through ppsp_query
    lat = []
    n_lat = q if args.latency_sample < 0 else min(args.latency_sample, q)
    for i in range(n_lat):
        s, t = int(pairs[i, 0]), int(pairs[i, 1])
        a = time.perf_counter()
        dd = G.query(s, t, algo=args.algo, delta=args.delta)
        lat.append(1000.0 * (time.perf_counter() - a))
        assert dd == int(dist0[i]), "single query disagrees with the batch"
    rates = None if args.no_randbench else random_access_rates()
    dom, roofs = kernel_rooflines(agg, "lattice2048", rates)
    out = {
        "metric": "exact s-t queries/sec",
        "value": round(qps, 2), "unit": "queries/s", "n_gpus": 1, "steps": K, "warmup": args.warmup,
        "ms_per_step": round(1000.0 * elapsed / K, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {
            "workload": "road-like jittered lattice 2048x2048 (4,194,304 vertices, %d arcs, w=ceil(1000*len)), "
                        "1,000 uniform s-t pairs per step, %s, %s batch" % (g.m, args.algo, args.batch),
            "queries_per_step": int(q),
            "delta": int(G.get_option("default_delta") if args.delta == 0 else args.delta),
        },
        "ms_per_step_median": round(float(np.median(step_ms)), 3),
        "gteps": round(agg["scanned_arcs"] / elapsed / 1e9, 4),
        "sssp_equivalent_gteps": round(g.m * qps / 1e9, 3),
        "scanned_arcs_per_query": int(agg["scanned_arcs"] / (K * q)),
        "rounds_per_step": int(agg["rounds"] / K),
        "all_distances_checked_against_oracle": int(q),
        "single_query_count": len(lat),
        "single_query_p50_ms": round(float(np.percentile(lat, 50)), 3) if lat else None,
        "single_query_p99_ms": round(float(np.percentile(lat, 99)), 3) if lat else None,
        "roofline": {k: v for k, v in roofs[dom].items() if k != "random_access"},
        "rooflines": roofs,
    }
    if not args.no_cpu:
        threads = cpu_threads()
        n_cpu = min(q, max(args.cpu_sample, threads))
        exp2, cb = _cpu_baseline(g, pairs[:n_cpu], "the 1,000 (the first %d)" % n_cpu, threads)
        assert np.array_equal(exp2, dist0[:n_cpu])
        a = time.perf_counter()
        one = oracle.pp_batch(g.n, g.row_ptr, g.col, g.w, pairs[:4], nthreads=1)
        cb["single_thread_ms_per_query"] = round(1000.0 * (time.perf_counter() - a) / 4, 2)
        assert np.array_equal(one, dist0[:4])
        out["cpu_baseline"] = cb
    G.close()
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="rmat24",
                    choices=["rmat24", "lattice2048", "lattice4096hub", "serve", "ranks", "profile"],
                    help="rmat24: the headline (learned vs fixed schedules); the others are further measured "
                         "workloads; profile: one batch of a fixed setting, for counter runs")
    ap.add_argument("--algo", default="bidastar", help="lattice2048: the search algorithm")
    ap.add_argument("--batch", default="plainstar", help="lattice2048: the batch strategy")
    ap.add_argument("--delta", type=int, default=0, help="lattice2048: Delta (0 = the graph default)")
    ap.add_argument("--cmp-steps", type=int, default=3, help="rmat24: timed batches of each comparison schedule")
    ap.add_argument("--epochs", type=int, default=30, help="rmat24: training epochs of the learned schedule")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-randbench", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=16)
    ap.add_argument("--latency-sample", type=int, default=-1, help="lattice2048: pairs answered alone (-1: all)")
    ap.add_argument("--profile-graph", default="rmat24", help="profile: rmat24 or lattice2048")
    ap.add_argument("--schedule", default=None, help="profile: the schedule file a headline run saved")
    ap.add_argument("--save-schedule", default=None, help="rmat24: save the trained schedule (.npz) here")
    ap.add_argument("--serve-requests", type=int, default=24, help="serve: requests per load level (and of the "
                    "saturation run)")
    ap.add_argument("--serve-budget-gb", type=int, default=160, help="serve: search-state budget (GiB)")
    ap.add_argument("--copy-kernel", action="store_true", help="run the 1 GiB copy used to calibrate counters")
    args = ap.parse_args()
    if args.copy_kernel:
        copy_kernel()
        return
    if args.gpus != 1:
        print("bench.py: one GPU only (queries shard across GPUs with no exchange, so a multi-GPU run "
              "is N independent copies of this one); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    WORKLOADS[args.workload](args)


def workload_profile(args):
    """Batches of one workload's timed step alone, for rocprofv3 counter runs
    (--steps batches): R-MAT 24 under the learned schedule that a headline
    run saved with --save-schedule (--schedule FILE: its network, Delta,
    threshold rule, hub window and launch shape), or the 2048^2 lattice
    BiD-A* batch at the default Delta (--profile-graph lattice2048)."""
    import numpy as np
    import torch
    import gen
    import paper_2506_16488_amd as P
    torch.cuda.set_device(0)
    g = gen.workload_graph(args.profile_graph)
    G = P.Graph.from_host(g, device=0, reorder=True)
    G.set_option("timeout_ms", 900000)
    if args.profile_graph == "rmat24":
        pairs = gen.workload_pairs("rmat24", g, cand=gen.lcc(g))
        s = np.load(args.schedule)
        G.set_option("theta_mode", int(s["theta_mode"]))
        G.set_option("heavy_window", int(s["heavy_window"]))
        G.set_option("grid_blocks", int(s["grid_blocks"]))
        G.set_option("dense_min", int(s["dense_min"]))
        G.set_option("dense_ring", int(s["dense_ring"]))
        G.mlp_load(s["params"])
        sched = "fixed" if int(s["plain_fallback"]) else "learned"
        run = lambda: G.batch_query(pairs, algo="bids", sched=sched, delta=int(s["delta"]))
    else:
        pairs = gen.workload_pairs("lattice2048", g)
        run = lambda: G.batch_query(pairs, algo="bidastar")
    for k in range(max(1, args.steps)):
        run()
        st = G.stats()
        print("profile batch %d: rounds %d, launches %d, arcs %d, hub arcs %d" % (
            k, st["rounds"], st["relax_launches"], st["scanned_arcs"], st["heavy_arcs"]), flush=True)
    G.close()


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


def workload_serve(args):
    """Serving (continuous batching): the 4096 x 4096 lattice (BiD-A*) and
    R-MAT 24 (BiDS, autotuned Delta and threshold rule) resident together in
    one server, both under their learned step schedule (trained by
    ppsp_mlp_fit on held-out sample pairs); requests of log-uniform size in
    [1, 4096] pairs on either graph (50/50); saturation from requests
    submitted at once (the request sequence below), then Poisson arrivals
    offering 50% and 80% of its query rate, both levels with the same
    request sequence (so their latencies compare). The
    first 12 requests of the last level are checked against their own runs
    alone."""
    import numpy as np
    import torch
    import gen
    import oracle
    import paper_2506_16488_amd as P
    torch.cuda.set_device(0)
    t0 = time.time()
    hosts = [gen.workload_graph("lattice4096"), gen.workload_graph("rmat24")]
    lcc = gen.lcc(hosts[1])
    Gs = [P.Graph.from_host(h, reorder=True) for h in hosts]
    for G in Gs:
        G.set_option("timeout_ms", 900000)
    _log("graphs built in %.1fs" % (time.time() - t0))
    rm_sample = gen.pairs_uniform(lcc, 32, seed=1104)
    tr = Gs[1].tune(rm_sample, algo="bids", batch="plainstar")
    Gs[1].set_option("theta_mode", int(tr["theta_mode"]))
    Gs[1].set_option("heavy_window", int(tr["heavy_window"]))
    _log("R-MAT tuned: %s" % {k: tr[k] for k in ("delta", "theta_mode", "heavy_window")})
    # served graphs run sparse frontiers; the tuned step may have been chosen with dense ones,
    # so it and two wider steps are timed again on the sample without them
    sparse_check = []
    for d in (int(tr["delta"]), 2 * int(tr["delta"]), 4 * int(tr["delta"])):
        Gs[1].batch_query(rm_sample, algo="bids", delta=d)
        a = time.perf_counter()
        Gs[1].batch_query(rm_sample, algo="bids", delta=d)
        sparse_check.append([d, round(1000.0 * (time.perf_counter() - a), 1)])
    d_srv = min(sparse_check, key=lambda x: x[1])[0]
    _log("served R-MAT step (sparse frontiers): %d from %s" % (d_srv, sparse_check))
    fits = []
    a = time.perf_counter()
    _, rep0 = Gs[0].mlp_fit(gen.pairs_uniform(hosts[0].n, 32, seed=1103), gen.mlp_init(3), algo="bidastar",
                            epochs=args.epochs, seed=3, labels="counterfactual")
    _log("lattice schedule fitted in %.1fs" % (time.perf_counter() - a))
    _, rep1 = Gs[1].mlp_fit(rm_sample, gen.mlp_init(4), algo="bids", epochs=args.epochs, seed=4,
                            delta=d_srv, labels="counterfactual")
    for rep in (rep0, rep1):
        fits.append({k: rep[k] for k in ("label_hist", "heldout_learned_ms", "heldout_fixed_ms", "plain_fallback")})
    _log("schedules fitted in %.1fs: %s" % (time.perf_counter() - a, fits))
    deltas = [0, d_srv]
    algos = ["bidastar", "bids"]

    def make_requests(k, seed):
        r = np.random.default_rng(seed)
        out = []
        for j in range(k):
            gi = int(r.integers(0, 2))
            size = int(np.clip(np.floor(np.exp(r.uniform(0, np.log(4097)))), 1, 4096))
            cand = None if gi == 0 else lcc
            out.append((gi, gen.pairs_uniform(hosts[gi].n if cand is None else cand, size, seed=seed * 100000 + j)))
        return out

    S = P.Server(Gs, algo=algos, delta=deltas, sched="learned", state_budget_bytes=args.serve_budget_gb << 30)
    out = {"slots": S.stats()["slots"], "fits": fits,
           "tuned_rmat": {k: tr[k] for k in ("delta", "theta_mode", "heavy_window", "dense_min")},
           "served_rmat_delta": d_srv, "sparse_step_check_ms": sparse_check}
    # saturation: everything submitted at once
    level_reqs = make_requests(args.serve_requests, 2)
    reqs = level_reqs
    a = time.perf_counter()
    ids = [S.submit(gi, p) for gi, p in reqs]
    for j, r in enumerate(ids):
        S.wait(r, timeout_ms=1800000)
        _log("saturation: request %d of %d done" % (j + 1, len(ids)))
    sat_s = time.perf_counter() - a
    nq = sum(p.shape[0] for _, p in reqs)
    sat_rps = len(reqs) / sat_s
    _log("saturation: %.3f requests/s, %.1f queries/s" % (sat_rps, nq / sat_s))
    out.update({"saturation_requests": len(reqs), "saturation_requests_per_s": round(sat_rps, 4),
                "saturation_queries_per_s": round(nq / sat_s, 2)})
    rng = np.random.default_rng(105)
    check = None
    # offered load: a fraction of the saturation query rate, in requests of the level's mean size
    mean_pairs = sum(p.shape[0] for _, p in level_reqs) / len(level_reqs)
    for frac in (0.5, 0.8):
        lam = frac * (nq / sat_s) / mean_pairs
        reqs = level_reqs
        gaps = rng.exponential(1.0 / lam, len(reqs))
        a = time.perf_counter()
        t_next = a
        ids = []
        for j, ((gi, p), gap) in enumerate(zip(reqs, gaps)):
            t_next += gap
            while time.perf_counter() < t_next:
                time.sleep(0.001)
            ids.append(S.submit(gi, p))
            if j % 8 == 7:
                _log("load %.0f%%: %d requests submitted" % (100 * frac, j + 1))
        lats, res = [], []
        for j, r in enumerate(ids):
            d, lat = S.wait(r, timeout_ms=1800000)
            lats.append(lat)
            res.append(d)
            _log("load %.0f%%: request %d of %d (%d pairs) done, %.0f ms" % (100 * frac, j + 1, len(ids), d.shape[0], lat))
        wall = time.perf_counter() - a
        lats = np.array(lats)
        q = sum(p.shape[0] for _, p in reqs)
        out["load_%d" % int(frac * 100)] = {
            "offered_requests_per_s": round(lam, 4), "requests": len(reqs), "queries": int(q),
            "mean_request_pairs": round(q / len(reqs), 1),
            "queries_per_s": round(q / wall, 2), "p50_ms": round(float(np.percentile(lats, 50)), 1),
            "p99_ms": round(float(np.percentile(lats, 99)), 1),
            "p50_ms_by_graph": [round(float(np.percentile(lats[[gi == k for gi, _ in reqs]], 50)), 1)
                                if any(gi == k for gi, _ in reqs) else None for k in (0, 1)]}
        _log("load %.0f%%: %s" % (100 * frac, out["load_%d" % int(frac * 100)]))
        check = (reqs, res)
    S.close()
    # requests of the last level equal their runs alone (the same library, learned schedule)
    for j, ((gi, p), d) in enumerate(list(zip(*check))[:12]):
        alone = Gs[gi].batch_query(p, algo=algos[gi], delta=deltas[gi], sched="learned")
        assert np.array_equal(alone, d), "a served request differs from its run alone"
        _log("request %d equals its run alone" % j)
    small = [(gi, p) for gi, p in check[0] if p.shape[0] <= 8][:4]
    for gi, p in small:
        exp = oracle.pp_batch(hosts[gi].n, hosts[gi].row_ptr, hosts[gi].col, hosts[gi].w, p, nthreads=cpu_threads())
        assert np.array_equal(exp, Gs[gi].batch_query(p, algo=algos[gi], delta=deltas[gi]))
    out["checked_against_own_run_alone"] = min(12, len(check[0]))
    for G in Gs:
        G.close()
    _line(args, "serving: lattice 4096x4096 (BiD-A*) + R-MAT 24 (BiDS, autotuned) resident together, learned "
                "schedules, requests of log-uniform 1..4096 pairs on either graph, Poisson arrivals at 50%% and 80%% "
                "of the saturation query rate (%d requests per level)" % args.serve_requests,
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


WORKLOADS = {"rmat24": workload_rmat24, "lattice2048": workload_lattice2048, "lattice4096hub": workload_lattice4096hub,
             "serve": workload_serve, "ranks": workload_ranks, "profile": workload_profile}


if __name__ == "__main__":
    main()
