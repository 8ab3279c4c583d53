#!/usr/bin/env python3
"""Benchmark of the IMM hot path on one MI355X.

A step is one full IMM run (all sampling rounds with fused counting, pool
compaction, inverted index, greedy selection, theta schedule; the graph is
resident in HBM before timing starts). The default workload is the
LiveJournal-shaped one: directed Chung-Lu graph (degree exponent 2.0,
n = 4.8 M, m = 69 M), LT model with per-column uniform in-weights normalised
to one as 32-bit cumulative tables, k = 50, eps = 0.13, ell = 1, Philox seed
42 (`--workload youtube_ic` runs the Youtube-shaped IC workload instead).
Inputs are synthetic (seeded generator), standing in for the paper's SNAP
graphs.

Prints one JSON line: whole-run RRR sets/s as `value`, time-to-seeds as
ms_per_step, the roofline figure of the dominant sampling kernel (its
algorithmic bytes per launch over its mean launch time, measured with HIP
events on the stream it runs on), a steady-state sampling figure on the same
graph (outside the timed steps), and the CPU oracle's time to seeds on the
same workload.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time
from pathlib import Path

ROOT = Path(__file__).resolve().parent
sys.path.insert(0, str(ROOT))

HBM_PEAK_GBPS = 8000.0  # MI355X HBM3E
# 32-bit VALU: 256 CUs x 4 SIMDs x 16 lanes at 2.4 GHz, in tera lane-ops/s
ALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
# VALU instructions of one Philox4x32-10 call in the gfx950 code (20 64-bit
# multiply-adds, 40 xor/add), each one lane-op per lane
PHILOX_OPS = 60

# HBM bytes per launch measured with rocprofv3 --pmc (FETCH_SIZE x 2.0 +
# WRITE_SIZE x 1.0, scaled by the 1 GiB copy calibration), for the kernel
# and workload named (an IMM run, or "<workload>:sample<count>" for a
# steady-state sampling run of that many ids), as recorded in profiles/; a
# kernel changed since its counters were taken has no entry.
MEASURED_TRAFFIC = {
    ("lj_lt", "lt_small_kernel"): 4.200e9,
    ("lj_lt:sample16777216", "lt_small_kernel"): 292.52e9,
    ("youtube_ic", "ic_large_kernel"): 8.162e9,
    ("youtube_ic:sample16777216", "ic_large_kernel"): 63.37e9,
}


WORKLOAD_TEXT = {
    "lj_lt": "LT, directed Chung-Lu gamma=2.0 (LiveJournal-shaped)",
    "youtube_ic": "IC p=0.01, directed Chung-Lu gamma=2.1 (Youtube-shaped)",
}


def algorithmic_bytes(model: str, sets: int, entries: int, edges: int, live: int) -> int:
    """Bytes the sampling method must move, per unit of work:

    IC, per sample: 8 B column offsets and 8 B of (source, threshold) per
    in-edge examined of every member, 4 B pool write and 8 B count
    read-modify-write per member, 4 B set size:
    20 B x members + 8 B x coins + 4 B x sets.
    LT, per walk step: 8 B column offsets, 4 B per cumulative-table entry
    probed, 4 B source; per member 12 B (pool write, count):
    12 B x steps + 4 B x probes + 12 B x members."""
    if model == "ic":
        return 20 * entries + 8 * edges + 4 * sets
    return 12 * edges + 4 * live + 12 * entries


def kernel_table(model: str, stats: list) -> dict:
    """Per sampling kernel: name, launches, summed HIP-event time and the
    algorithmic bytes of the sets it finished, over a list of stats dicts."""
    def tot(key):
        return sum(x[key] for x in stats)

    main = (tot("main_sets"), tot("main_entries"), tot("main_edges"), tot("main_live"))
    lane = (tot("lane_sets"), tot("lane_sets"), tot("lane_edges"), 0)
    big = (tot("sets") - main[0] - lane[0], tot("entries") - main[1] - lane[1],
           tot("edges") - main[2] - lane[2], tot("live") - main[3])
    ic = model == "ic"

    def philox_ops(edges):
        # IC: one call per aligned group of four coins (at least edges / 4);
        # LT: one call per walk step
        return (edges / 4.0 if ic else float(edges)) * PHILOX_OPS

    out = {
        "main": dict(name="ic_bfs_kernel" if ic else "lt_small_kernel", ms=tot("ms_sample_main"),
                     launches=tot("main_launches"), bytes=algorithmic_bytes(model, *main),
                     ops=philox_ops(main[2])),
        "large": dict(name="ic_large_kernel" if ic else "lt_large_kernel",
                      ms=tot("ms_sample_big"), launches=tot("big_launches"),
                      bytes=algorithmic_bytes(model, *big), ops=philox_ops(big[2])),
    }
    if ic:
        out["lane"] = dict(name="ic_lane_kernel", ms=tot("ms_sample_lane"),
                           launches=tot("lane_launches"), bytes=algorithmic_bytes(model, *lane),
                           ops=philox_ops(lane[2]))
    return out


def roofline_of(kernels: dict, workload: str) -> dict:
    """Roofline entry of the kernel with the most time among those that
    finished sets (a launch over an empty list only costs its launch). Per
    launch: its algorithmic bytes and its Philox lane-ops over its mean launch
    duration; the bound is whichever roof (HBM or 32-bit ALU) it is nearer
    to."""
    working = [k for k in kernels.values() if k["bytes"] > 0] or list(kernels.values())
    dom = max(working, key=lambda k: k["ms"])
    launches = max(dom["launches"], 1)
    avg_ms = dom["ms"] / launches
    per_launch = dom["bytes"] / launches
    ops_launch = dom["ops"] / launches
    gbps = per_launch / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else 0.0
    tops = ops_launch / (avg_ms * 1e-3) / 1e12 if avg_ms > 0 else 0.0
    hbm = {"achieved": gbps, "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": gbps / HBM_PEAK_GBPS}
    alu = {"achieved": tops, "peak": ALU_PEAK_TOPS, "unit": "TOP/s", "frac": tops / ALU_PEAK_TOPS}
    near, other, bound = (alu, hbm, "alu") if alu["frac"] > hbm["frac"] else (hbm, alu, "hbm")
    out = {"kernel": dom["name"], "bound": bound, **near,
           "traffic": MEASURED_TRAFFIC.get((workload, dom["name"])),
           "avg_launch_ms": avg_ms, "bytes_per_launch": per_launch,
           "philox_ops_per_launch": ops_launch,
           ("hbm" if bound == "alu" else "alu"): other}
    return out


def kernel_summary(kernels: dict) -> dict:
    return {k: {"name": v["name"], "launches": v["launches"],
                "avg_ms": v["ms"] / max(v["launches"], 1),
                "GBps": (v["bytes"] / (v["ms"] * 1e-3) / 1e9) if v["ms"] > 0 else None}
            for k, v in kernels.items()}


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(g, spec, reps: int):
    """The oracle's whole IMM run (same graph, k, eps, ell, seed) timed on the
    host: the median of `reps` runs on up to 16 threads (OpenMP over sample
    ids, atomic counts), and one single-thread run. Value: its RRR sets per
    second of time to seeds."""
    import statistics

    import oracle

    threads = max(1, min(16, os.cpu_count() or 1))
    times, o = [], None
    for _ in range(max(1, reps)):
        t0 = time.perf_counter()
        o = oracle.imm(g, spec["k"], spec["eps"], spec["ell"], spec["seed"], threads=threads)
        times.append(time.perf_counter() - t0)
    t_med = statistics.median(times)
    t0 = time.perf_counter()
    o1 = oracle.imm(g, spec["k"], spec["eps"], spec["ell"], spec["seed"], threads=1)
    t_one = time.perf_counter() - t0
    assert list(o1["seeds"]) == list(o["seeds"]) and o1["theta"] == o["theta"]
    return {"value": o["theta"] / t_med, "unit": "RRR sets/s", "cores": threads, "kind": "oracle",
            "sample": f"the whole oracle IMM run (theta {o['theta']}, {o['rounds']} rounds, "
                      f"k={spec['k']}, eps={spec['eps']}, seed {spec['seed']}): median of "
                      f"{len(times)} runs on {threads} threads, time to seeds "
                      f"{t_med * 1e3:.0f} ms; one run on 1 thread {t_one * 1e3:.0f} ms",
            "time_to_seeds_ms": t_med * 1e3, "time_to_seeds_ms_1thread": t_one * 1e3,
            "host_cpus": os.cpu_count(), "cpu_model": _cpu_model()}


def steady_state(imm, g, dg, spec, count, reps, stream, workload):
    """Steady-state Generate_RRRsets: `reps` imm_sample calls of `count` ids
    (kernel times from HIP events); sets/s, walk steps or coins per second,
    and the roofline entry of the dominant sampling kernel."""
    pools = []
    for _ in range(reps):
        p = imm.imm_sample(dg, spec["seed"], 0, count, flags=imm.IMM_TIMING, stream=stream)
        pools.append(p.stats)
        p.close()
    st = pools[-1]
    samp_ms = sum(x["ms_sample"] for x in pools) / len(pools)
    nbytes = algorithmic_bytes(g.model, st["sets"], st["entries"], st["edges"], st["live"])
    kernels = kernel_table(g.model, pools)
    return {"ids": count, "calls": reps, "sets_per_s": st["sets"] / (samp_ms * 1e-3),
            "sampling_ms": samp_ms, "sampling_GBps": nbytes / (samp_ms * 1e-3) / 1e9,
            "edges_per_s": st["edges"] / (samp_ms * 1e-3), "entries": st["entries"],
            "edges": st["edges"], "probes": st["live"], "deferred": st["deferred"],
            "kernels": kernel_summary(kernels),
            "roofline": roofline_of(kernels, f"{workload}:sample{count}")}


def sample_mode(args, imm, g, dg, spec, stream, torch):
    """Steady-state Generate_RRRsets throughput: one imm_sample call of
    args.sample_count ids per step (kernel times from HIP events)."""
    for _ in range(args.warmup):
        imm.imm_sample(dg, spec["seed"], 0, args.sample_count, flags=imm.IMM_TIMING,
                       stream=stream).close()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ss = steady_state(imm, g, dg, spec, args.sample_count, args.steps, stream, args.workload)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    print(json.dumps({
        "metric": "RRR sets/s (steady-state sampling)", "value": ss["sets_per_s"],
        "unit": "RRR sets/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "strong", "vs_baseline": None,
        "dtype": "u32", "data": "synthetic",
        "config": {"workload": f"{args.workload}: imm_sample of {args.sample_count} ids",
                   "seed": spec["seed"]},
        **{k: v for k, v in ss.items() if k not in ("sets_per_s",)},
    }))


def counter_update_mode(args, imm, torch):
    """Selection time of a whole IMM run under each counter update of the
    greedy (Section IV-C's adaptive update against decrement-only and
    recount-only), on each named workload; the seeds must not change."""
    import statistics

    import synth
    modes = {"adaptive": 0, "decrement": imm.IMM_UPDATE_DECREMENT,
             "recount": imm.IMM_UPDATE_RECOUNT}
    stream = torch.cuda.current_stream()
    out = {}
    for name in args.counter_update.split(","):
        spec = synth.WORKLOADS[name]
        g = synth.make_graph(name)
        dg = imm.graph_from(g, stream=stream)
        torch.cuda.synchronize()
        row, seeds = {}, None
        for mode, fl in modes.items():
            runs = []
            for i in range(args.warmup + args.steps):
                r = imm.imm_run(dg, spec["k"], spec["eps"], spec["ell"], spec["seed"],
                                flags=imm.IMM_TIMING | fl, stream=stream)
                if i >= args.warmup:
                    runs.append(r)
            if seeds is None:
                seeds = list(runs[0].seeds)
            assert all(list(r.seeds) == seeds for r in runs), f"{name}: {mode} changed seeds"
            row[mode] = {"select_ms": statistics.median(r.stats["ms_select"] for r in runs),
                         "total_ms": statistics.median(r.stats["ms_total"] for r in runs)}
        row["speedup_vs_decrement"] = row["decrement"]["select_ms"] / row["adaptive"]["select_ms"]
        row["speedup_vs_recount"] = row["recount"]["select_ms"] / row["adaptive"]["select_ms"]
        out[name] = row
        dg.close()
        print(f"[bench] counter update {name} done", file=sys.stderr, flush=True)
    print(json.dumps({"metric": "IMM selection time by counter update (median ms)",
                      "steps": args.steps, "warmup": args.warmup, "workloads": out}))


def dense_compare_mode(args, imm, torch):
    """The adaptive set representation against list-only sets on one
    workload: time to seeds (median of the timed runs), device memory and
    the number of bitmap sets; the seeds must not change. A list-only run
    that does not fit the budget reports its error instead."""
    import statistics

    import synth
    name = args.dense_compare
    spec = synth.WORKLOADS[name]
    g = synth.make_graph(name)
    stream = torch.cuda.current_stream()
    dg = imm.graph_from(g, stream=stream)
    torch.cuda.synchronize()
    out, seeds = {}, None
    for label, fl in (("bitmaps", 0), ("lists", imm.IMM_LIST_SETS)):
        runs, err = [], None
        try:
            for i in range(args.warmup + args.steps):
                t0 = time.perf_counter()
                r = imm.imm_run(dg, spec["k"], spec["eps"], spec["ell"], spec["seed"],
                                flags=imm.IMM_TIMING | fl, stream=stream,
                                max_device_bytes=args.dense_budget << 30)
                torch.cuda.synchronize()
                if i >= args.warmup:
                    runs.append((time.perf_counter() - t0, r))
                print(f"[bench] {label} run {i + 1} done", file=sys.stderr, flush=True)
        except imm.ImmError as e:
            err = str(e)
        if err or not runs:
            out[label] = {"error": err}
            continue
        r = runs[-1][1]
        if seeds is None:
            seeds = list(r.seeds)
        assert list(r.seeds) == seeds, f"{label}: seeds changed"
        out[label] = {"time_to_seeds_ms": statistics.median(t for t, _ in runs) * 1e3,
                      "phase_ms": {k: r.stats[f"ms_{k}"] for k in
                                   ("sample", "compact", "index", "select")},
                      "theta": r.theta, "dense_sets": r.stats["dense_sets"],
                      "entries": r.stats["entries"], "device_GB": r.stats["device_bytes"] / 1e9}
    print(json.dumps({"metric": "IMM time to seeds, bitmap vs list sets", "workload": name,
                      "n": g.n, "m": g.m, "steps": args.steps, "warmup": args.warmup,
                      "budget_GiB": args.dense_budget, **out}))


def _gen_instance(arg):
    import synth
    i, s = arg
    return synth.make_graph(f"batch{i}", gen=s["gen"], model=s["model"], enc=s["enc"],
                            gseed=s["gseed"])


def make_batch_graphs(count: int):
    """The multi-instance workload's graphs, generated in worker processes
    (before this process touches the GPU)."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor

    import synth
    insts = synth.batch_instances(count)
    workers = max(1, min(8, os.cpu_count() or 1))
    with ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("fork")) as ex:
        graphs = list(ex.map(_gen_instance, enumerate(insts)))
    return insts, graphs


def batch_mode(args, imm, insts, graphs, stream, torch):
    """Aggregate IMM queries/s of the multi-instance workload: all instances
    in one imm_run_batch call per step, against the same instances run one
    at a time with imm_run on the same GPU."""
    if args.graph_select:
        stream = torch.cuda.Stream()  # a capturable stream (default priority)
    dgs = [imm.graph_from(g, stream=stream) for g in graphs]
    torch.cuda.synchronize()
    fl = imm.IMM_GRAPH_SELECT if args.graph_select else 0
    qs = [(d, dict(k=s["k"], epsilon=s["eps"], ell=s["ell"], seed=s["seed"], flags=fl))
          for d, s in zip(dgs, insts)]

    def batched():
        return imm.imm_run_batch(qs, stream=stream)

    def one_by_one():
        return [imm.imm_run(d, q["k"], q["epsilon"], q["ell"], q["seed"], stream=stream)
                for d, q in qs]

    for _ in range(args.warmup):
        batched()
        one_by_one()
    print("[bench] batch warmup done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        rb = batched()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    print("[bench] batched steps done", file=sys.stderr, flush=True)
    for _ in range(args.steps):
        rs = one_by_one()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    print("[bench] one-at-a-time steps done", file=sys.stderr, flush=True)
    for a, b in zip(rb, rs):
        assert a.theta == b.theta and list(a.seeds) == list(b.seeds), "batched != alone"
    nq = len(qs)
    ms_b = (t1 - t0) * 1e3 / args.steps
    ms_s = (t2 - t1) * 1e3 / args.steps
    sets = sum(r.stats["sets"] for r in rb)
    print(json.dumps({
        "metric": "IMM queries/s (batched)", "value": nq / (ms_b * 1e-3), "unit": "queries/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_b,
        "higher_is_better": True, "scaling": "strong", "vs_baseline": None, "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": f"{nq} IC instances: weighted-cascade R-MAT, scale U{{12..20}}, "
                               f"degree U{{4..32}}, k in {{5,10,25,50}}, eps in {{0.5,0.3,0.13}}",
                   "parallelism": "single GPU"},
        "one_at_a_time_queries_per_s": nq / (ms_s * 1e-3),
        "one_at_a_time_ms": ms_s,
        "speedup": ms_s / ms_b,
        "sets_per_s": sets / (ms_b * 1e-3),
        "theta_range": [min(r.theta for r in rb), max(r.theta for r in rb)],
        "graph_select": bool(args.graph_select),
        "select_graphs": sum(r.stats["select_graphs"] for r in rb),
        "select_captures": sum(r.stats["select_captures"] for r in rb),
    }))


def _gen_named(name):
    import synth
    return synth.make_graph(name)


def make_named_graphs(names):
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor
    with ProcessPoolExecutor(max_workers=len(names), mp_context=mp.get_context("fork")) as ex:
        return dict(zip(names, ex.map(_gen_named, names)))


def serve_mode(args, imm, hgraphs, stream, torch):
    """A Poisson stream of queries (the served workload) through the query
    server, against the same stream answered one query at a time, in
    arrival order, with imm_run. Latency is submission to completion."""
    import threading

    import numpy as np

    import synth
    qs = synth.served_queries(args.serve, rate=args.rate)
    dgs = {nm: imm.graph_from(g, stream=stream) for nm, g in hgraphs.items()}
    torch.cuda.synchronize()
    # warm-up: tune every graph and fill its workspace cache
    for nm, dg in dgs.items():
        for _ in range(max(1, args.warmup)):
            imm.imm_run(dg, 50, 0.13, 1.0, 1, stream=stream)
    torch.cuda.synchronize()
    print("[bench] served warmup done", file=sys.stderr, flush=True)

    if args.saturate:
        # every query is queued at t = 0
        qs = [dict(q, t=0.0) for q in qs]
    srv = imm.Server(budget_bytes=args.serve_budget << 30, max_slots=args.serve_slots)
    tickets = [None] * len(qs)

    def submitter(t0):
        for i, q in enumerate(qs):
            dt = t0 + q["t"] - time.perf_counter()
            if dt > 0:
                time.sleep(dt)
            tickets[i] = srv.submit(dgs[q["graph"]], k=q["k"], epsilon=q["eps"], ell=q["ell"],
                                    seed=q["seed"],
                                    flags=imm.IMM_GRAPH_SELECT if args.graph_select else 0)

    t0 = time.perf_counter()
    th = threading.Thread(target=submitter, args=(t0,))
    th.start()
    th.join()
    res = [srv.poll(t) for t in tickets]
    t_end = time.perf_counter()
    srv.close()
    lat = np.array([r.stats["ms_total"] for r in res])
    served_qps = len(qs) / (t_end - t0)
    print("[bench] served run done", file=sys.stderr, flush=True)

    # the same arrivals answered one at a time on the plain path
    lat1 = []
    t0 = time.perf_counter()
    seq = []
    for q in qs:
        now = time.perf_counter() - t0
        if now < q["t"]:
            time.sleep(q["t"] - now)
        r = imm.imm_run(dgs[q["graph"]], q["k"], q["eps"], q["ell"], q["seed"], stream=stream)
        lat1.append((time.perf_counter() - t0 - q["t"]) * 1e3)
        seq.append(r)
    t_end1 = time.perf_counter()
    one_qps = len(qs) / (t_end1 - t0)
    for a, b in zip(res, seq):
        assert a.theta == b.theta and list(a.seeds) == list(b.seeds), "served != alone"
    lat1 = np.array(lat1)
    print("[bench] one-at-a-time run done", file=sys.stderr, flush=True)
    print(json.dumps({
        "metric": "IMM queries/s (served, " + ("all queued at t=0" if args.saturate
                                               else "Poisson arrivals") + ")",
        "value": served_qps,
        "unit": "queries/s", "n_gpus": 1, "steps": len(qs), "warmup": args.warmup,
        "ms_per_step": float(np.mean(lat)), "higher_is_better": True, "scaling": "strong",
        "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": f"{len(qs)} queries "
                               + ("queued at once" if args.saturate else f"at {args.rate}/s")
                               + " over rmat18_wc (IC), youtube_ic (IC) and orkut_lt (LT); "
                               "k in {10,50,100}, eps in {0.5,0.13}",
                   "max_slots": args.serve_slots, "budget_GiB": args.serve_budget,
                   "parallelism": "single GPU"},
        "graph_select": bool(args.graph_select),
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                       "mean": float(np.mean(lat))},
        "one_at_a_time": {"queries_per_s": one_qps,
                          "latency_ms": {"p50": float(np.percentile(lat1, 50)),
                                         "p99": float(np.percentile(lat1, 99)),
                                         "mean": float(np.mean(lat1))}},
    }))


def copy_calibration(torch):
    """A plain device-to-device copy of 1 GiB, three times: the reference
    that scales the HBM byte counters (FETCH_SIZE, WRITE_SIZE) of a profile
    run, since a copy moves exactly its size in each direction."""
    n = 1 << 30
    src = torch.empty(n, dtype=torch.uint8, device="cuda")
    dst = torch.empty(n, dtype=torch.uint8, device="cuda")
    src.fill_(1)
    torch.cuda.synchronize()
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": n, "copies": 3, "kib_per_copy": n / 1024}))


def chase_probe():
    """Dependent random 64-byte row reads, the LT walk's memory pattern
    without its arithmetic (libimm_probe.so): chains of reads through a table
    of 69 M rows (4.4 GB, the LiveJournal-shaped window table's size) or 2 M
    rows (128 MB, inside the Infinity Cache), with 2 to 8 waves of 16
    chains per SIMD, and with one random count atomic per step (counters of
    a 4.8 M-vertex graph) or none. 2000 steps per chain; chain steps per
    second from HIP events around the kernel."""
    import ctypes as C

    lib = C.CDLL(str(ROOT / "paper_2411_09473_amd" / "libimm_probe.so"))
    lib.imm_probe_chase.restype = C.c_int
    lib.imm_probe_chase.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_int,
                                    C.c_uint32, C.POINTER(C.c_double), C.POINTER(C.c_uint64)]
    out = []
    for rows, waves, count in ((69_000_000, 2, 0), (69_000_000, 4, 0), (69_000_000, 5, 0),
                               (69_000_000, 8, 0), (69_000_000, 5, 1), (69_000_000, 8, 1),
                               (2_000_000, 5, 0), (2_000_000, 5, 1)):
        wg = waves  # four-wave workgroups per CU: one wave per SIMD each
        lds = min(64 * 1024, (160 * 1024) // wg // 256 * 256)
        ms, steps = C.c_double(), C.c_uint64()
        rc = lib.imm_probe_chase(rows, wg, lds, 2000, count, 4_800_000, C.byref(ms), C.byref(steps))
        if rc != 0:
            raise RuntimeError(f"imm_probe_chase failed ({rc})")
        out.append({"table_GB": rows * 64 / 1e9, "waves_per_simd": waves,
                    "chains": steps.value // 2000, "count_atomic": bool(count), "ms": ms.value,
                    "G_steps_per_s": steps.value / (ms.value * 1e-3) / 1e9,
                    "row_GBps": steps.value * 64 / (ms.value * 1e-3) / 1e9})
        print(f"[bench] chase {out[-1]}", file=sys.stderr, flush=True)
    print(json.dumps({"metric": "dependent random 64-byte row reads (chase probe)",
                      "steps_per_chain": 2000, "runs": out}))


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="lj_lt")
    ap.add_argument("--cpu-reps", type=int, default=3,
                    help="oracle runs on the host cores (median); plus one single-thread run")
    ap.add_argument("--steady-ids", type=int, default=1 << 24,
                    help="ids of the steady-state sampling call reported beside the timed "
                         "steps (0: none)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--sample-count", type=int, default=0,
                    help="steady-state sampling mode: each step generates this many "
                         "RRR sets with imm_sample (no selection)")
    ap.add_argument("--batch", type=int, default=0,
                    help="multi-instance mode: this many IMM instances per step, "
                         "batched, against the same run one at a time")
    ap.add_argument("--no-graph-select", dest="graph_select", action="store_false",
                    help="batch and served modes: launch the seed steps directly instead of "
                         "as captured hipGraphs (IMM_GRAPH_SELECT)")
    ap.add_argument("--serve", type=int, default=0,
                    help="served mode: this many Poisson-arrival queries through the "
                         "query server, against the same stream one at a time")
    ap.add_argument("--rate", type=float, default=50.0, help="served mode: arrivals per second")
    ap.add_argument("--saturate", action="store_true",
                    help="served mode: queue every query at t=0 (aggregate throughput) "
                         "instead of Poisson arrivals")
    ap.add_argument("--dense-compare", default="",
                    help="a workload: time to seeds with dense sets as bitmaps against "
                         "every set as a list (IMM_LIST_SETS)")
    ap.add_argument("--dense-budget", type=int, default=240,
                    help="dense-compare mode: device memory budget in GiB per run")
    ap.add_argument("--counter-update", default="",
                    help="comma-separated workloads: selection time of an IMM run under "
                         "each counter update (adaptive, decrement-only, recount-only)")
    ap.add_argument("--serve-slots", type=int, default=8, help="served mode: concurrent queries")
    ap.add_argument("--serve-budget", type=int, default=192,
                    help="served mode: device memory budget in GiB")
    ap.add_argument("--chase-probe", action="store_true",
                    help="only run the random-read chase probe (the LT walk's memory pattern "
                         "without its arithmetic)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run the 1 GiB device copy that calibrates HBM byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported: the "
              "library has no multi-GPU path (sampling would shard by sample-id range, "
              "with one reduction of the counts per round)", file=sys.stderr)
        sys.exit(2)

    batch = None
    served = None
    if args.serve:
        served = make_named_graphs(["rmat18_wc", "youtube_ic", "orkut_lt"])
        print("[bench] served graphs ready", file=sys.stderr, flush=True)
    if args.batch:
        batch = make_batch_graphs(args.batch)
        print(f"[bench] {args.batch} batch graphs ready", file=sys.stderr, flush=True)

    import torch

    import paper_2411_09473_amd as imm
    import synth

    torch.cuda.set_device(0)
    if args.copy_calibration:
        return copy_calibration(torch)
    if args.chase_probe:
        return chase_probe()
    if args.counter_update:
        return counter_update_mode(args, imm, torch)
    if args.dense_compare:
        return dense_compare_mode(args, imm, torch)
    if served is not None:
        return serve_mode(args, imm, served, torch.cuda.current_stream(), torch)
    if batch is not None:
        return batch_mode(args, imm, batch[0], batch[1], torch.cuda.current_stream(), torch)
    spec = synth.WORKLOADS[args.workload]
    g = synth.make_graph(args.workload)
    stream = torch.cuda.current_stream()
    dg = imm.graph_from(g, stream=stream)
    torch.cuda.synchronize()

    if args.sample_count:
        return sample_mode(args, imm, g, dg, spec, stream, torch)

    def step():
        return imm.imm_run(dg, spec["k"], spec["eps"], spec["ell"], spec["seed"],
                           flags=imm.IMM_TIMING, stream=stream)

    for i in range(args.warmup):
        step()
        print(f"[bench] warmup {i + 1}/{args.warmup} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results = []
    for i in range(args.steps):
        results.append(step())
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    print(f"[bench] {args.steps} timed steps done", file=sys.stderr, flush=True)

    ms_per_step = (t1 - t0) * 1e3 / args.steps
    r = results[-1]
    for x in results:
        assert x.theta == r.theta and list(x.seeds) == list(r.seeds), "runs must be identical"
    # the final selection's pool (every set it used); the sets a run drew
    # ahead and never used are not counted
    sets = r.theta
    value = sets / (ms_per_step / 1e3)

    kernels = kernel_table(g.model, [x.stats for x in results])
    samp_bytes = algorithmic_bytes(g.model, sets, r.stats["entries"], r.stats["edges"],
                                   r.stats["live"])
    ms_sample = r.stats["ms_sample"]

    out = {
        "metric": "RRR sets/s + edges traversed/s (HBM GB/s); IMM time-to-seeds, k=50",
        "value": value,
        "unit": "RRR sets/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {
            "workload": f"{args.workload}: IMM, " + WORKLOAD_TEXT.get(
                args.workload, g.model.upper()) + f", n={g.n}, m={g.m}",
            "k": spec["k"], "epsilon": spec["eps"], "ell": spec["ell"], "seed": spec["seed"],
            "diffusion": g.model.upper(), "parallelism": "single GPU",
        },
        "time_to_seeds_ms": ms_per_step,
        "theta": r.theta,
        "rounds": r.rounds,
        "ic_team": r.stats["team"],
        "ic_big_block": r.stats["big_block"],
        "edges_per_s": r.stats["edges"] / (ms_per_step / 1e3),
        "phase_ms": {"sample": ms_sample, "compact": r.stats["ms_compact"],
                     "index": r.stats["ms_index"], "select": r.stats["ms_select"],
                     "host_wall": r.stats["ms_total"]},
        "sampling_GBps": samp_bytes / (ms_sample * 1e-3) / 1e9 if ms_sample > 0 else None,
        "sampling_sets_per_s": sets / (ms_sample * 1e-3) if ms_sample > 0 else None,
        "walk_lanes": r.stats["walk_lanes"],
        "bloom_bits": r.stats["bloom_bits"],
        "kernels": kernel_summary(kernels),
        "roofline": roofline_of(kernels, args.workload),
    }
    if args.steady_ids:
        out["steady_state"] = steady_state(imm, g, dg, spec, args.steady_ids, 2, stream,
                                           args.workload)
        print("[bench] steady-state sampling done", file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(g, spec, args.cpu_reps)
        print("[bench] cpu baseline done", file=sys.stderr, flush=True)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
