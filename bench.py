#!/usr/bin/env python3
"""Benchmark of the columnar query hot path on one MI355X.

Default workload (join_agg): dimension 1.5M rows (key, group, date), fact 6M
rows (fk, price, discount). One step = filter the dimension to a 365-day
window, build the open-addressing table, probe it with every fact row while
aggregating SUM(price * (100 - discount)) and COUNT per group, and finalize the
25 groups in key order (the finalize also empties the group-by state for the
next step). Inputs are device resident; four copies rotate so that
consecutive steps do not find their input in the 256 MiB Infinity Cache.

value = input bytes the query must read (16 B per dimension row + 24 B per fact
row = 168 MB) / wall time per step, in GB/s. Steps are replayed from HIP graphs
(several steps per graph) so that host launch cost does not set the pace, and
consecutive steps alternate between --streams streams, each with its own table
and group-by state (several compute streams, each running whole tasks, as the
paper's executor does), so that one step's short kernels overlap another's.

Prints ONE JSON line. Other workloads: --workload filter_groupby | ooc | batched | serving | scaling | copy | scan.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

HBM_PEAK_GBS = 8000.0

# HBM bytes per launch of the probe kernel from rocprofv3 counter runs (FETCH_SIZE and
# WRITE_SIZE in KiB per dispatch, each scaled by what the counter reads for a plain copy
# kernel of known size; the runs are summarised under profiles/). They describe the kernel
# built from these exact sources: if any of them changes, the traffic is reported as null.
PROBE_COUNTERS = {
    "sources": ["paper_2508_05029_amd/csrc/join_ops.hip", "paper_2508_05029_amd/csrc/table.h",
                "paper_2508_05029_amd/csrc/groupby.h", "paper_2508_05029_amd/csrc/common.h"],
    "sha1": "5bd2ff6c5f044cae7e76668ab0a367604e93ecec",
    "fetch_kib": 114927.2, "fetch_scale": 2.000,
    "write_kib": 104.0, "write_scale": 0.9946,
}


def probe_traffic():
    import hashlib
    h = hashlib.sha1()
    for f in PROBE_COUNTERS["sources"]:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest() != PROBE_COUNTERS["sha1"]:
        return None
    c = PROBE_COUNTERS
    return round((c["fetch_kib"] * c["fetch_scale"] + c["write_kib"] * c["write_scale"]) * 1024)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def graph_steps_for(steps, want):
    """Steps per graph: the largest divisor of `steps` not above `want`, so that whole
    replays time exactly `steps` steps."""
    for g in range(max(1, min(want, steps)), 0, -1):
        if steps % g == 0:
            return g
    return 1


def host_cpu():
    """(model name, logical CPUs this process may run on, os.cpu_count())."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return model, usable, os.cpu_count()


# threads of the all-cores oracle run: the host share a single-GPU job is given (16 cores
# per GPU), whatever larger count the machine itself reports
HOST_THREADS_MAX = 16


def events_ms(pairs):
    import torch
    torch.cuda.synchronize()
    return [a.elapsed_time(b) for a, b in pairs]


def cpu_baseline_join_agg(dim, fact, q, budget_s=12.0):
    """The oracle as it stands, single-threaded, on the full workload."""
    import oracle
    times = []
    res = None
    while len(times) < 5 and sum(times) < budget_s:
        t0 = time.perf_counter()
        res = oracle.join_agg(dim, fact, q)
        times.append(time.perf_counter() - t0)
    return res, float(np.median(times)), len(times)


def cpu_all_cores_join_agg(dim, fact, q, want, threads):
    """The same oracle run on `threads` slices of the fact table at once (its C calls
    release the interpreter lock); the slices' groups are merged by adding COUNT and
    SUM (int64, wrapping) and the AVG recomputed as the oracle defines it. Returns
    (seconds, whether the merge equals the one-thread result)."""
    from concurrent.futures import ThreadPoolExecutor
    import oracle
    n = len(fact[q.probe_key])
    cuts = [n * i // threads for i in range(threads + 1)]
    slices = [{k: v[cuts[i]:cuts[i + 1]] for k, v in fact.items()} for i in range(threads)]
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        parts = list(ex.map(lambda f: oracle.join_agg(dim, f, q), slices))
    count, sums = {}, {}
    for r in parts:
        for g, k in enumerate(r["keys"].reshape(-1).tolist()):
            count[k] = count.get(k, 0) + int(r["count"][g])
            s_ = sums.setdefault(k, [0] * r["sums"].shape[1])
            for j in range(r["sums"].shape[1]):
                s_[j] = (s_[j] + int(r["sums"][g, j]) + 2**63) % 2**64 - 2**63
    dt = time.perf_counter() - t0
    keys = sorted(count)
    ok = (keys == want["keys"].reshape(-1).tolist() and [count[k] for k in keys] == want["count"].tolist()
          and [sums[k] for k in keys] == want["sums"].tolist())
    return dt, ok


def bench_join_agg(args):
    import torch
    from paper_2508_05029_amd import pipeline
    from paper_2508_05029_amd.datagen import workloads as wl

    n_dim, n_fact = 1_500_000, 6_000_000
    dim, fact = wl.join_agg_tables(n_dim, n_fact)
    q = wl.JOIN_AGG_QUERY
    in_bytes = n_dim * 16 + n_fact * 24
    probe_bytes = n_fact * 24
    copies = [(pipeline.to_device(dim), pipeline.to_device(fact)) for _ in range(args.copies)]
    ja = pipeline.JoinAgg(q, n_dim, args.load_factor)
    stream = torch.cuda.current_stream()
    nstreams = max(1, args.streams)
    jas = [ja] + [pipeline.JoinAgg(q, n_dim, args.load_factor) for _ in range(nstreams - 1)]
    extra_streams = [torch.cuda.Stream() for _ in range(nstreams - 1)]

    # A step: build, probe with the fused group-by, finalize. The finalize leaves the
    # group-by state empty (tq_groupby_finalize_reset), so the state is set up once here
    # and each step starts from zero without a launch of its own.
    for j in jas:
        j.init_state()

    def step(i):
        d, f = copies[i % len(copies)]
        ja.build(d)
        ja.probe(f)
        ja.finalize(reset=True)

    # eager warmup, then per-kernel timing with HIP events on the launch stream
    for i in range(max(args.warmup, 3)):
        step(i)
    torch.cuda.synchronize()
    ev = {k: [] for k in ("build", "probe", "finalize")}
    for i in range(args.event_steps):
        d, f = copies[i % len(copies)]
        marks = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        marks[0].record(stream)
        ja.build(d)
        marks[1].record(stream)
        ja.probe(f)
        marks[2].record(stream)
        ja.finalize(reset=True)
        marks[3].record(stream)
        for j, k in enumerate(ev):
            ev[k].append((marks[j], marks[j + 1]))
    kern_ms = {k: float(np.mean(events_ms(v))) for k, v in ev.items()}
    # the probe alone: back-to-back launches between two events on its stream, over the
    # rotating copies so that no launch finds its columns in the Infinity Cache (its state
    # just accumulates, and is set up afresh below)
    k_probe = 20
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for i in range(k_probe):
        ja.probe(copies[i % len(copies)][1])
    e1.record(stream)
    kern_ms["probe"] = events_ms([(e0, e1)])[0] / k_probe
    ja.init_state()

    # graph: args.graph_steps consecutive steps per replay, rotating the copies; step i
    # runs on stream i % nstreams with that stream's table and state
    gs = graph_steps_for(args.steps, args.graph_steps)

    def steps_on_streams(ns):
        cur = torch.cuda.current_stream()
        for s in extra_streams[:ns - 1]:
            s.wait_stream(cur)
        for i in range(gs):
            k = i % ns
            d, f = copies[i % len(copies)]
            with torch.cuda.stream(cur if k == 0 else extra_streams[k - 1]):
                jas[k].build(d)
                jas[k].probe(f)
                jas[k].finalize(reset=True)
        for s in extra_streams[:ns - 1]:
            cur.wait_stream(s)

    def timed(ns, k_steps):
        """Exactly k_steps steps (k_steps / gs replays); wall time of the whole run, and
        each replay's device time from HIP events around it on the replay stream."""
        side = torch.cuda.Stream()
        side.wait_stream(stream)
        with torch.cuda.stream(side):
            steps_on_streams(ns)
        stream.wait_stream(side)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            steps_on_streams(ns)
        torch.cuda.synchronize()
        for _ in range(max(1, -(-args.warmup // gs))):
            graph.replay()
        torch.cuda.synchronize()
        reps = k_steps // gs
        marks = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
        t0 = time.perf_counter()
        marks[0].record(stream)
        for r in range(reps):
            graph.replay()
            marks[r + 1].record(stream)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) * 1e3 / (reps * gs)
        per = [marks[r].elapsed_time(marks[r + 1]) / gs for r in range(reps)]
        return wall, reps * gs, per

    ms_one_stream = timed(1, args.steps)[0] if nstreams > 1 else None
    ms_step, steps, per_replay = timed(nstreams, args.steps)

    # timed probe launches inside graph replays are measured by the eager events above;
    # the result of each stream's last replayed step is checked against the oracle below
    gots = [j.result() for j in jas[:min(nstreams, gs)]]
    cpu = cpu_all = None
    parity = None
    if not args.no_cpu_baseline:
        want, t_cpu, runs = cpu_baseline_join_agg(dim, fact, q)
        parity = all(got["keys"].tolist() == want["keys"].tolist() and got["count"].tolist() == want["count"].tolist()
                     and got["sums"].tolist() == want["sums"].tolist() for got in gots)
        cpu = {"value": round(in_bytes / t_cpu / 1e9, 4), "unit": "GB/s", "cores": 1, "kind": "oracle",
               "sample": f"the whole workload (1.5M x 6M rows), median of {runs} runs of the sort-based C oracle, "
                         f"{t_cpu:.2f} s per run"}
        model, usable, total = host_cpu()
        threads = max(1, min(HOST_THREADS_MAX, usable))
        t_all, ok_all = cpu_all_cores_join_agg(dim, fact, q, want, threads)
        cpu_all = {"value": round(in_bytes / t_all / 1e9, 4), "unit": "GB/s", "cores": threads, "kind": "oracle",
                   "sample": f"the whole workload, the fact table in {threads} slices run at once, {t_all:.2f} s",
                   "equal_to_one_thread": ok_all, "host_cpu": model, "host_cpus_usable": usable,
                   "host_cpus_reported": total}
    gbs = in_bytes / (ms_step / 1e3) / 1e9
    probe_gbs = probe_bytes / (kern_ms["probe"] / 1e3) / 1e9
    from bench_workloads import measured_read_peak
    read_peak = measured_read_peak()
    line = {
        "metric": "input GB/s filter-join-aggregate (% of HBM peak)",
        "value": round(gbs, 2), "unit": "GB/s", "n_gpus": 1, "steps": steps, "warmup": args.warmup,
        "ms_per_step": round(ms_step, 5), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int64", "data": "synthetic (seeded generators; stands in for TPC-H/TPC-DS tables)",
        "config": {"workload": "join_agg: dim 1.5M rows (key perm, group U0..24, date U0..2405), fact 6M rows "
                               "(fk U over dim keys, price, discount); date window [730,1094]; "
                               "SUM(price*(100-disc)), COUNT by group",
                   "input_bytes": in_bytes, "load_factor": args.load_factor, "copies": args.copies,
                   "graph_steps": gs, "streams": nstreams},
        "pct_hbm_peak": round(100 * gbs / HBM_PEAK_GBS, 2),
        "ms_per_step_one_stream": None if ms_one_stream is None else round(ms_one_stream, 5),
        "ms_per_step_device": {"replays": len(per_replay), "steps_per_replay": gs,
                               "median": round(float(np.median(per_replay)), 5),
                               "min": round(float(np.min(per_replay)), 5), "max": round(float(np.max(per_replay)), 5)},
        "measured_read_peak_gbs": round(read_peak, 1),
        "pct_measured_read_peak": round(100 * gbs / read_peak, 2),
        "rows_per_s": round((n_dim + n_fact) / (ms_step / 1e3), 1),
        "kernel_ms": {k: round(v, 5) for k, v in kern_ms.items()},
        "roofline": {"bound": "hbm", "achieved": round(probe_gbs, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(probe_gbs / HBM_PEAK_GBS, 4), "traffic": probe_traffic(),
                     "kernel": "k_probe_compact (join probe + fused group-by)", "bytes_per_launch": probe_bytes},
        "cpu_baseline": cpu,
        "cpu_baseline_all_cores": cpu_all,
        "parity_vs_oracle": parity,
    }
    return line


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=16)
    ap.add_argument("--workload", default="join_agg",
                    choices=["join_agg", "filter_groupby", "ooc", "batched", "serving", "copy", "scaling", "scan"])
    ap.add_argument("--copies", type=int, default=4)
    ap.add_argument("--graph-steps", type=int, default=8)
    ap.add_argument("--streams", type=int, default=2, help="join_agg, filter_groupby: compute streams the steps alternate between")
    ap.add_argument("--event-steps", type=int, default=20)
    ap.add_argument("--load-factor", type=float, default=0.5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--ooc-scale", type=float, default=1.0, help="fraction of the 600M x 150M out-of-core tables")
    ap.add_argument("--instances", type=int, default=4096, help="batched workload: number of instances")
    ap.add_argument("--requests", type=int, default=2000,
                    help="serving workload: measured requests (after 100 warm-up requests)")
    ap.add_argument("--workers", type=int, default=6, help="serving workload: concurrent workers")
    ap.add_argument("--serve-base-rows", type=int, default=100_000_000,
                    help="serving workload: rows of each base table")
    args = ap.parse_args()
    if args.steps < 1 or args.warmup < 0:
        ap.error("--steps must be at least 1 and --warmup at least 0")
    if args.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU; --gpus above 1 is not supported",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}), flush=True)
        sys.exit(1)
    fn = {"join_agg": bench_join_agg}.get(args.workload)
    if fn is None:
        import bench_workloads
        fn = getattr(bench_workloads, "bench_" + args.workload)
    line = fn(args)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
