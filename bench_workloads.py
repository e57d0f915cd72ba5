"""Benchmarks of the other workloads (bench.py --workload ...). Each returns one
JSON-serialisable dict. Not imported by the library itself."""
from __future__ import annotations

import ctypes
import sys
import time

import numpy as np
import torch

from paper_2508_05029_amd import autotune, pipeline, tq
from paper_2508_05029_amd.datagen import workloads as wl
from paper_2508_05029_amd.hosttable import HostTable

HBM_PEAK_GBS = 8000.0
PCIE_GBS = 63.0  # PCIe 5.0 x16, one direction


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def _events():
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def _base(metric, value, unit, args, ms, steps, workload, extra):
    d = {"metric": metric, "value": round(value, 3), "unit": unit, "n_gpus": 1, "steps": steps,
         "warmup": args.warmup, "ms_per_step": round(ms, 5), "higher_is_better": True, "scaling": "weak",
         "vs_baseline": None, "dtype": "int64", "data": "synthetic (seeded generators; stands in for TPC-H/TPC-DS)",
         "config": {"workload": workload}}
    d.update(extra)
    return d


# ------------------------------------------------------------------ filter + group-by

def bench_filter_groupby(args):
    n = 1_000_000
    t = wl.filter_groupby_tables(n)
    q = wl.FILTER_GROUPBY_QUERY
    copies = [pipeline.to_device(t) for _ in range(args.copies)]
    fg = pipeline.FilterGroupBy(q)
    in_bytes = n * 38
    for i in range(max(3, args.warmup)):
        fg.run(copies[i % len(copies)])
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    # the aggregation kernel alone: back-to-back launches over the rotating copies between
    # two events on its stream (the state just accumulates; the timed steps start afresh)
    k_agg = 20
    tq.groupby_init(fg.state, fg.domain, fg.nsum)
    a, b = _events()
    a.record(stream)
    for i in range(k_agg):
        cols = [copies[i % len(copies)][c] for c in fg.names]
        tq.groupby_agg(fg.state, fg.domain, cols, n, fg.preds, fg.key, fg.exprs)
    b.record(stream)
    torch.cuda.synchronize()
    agg_ms = a.elapsed_time(b) / k_agg
    # steps alternate between args.streams compute streams, each with its own state
    from bench import graph_steps_for
    gs = graph_steps_for(args.steps, args.graph_steps)
    nstreams = max(1, args.streams)
    fgs = [fg] + [pipeline.FilterGroupBy(q) for _ in range(nstreams - 1)]
    extra = [torch.cuda.Stream() for _ in range(nstreams - 1)]

    def steps_on_streams(ns):
        cur = torch.cuda.current_stream()
        for s in extra[:ns - 1]:
            s.wait_stream(cur)
        for i in range(gs):
            k = i % ns
            with torch.cuda.stream(cur if k == 0 else extra[k - 1]):
                fgs[k].run(copies[i % len(copies)])
        for s in extra[:ns - 1]:
            cur.wait_stream(s)

    def timed(ns):
        """Exactly args.steps steps (whole replays of gs steps); wall time, and each
        replay's device time from HIP events around it."""
        g = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream()
        side.wait_stream(stream)
        with torch.cuda.stream(side):
            steps_on_streams(ns)
        stream.wait_stream(side)
        torch.cuda.synchronize()
        with torch.cuda.graph(g):
            steps_on_streams(ns)
        g.replay()
        torch.cuda.synchronize()
        reps = args.steps // gs
        marks = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
        t0 = time.perf_counter()
        marks[0].record(stream)
        for r in range(reps):
            g.replay()
            marks[r + 1].record(stream)
        torch.cuda.synchronize()
        per = [marks[r].elapsed_time(marks[r + 1]) / gs for r in range(reps)]
        return (time.perf_counter() - t0) * 1e3 / (reps * gs), reps, per

    ms_one = timed(1)[0] if nstreams > 1 else None
    ms, reps, per_replay = timed(nstreams)
    got = fgs[min(nstreams, gs) - 1].result()
    cpu = None
    parity = None
    if not args.no_cpu_baseline:
        import oracle
        ts = []
        for _ in range(5):
            t1 = time.perf_counter()
            want = oracle.filter_groupby(t, q)
            ts.append(time.perf_counter() - t1)
        tc = float(np.median(ts))
        parity = all(r["sums"].tolist() == want["sums"].tolist() and r["count"].tolist() == want["count"].tolist()
                     for r in [f.result() for f in fgs[:min(nstreams, gs)]])
        cpu = {"value": round(in_bytes / tc / 1e9, 4), "unit": "GB/s", "cores": 1, "kind": "oracle",
               "sample": f"the whole 1M-row workload, median of 5 runs, {tc:.3f} s per run"}
    gbs = in_bytes / (ms / 1e3) / 1e9
    kgbs = in_bytes / (agg_ms / 1e3) / 1e9
    return _base("input GB/s filter-group-by (% of HBM peak)", gbs, "GB/s", args, ms, reps * gs,
                 "filter_groupby: 1M rows, date<=2436, group (flagA, flagB), 5 sums + COUNT + AVG",
                 {"pct_hbm_peak": round(100 * gbs / HBM_PEAK_GBS, 2), "streams": nstreams,
                  "ms_per_step_one_stream": None if ms_one is None else round(ms_one, 5),
                  "ms_per_step_device": {"replays": len(per_replay), "steps_per_replay": gs,
                                         "median": round(float(np.median(per_replay)), 5),
                                         "min": round(float(np.min(per_replay)), 5),
                                         "max": round(float(np.max(per_replay)), 5)},
                  "roofline": {"bound": "hbm", "achieved": round(kgbs, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                               "frac": round(kgbs / HBM_PEAK_GBS, 4), "traffic": None,
                               "kernel": "k_groupby", "bytes_per_launch": in_bytes},
                  "cpu_baseline": cpu, "parity_vs_oracle": parity})


# ------------------------------------------------------------------ out of core

def merge_groups(parts):
    """Groups of several partial results merged: COUNT and SUM added (int64, wrapping
    mod 2^64), in ascending key order. Returns (keys, count, sums) as lists."""
    count, sums = {}, {}
    for r in parts:
        for g, k in enumerate(r["keys"].reshape(-1).tolist()):
            count[k] = count.get(k, 0) + int(r["count"][g])
            s_ = sums.setdefault(k, [0] * r["sums"].shape[1])
            for j in range(r["sums"].shape[1]):
                s_[j] = (s_[j] + int(r["sums"][g, j]) + 2**63) % 2**64 - 2**63
    keys = sorted(count)
    return keys, [count[k] for k in keys], [sums[k] for k in keys]


def ooc_oracle_full(n_fact, n_dim, q, threads):
    """The oracle over the whole out-of-core workload: the dimension generated once, the
    fact table in `threads` row slices generated and joined at once (each slice's C calls
    release the interpreter lock), the slices' groups merged mod 2^64. Only the fact
    columns the query reads are generated. Returns ((keys, count, sums), seconds)."""
    from concurrent.futures import ThreadPoolExecutor
    import oracle
    t0 = time.perf_counter()
    dim = {}
    for name, dt in wl.OOC_DIM_COLS:
        a = np.empty(n_dim, dtype=dt)
        wl.ooc_fill_dim(name, a.ctypes.data, 0, n_dim, n_dim)
        dim[name] = a
    need = {q.probe_key} | {f.col for e in q.sums for f in e if f.col is not None}
    cuts = [n_fact * i // threads for i in range(threads + 1)]

    def one(i):
        a, b = cuts[i], cuts[i + 1]
        f = {}
        for name, dt in wl.OOC_FACT_COLS:
            if name in need:
                arr = np.empty(b - a, dtype=dt)
                wl.ooc_fill_fact(name, arr.ctypes.data, a, b - a, n_dim)
                f[name] = arr
        r = oracle.join_agg(dim, f, q)
        del f
        return r

    with ThreadPoolExecutor(max_workers=threads) as ex:
        parts = list(ex.map(one, range(threads)))
    return merge_groups(parts), time.perf_counter() - t0


def _pinned_copy_peak(pool_bytes=1 << 30):
    h = torch.empty(pool_bytes, dtype=torch.uint8, pin_memory=True)
    d = torch.empty(pool_bytes, dtype=torch.uint8, device="cuda")
    d.copy_(h, non_blocking=True)
    torch.cuda.synchronize()
    a, b = _events()
    a.record()
    for _ in range(4):
        d.copy_(h, non_blocking=True)
    b.record()
    torch.cuda.synchronize()
    gbs = 4 * pool_bytes / (a.elapsed_time(b) / 1e3) / 1e9
    del h, d
    return gbs


def bench_ooc(args):
    scale = args.ooc_scale
    n_fact, n_dim = int(wl.OOC_FACT_ROWS * scale), int(wl.OOC_DIM_ROWS * scale)
    page = 64 << 20
    rows_per_batch = 3 * page // 44 // 256 * 256  # about three pages per fact batch
    budget = int(24e9 * scale) if scale < 1 else int(24e9)
    fact_bytes = n_fact * 44
    dim_bytes = n_dim * 16
    # table pages (with per-batch alignment slack) plus room to spill the whole fact side
    n_pages = int((fact_bytes + dim_bytes) / page * 1.08) + 64 + int(fact_bytes / page) + 32
    log(f"ooc: fact {n_fact} rows, dim {n_dim} rows, {n_pages} pages of 64 MiB, budget {budget / 1e9:.1f} GB")
    t0 = time.perf_counter()
    pool = tq.PagePool(page, n_pages, pinned=True)
    log(f"pinned pool: {time.perf_counter() - t0:.1f} s")
    dt = HostTable(pool, wl.OOC_DIM_COLS, n_dim, rows_per_batch)
    ft = HostTable(pool, wl.OOC_FACT_COLS, n_fact, rows_per_batch)
    t0 = time.perf_counter()
    dt.fill(lambda name, addr, first, count: wl.ooc_fill_dim(name, addr, first, count, n_dim))
    ft.fill(lambda name, addr, first, count: wl.ooc_fill_fact(name, addr, first, count, n_dim))
    log(f"generated into pages: {time.perf_counter() - t0:.1f} s")
    q = wl.JOIN_AGG_QUERY
    peak_link = _pinned_copy_peak()
    results = {}
    # the Adaptive Exchange as a caller gets it, then the partitioned exchange forced,
    # carrying every fact column or only the ones the join reads
    for label, keep_all, exchange in (("adaptive", True, "auto"), ("partitioned_all_columns", True, "partitioned"),
                                      ("partitioned_projected", False, "partitioned")):
        job = pipeline.OocJoinAgg(q, dt, ft, budget, log2_fanout=8, chunk_bytes=4 << 20, nslots=3, keep_all=keep_all,
                                  exchange=exchange)
        st = job.run()
        torch.cuda.synchronize()
        r = job.result()
        results[label] = (st.as_dict(), r)
        log(label, st.as_dict())
        del job
        torch.cuda.empty_cache()
    st, r = results["adaptive"]
    ms = st["ms_total"]
    # every group of every full-size run against the oracle over the whole workload
    full = None
    if not args.no_cpu_baseline:
        from bench import HOST_THREADS_MAX, host_cpu
        _, usable, _ = host_cpu()
        threads = max(1, min(HOST_THREADS_MAX, usable))
        (wk, wc, ws), t_full = ooc_oracle_full(n_fact, n_dim, q, threads)
        full = {"rows": f"{n_fact} fact x {n_dim} dim (the whole workload)", "threads": threads,
                "oracle_s": round(t_full, 1), "groups": len(wk)}
        for label, (_, rr) in results.items():
            full["equal_" + label] = (rr["keys"].reshape(-1).tolist() == wk and rr["count"].tolist() == wc
                                      and rr["sums"].tolist() == ws)
        log("ooc full-size oracle", full)
    in_bytes = fact_bytes + n_dim * 16
    link_gbs = st["bytes_h2d"] / (ms / 1e3) / 1e9
    # parity on a sample scale against the oracle
    parity = None
    if not args.no_cpu_baseline:
        import oracle
        sd, sf = wl.ooc_tables_numpy(2_000_000, 500_000)
        spool = tq.PagePool(1 << 20, 400, pinned=True)
        sdt = HostTable(spool, wl.OOC_DIM_COLS, len(sd["key"]), 100_000)
        sdt.fill_numpy(sd)
        sft = HostTable(spool, wl.OOC_FACT_COLS, len(sf["fk"]), 100_000)
        sft.fill_numpy(sf)
        gots = {}
        for exchange in ("auto", "partitioned"):
            sj = pipeline.OocJoinAgg(q, sdt, sft, 64 << 20, log2_fanout=6, chunk_bytes=256 << 10, exchange=exchange)
            sj.run()
            gots[exchange] = (sj.result(), sj.stats)
            del sj
        t1 = time.perf_counter()
        want = oracle.join_agg(sd, sf, q)
        tc = time.perf_counter() - t1
        parity = {"sample": "2M fact x 500K dim rows, budget 64 MiB: adaptive (one table) and forced partitioned "
                            "(spills)",
                  "equal": all(g["sums"].tolist() == want["sums"].tolist() and g["count"].tolist() == want["count"].tolist()
                               for g, _ in gots.values()),
                  "exchange_auto": gots["auto"][1].exchange,
                  "spilled_chunks_partitioned": gots["partitioned"][1].spilled_chunks}
        cpu = {"value": round((2_000_000 * 44 + 500_000 * 16) / tc / 1e9, 4), "unit": "GB/s", "cores": 1,
               "kind": "oracle", "sample": f"2M x 500K rows of the same tables, {tc:.2f} s"}
        sdt.free()
        sft.free()
        spool.close()
    else:
        cpu = None
    out = _base("host-link GB/s out-of-core join-aggregate (% of PCIe and of the measured pinned-copy peak)",
                link_gbs, "GB/s", args, ms, 1,
                f"ooc_join_agg: fact {n_fact} rows x 6 cols (44 B/row) in 64 MiB pinned pages, dim {n_dim} rows, "
                f"Adaptive Exchange (one table when it fits, else 256 partitions), budget {budget / 1e9:.1f} GB",
                {"input_bytes": in_bytes, "input_gbs": round(in_bytes / (ms / 1e3) / 1e9, 3),
                 "pct_pcie_theoretical": round(100 * link_gbs / PCIE_GBS, 2),
                 "pct_measured_pinned_copy": round(100 * link_gbs / peak_link, 2),
                 "measured_pinned_copy_gbs": round(peak_link, 2),
                 "stats": st, "partitioned_all_columns": results["partitioned_all_columns"][0],
                 "partitioned_projected": results["partitioned_projected"][0],
                 "groups": len(r["count"]), "join_rows": r["join_rows"],
                 "roofline": {"bound": "host-link", "achieved": round(link_gbs, 3), "peak": PCIE_GBS, "unit": "GB/s",
                              "frac": round(link_gbs / PCIE_GBS, 4), "traffic": None,
                              "kernel": "tq_ooc_join_agg (whole pipeline)"},
                 "cpu_baseline": cpu, "parity_vs_oracle": parity, "parity_full_size": full})
    dt.free()
    ft.free()
    pool.close()
    return out


# ------------------------------------------------------------------ batched

def bench_batched(args):
    count = args.instances
    shapes = wl.batched_shapes(count)
    t0 = time.perf_counter()
    insts = []
    for i, s in enumerate(shapes):
        d, f = wl.batched_instance_tables(i, s)
        insts.append((d, f, s.groups))
    log(f"batched: {count} instances generated in {time.perf_counter() - t0:.1f} s; "
        f"fact rows {sum(s.n_fact for s in shapes)}, dim rows {sum(s.n_dim for s in shapes)}")
    q = wl.batched_query(8)
    table = autotune.tune_batched(q, insts, cache_path=None, sample=32, reps=2, log=log)
    params = autotune.params_for(insts, table)
    log(f"batched: tuned; laying out {count} instances on the device")
    job = pipeline.BatchedJoinAgg(q, insts, params)
    log("batched: instances uploaded and prepared")
    in_bytes = job.input_bytes
    stream = torch.cuda.current_stream()
    side = torch.cuda.Stream()
    side.wait_stream(stream)
    with torch.cuda.stream(side):
        job.run()
    stream.wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        job.run()
    for _ in range(max(1, args.warmup // 4)):
        g.replay()
    torch.cuda.synchronize()
    reps = max(3, args.steps // 40)
    a, b = _events()
    a.record()
    for _ in range(reps):
        g.replay()
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    job.check()
    log(f"batched: graph replays done, {ms:.2f} ms per pass")
    # one launch per instance, for comparison
    a, b = _events()
    job.run_per_instance()
    torch.cuda.synchronize()
    a.record()
    job.run_per_instance()
    b.record()
    torch.cuda.synchronize()
    ms_per_inst = a.elapsed_time(b)
    log(f"batched: one launch per instance, {ms_per_inst:.2f} ms per pass")
    # parity on a sample of instances against the oracle
    parity = None
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        job.run()
        torch.cuda.synchronize()
        # every instance against the oracle (on the host's cores at once); the single-core
        # baseline is timed on an evenly spaced sample of them
        from concurrent.futures import ThreadPoolExecutor
        from bench import HOST_THREADS_MAX, host_cpu
        got = job.results(list(range(count)))
        sample = set(range(0, count, max(1, count // 24)))

        def check(i):
            d, f, G = insts[i]
            want = oracle.join_agg(d, f, wl.batched_query(G))
            return (got[i]["keys"].reshape(-1).tolist() == want["keys"].reshape(-1).tolist()
                    and got[i]["sums"].tolist() == want["sums"].tolist()
                    and got[i]["count"].tolist() == want["count"].tolist()
                    and bool(np.all(np.abs(got[i]["avg"] - want["avg"]) <= 1e-12 * np.abs(want["avg"]))))

        _, usable, _ = host_cpu()
        threads = max(1, min(HOST_THREADS_MAX, usable))
        t1 = time.perf_counter()
        with ThreadPoolExecutor(max_workers=threads) as ex:
            oks = list(ex.map(check, range(count)))
        t_all = time.perf_counter() - t1
        bad = [i for i, o in enumerate(oks) if not o]
        tc = 0.0
        rows = 0
        for i in sorted(sample):
            d, f, G = insts[i]
            t1 = time.perf_counter()
            oracle.join_agg(d, f, wl.batched_query(G))
            tc += time.perf_counter() - t1
            rows += len(d["key"]) * 24 + len(f["fk"]) * 24
        parity = {"instances_checked": count, "equal": not bad, "unequal_instances": bad[:20],
                  "oracle_threads": threads, "oracle_s": round(t_all, 1)}
        cpu = {"value": round(rows / tc / 1e9, 4), "unit": "GB/s", "cores": 1, "kind": "oracle",
               "sample": f"{len(sample)} evenly spaced of the {count} instances, {tc:.2f} s"}
    gbs = in_bytes / (ms / 1e3) / 1e9
    return _base("input GB/s batched join-aggregate instances (% of HBM peak)", gbs, "GB/s", args, ms, reps,
                 f"batched: {count} instances, fact log-uniform 1e3..1e6, dim = fact/4, groups log-uniform "
                 f"4..65536 Zipf(1.1), int64 columns; one queue launch per phase, all in a hipGraph",
                 {"input_bytes": in_bytes, "pct_hbm_peak": round(100 * gbs / HBM_PEAK_GBS, 2),
                  "ms_one_launch_per_instance": round(ms_per_inst, 3),
                  "speedup_vs_per_instance": round(ms_per_inst / ms, 2),
                  "autotuned": {k: list(v) for k, v in table.items()},
                  "roofline": {"bound": "hbm", "achieved": round(gbs, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                               "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": None,
                               "kernel": "k_batched (+ k_batched_prep)", "bytes_per_launch": in_bytes},
                  "cpu_baseline": cpu, "parity_vs_oracle": parity})


# ------------------------------------------------------------------ serving

def _serve_expected(setup, q):
    """The oracle's result for one served request (its windows of the base tables)."""
    import oracle
    if q.shape == 0:
        t = {k: v[q.fact_first:q.fact_first + q.n_fact] for k, v in setup.fg.items()}
        return oracle.filter_groupby(t, setup.q0)
    d = {k: v[q.dim_first:q.dim_first + q.n_dim] for k, v in setup.dim.items()}
    if q.shape == 1:
        f = {k: v[q.fact_first:q.fact_first + q.n_fact] for k, v in setup.fact.items()}
    else:
        lo = setup.host.batches[q.fact_first][0]
        last = setup.host.batches[q.fact_first + q.n_fact - 1]
        f = {k: v[lo:last[0] + last[1]] for k, v in setup.hfact.items()}
    return oracle.join_agg(d, f, setup.q1)


def _serve_result(q, out, i):
    """(keys, COUNT, SUMs, AVGs) of served request i in the oracle's layout."""
    res, keys, count, sums, avg = out
    g = res[i].ngroups
    nsum = 5 if q.shape == 0 else 1
    k = keys[i, :g]
    k = np.stack([k // 2, k % 2], axis=1) if q.shape == 0 else k.reshape(-1, 1)
    return k, count[i, :g], sums[i, :g, :nsum], avg[i, :g, :nsum]


def _same(a, b):
    """Integer parts bit-equal, AVG within 1e-12 relative."""
    (ka, ca, sa, aa), (kb, cb, sb, ab) = a, b
    if not (ka.tolist() == kb.tolist() and ca.tolist() == cb.tolist() and sa.tolist() == sb.tolist()):
        return False
    return bool(np.all(np.abs(aa - ab) <= 1e-12 * np.abs(ab)))


def bench_serving(args):
    """Poisson arrivals of mixed requests at 0.5, 0.8, 1.0 and 1.2 times the FIFO service
    rate (measured first), each served one at a time (FIFO) and by concurrent workers;
    latency percentiles over the requests after a warm-up; every request's result alone
    (FIFO) equal to its result in the mix, and a sample against the oracle."""
    pool = tq.PagePool(64 << 20, 160, pinned=True)
    nbase = args.serve_base_rows
    setup = pipeline.ServingSetup(n0=nbase, n_dim=nbase // 4, n1=nbase, n2=nbase, batch_rows=1 << 20, pool=pool)
    budget_bytes = int(64e9)
    arena = torch.empty(min(budget_bytes, 48 << 30), dtype=torch.uint8, device="cuda")
    warm, n_meas = 100, args.requests
    n = warm + n_meas
    # the FIFO service rate, from calibration requests that all arrive at once
    cal = wl.serving_requests(200, qps=1e9, seed=wl.SERVE_SEED + 7)
    Rc = setup.requests(cal)
    res, *_ = tq.serve_run(setup.T, Rc, 1, tq.Budget(budget_bytes), arena, 25)
    mu = len(cal) / max(res[i].end_s for i in range(len(cal)))
    log(f"serving: FIFO service rate {mu:.1f} requests/s")
    base = wl.serving_requests(n, qps=1.0)  # arrival times at rate 1; scaled to each rate below
    sweep, kept = [], {}
    for f in (0.5, 0.8, 1.0, 1.2):
        lam = f * mu
        R = setup.requests(base, time_scale=1.0 / lam)
        for label, workers in (("fifo", 1), ("continuous", args.workers)):
            out = tq.serve_run(setup.T, R, workers, tq.Budget(budget_bytes), arena, 25)
            res = out[0]
            idx = range(warm, n)
            lat = np.array([res[i].end_s - R[i].arrival_s for i in idx])
            span = max(res[i].end_s for i in idx) - R[warm].arrival_s
            row = {"rate_x_fifo": f, "arrivals_per_s": round(lam, 2), "mode": label, "workers": workers,
                   "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 3),
                   "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 3),
                   "mean_ms": round(float(lat.mean()) * 1e3, 3), "qps": round(n_meas / span, 2),
                   "failed": int(sum(res[i].status != 0 for i in range(n))),
                   "retries": int(sum(res[i].retries for i in range(n))),
                   "mean_reserved_mib": round(float(np.mean([res[i].reserved_bytes for i in idx])) / 2**20, 2)}
            sweep.append(row)
            log(row)
            if f == 0.8:
                kept[label] = (R, out)
    # every request: alone (FIFO, one at a time) == in the mix (concurrent workers)
    R, fifo = kept["fifo"]
    _, mix = kept["continuous"]
    unequal = [i for i in range(n) if not _same(_serve_result(R[i], fifo, i), _serve_result(R[i], mix, i))]
    # a sample against the oracle: the smallest requests of each shape
    sizes = sorted(range(n), key=lambda i: (R[i].shape, R[i].n_fact))
    sample = []
    for shape in (0, 1, 2):
        sample += [i for i in sizes if R[i].shape == shape][:8]
    oracle_bad = [i for i in sample if not _same(_serve_result(R[i], mix, i), _packed_want(_serve_expected(setup, R[i])))]
    setup.host.free()
    pool.close()
    head = [r for r in sweep if r["rate_x_fifo"] == 0.8 and r["mode"] == "continuous"][0]
    return _base("p50/p99 served query latency (ms) and queries/s, continuous batching vs FIFO", head["qps"],
                 "queries/s", args, head["mean_ms"], n_meas,
                 f"serving: {n_meas} requests after {warm} warm-up, shapes 0/1/2 uniform, fact rows log-uniform "
                 f"1e4..1e8 (windows of {nbase}-row base tables), Poisson arrivals at 0.5/0.8/1.0/1.2 x the FIFO "
                 f"rate ({mu:.1f}/s), 64 GB budget, {args.workers} workers",
                 {"p50_ms": head["p50_ms"], "p99_ms": head["p99_ms"], "calibrated_fifo_qps": round(mu, 2),
                  "sweep": sweep,
                  "alone_equals_mix": {"requests": n, "unequal": unequal[:20], "equal": not unequal},
                  "oracle_sample": {"requests": sample, "unequal": oracle_bad, "equal": not oracle_bad},
                  "roofline": None, "cpu_baseline": None})


def _packed_want(w):
    return w["keys"], w["count"], w["sums"], w["avg"]


# ------------------------------------------------------------------ steady state at growing row counts

def measured_read_peak(nbytes=1 << 30, reps=5):
    """GB/s of k_read_peak over nbytes (the device's streaming-read ceiling, measured in the same run)."""
    x = torch.empty(nbytes // 8, dtype=torch.int64, device="cuda")
    part = torch.zeros(max(1, tq.read_peak_scratch_bytes() // 8), dtype=torch.int64, device="cuda")
    tq.fill(x, 0x01010101)
    tq.read_peak(x, part)
    torch.cuda.synchronize()
    a, b = _events()
    a.record()
    for _ in range(reps):
        tq.read_peak(x, part)
    b.record()
    torch.cuda.synchronize()
    gbs = nbytes / (a.elapsed_time(b) / reps / 1e3) / 1e9
    del x, part
    return gbs


def _replay_ms(step, ncopies, graph_steps, steps):
    """ms per step of `step(i)` (i picks the input copy), replayed from a HIP graph."""
    stream = torch.cuda.current_stream()
    for i in range(3):
        step(i % ncopies)
    side = torch.cuda.Stream()
    side.wait_stream(stream)
    with torch.cuda.stream(side):
        for i in range(graph_steps):
            step(i % ncopies)
    stream.wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for i in range(graph_steps):
            step(i % ncopies)
    g.replay()
    torch.cuda.synchronize()
    reps = max(1, steps // graph_steps)
    t0 = time.perf_counter()
    for _ in range(reps):
        g.replay()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / (reps * graph_steps), g


def bench_scaling(args):
    """The join+aggregate and filter+group-by steps at growing row counts (same value
    distributions), so that fixed per-launch costs fade and the steady state shows; each
    point is checked against the oracle."""
    import oracle
    peak = measured_read_peak()
    log(f"measured read peak {peak:.0f} GB/s")
    points = []
    jq = wl.JOIN_AGG_QUERY
    for n_dim, n_fact in ((1_500_000, 6_000_000), (6_000_000, 24_000_000), (25_000_000, 100_000_000)):
        dim, fact = wl.join_agg_tables(n_dim, n_fact)
        in_bytes = n_dim * 16 + n_fact * 24
        ncopies = max(2, min(4, (1 << 30) // in_bytes + 1))
        copies = [(pipeline.to_device(dim), pipeline.to_device(fact)) for _ in range(ncopies)]
        ja = pipeline.JoinAgg(jq, n_dim, args.load_factor)

        def step(i):
            d, f = copies[i]
            ja.init_state()
            ja.build(d)
            ja.probe(f)
            ja.finalize()

        steps = max(16, min(args.steps, int(4e9 // in_bytes) * 8))
        ms, g = _replay_ms(step, ncopies, 8, steps)
        got = ja.result()
        want = oracle.join_agg(dim, fact, jq)
        ok = (got["keys"].tolist() == want["keys"].tolist() and got["count"].tolist() == want["count"].tolist()
              and got["sums"].tolist() == want["sums"].tolist())
        gbs = in_bytes / (ms / 1e3) / 1e9
        points.append({"workload": "join_agg", "dim_rows": n_dim, "fact_rows": n_fact, "ms_per_step": round(ms, 4),
                       "gbs": round(gbs, 1), "pct_hbm_peak": round(100 * gbs / HBM_PEAK_GBS, 2),
                       "pct_measured_read_peak": round(100 * gbs / peak, 2), "parity_vs_oracle": ok})
        log(points[-1])
        del copies, ja, g
        torch.cuda.empty_cache()
    fq = wl.FILTER_GROUPBY_QUERY
    for n in (1_000_000, 10_000_000, 100_000_000):
        t = wl.filter_groupby_tables(n)
        in_bytes = n * 38
        ncopies = max(2, min(4, (1 << 30) // in_bytes + 1))
        copies = [pipeline.to_device(t) for _ in range(ncopies)]
        fg = pipeline.FilterGroupBy(fq)
        steps = max(16, min(args.steps, int(4e9 // in_bytes) * 8))
        ms, g = _replay_ms(lambda i: fg.run(copies[i]), ncopies, 8, steps)
        got = fg.result()
        want = oracle.filter_groupby(t, fq)
        ok = got["sums"].tolist() == want["sums"].tolist() and got["count"].tolist() == want["count"].tolist()
        gbs = in_bytes / (ms / 1e3) / 1e9
        points.append({"workload": "filter_groupby", "rows": n, "ms_per_step": round(ms, 4), "gbs": round(gbs, 1),
                       "pct_hbm_peak": round(100 * gbs / HBM_PEAK_GBS, 2),
                       "pct_measured_read_peak": round(100 * gbs / peak, 2), "parity_vs_oracle": ok})
        log(points[-1])
        del copies, fg, g
        torch.cuda.empty_cache()
    big = points[2]
    return _base("input GB/s filter-join-aggregate at growing row counts (steady state)", big["gbs"], "GB/s", args,
                 big["ms_per_step"], 0,
                 "scaling: join_agg at 1.5Mx6M, 6Mx24M, 25Mx100M rows; filter_groupby at 1M, 10M, 100M rows; "
                 "value = the largest join",
                 {"measured_read_peak_gbs": round(peak, 1), "points": points, "roofline": None, "cpu_baseline": None})


# ------------------------------------------------------------------ plain copy kernels (calibration)

def bench_copy(args):
    """Read-only and write-only passes over 1 GiB: the measured HBM ceilings, and
    the kernels whose FETCH_SIZE / WRITE_SIZE counters calibrate those of the
    query kernels (k_read_peak reads exactly 1 GiB, k_fill writes exactly 1 GiB)."""
    nbytes = 1 << 30
    x = torch.empty(nbytes // 8, dtype=torch.int64, device="cuda")
    part = torch.zeros(max(1, tq.read_peak_scratch_bytes() // 8), dtype=torch.int64, device="cuda")
    tq.fill(x, 0x01010101)
    for _ in range(3):
        tq.read_peak(x, part)
    torch.cuda.synchronize()
    reps = max(4, min(args.steps, 50))
    a, b = _events()
    a.record()
    for _ in range(reps):
        tq.read_peak(x, part)
    b.record()
    torch.cuda.synchronize()
    ms_r = a.elapsed_time(b) / reps
    a.record()
    for _ in range(reps):
        tq.fill(x, 7)
    b.record()
    torch.cuda.synchronize()
    ms_w = a.elapsed_time(b) / reps
    rd = nbytes / (ms_r / 1e3) / 1e9
    wr = nbytes / (ms_w / 1e3) / 1e9
    return _base("HBM GB/s of a plain read and a plain write of 1 GiB", rd, "GB/s", args, ms_r, reps,
                 "copy: k_read_peak over 1 GiB, k_fill over 1 GiB",
                 {"read_gbs": round(rd, 1), "write_gbs": round(wr, 1), "ms_read": round(ms_r, 4),
                  "ms_write": round(ms_w, 4), "bytes_per_launch": nbytes,
                  "roofline": {"bound": "hbm", "achieved": round(rd, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                               "frac": round(rd / HBM_PEAK_GBS, 4), "traffic": None, "kernel": "k_read_peak"},
                  "cpu_baseline": None})


# ------------------------------------------------------------------ Parquet scan

def _write_parquet(path, table, codec, page_bytes=1 << 20, row_group_rows=None):
    import pyarrow as pa
    import pyarrow.parquet as pq
    arrays = {k: pa.array(v) for k, v in table.items()}
    schema = pa.schema([pa.field(k, a.type, nullable=False) for k, a in arrays.items()])
    pq.write_table(pa.Table.from_pydict(arrays, schema=schema), path, compression=codec, data_page_size=page_bytes,
                   row_group_size=row_group_rows)
    import os
    return os.path.getsize(path)


def bench_scan(args):
    """The join + aggregate tables (1.5M x 6M rows) as Parquet files with 1 MiB
    pages, dictionary encoding where it fits (pyarrow's default), Snappy and
    uncompressed. A step: preload both files' byte ranges into pool pages,
    decode them on the GPU, run the join + aggregate on the decoded columns."""
    import os
    import shutil
    import tempfile
    import oracle
    n_dim, n_fact = 1_500_000, 6_000_000
    dim, fact = wl.join_agg_tables(n_dim, n_fact)
    q = wl.JOIN_AGG_QUERY
    want = oracle.join_agg(dim, fact, q)
    tmp = tempfile.mkdtemp(prefix="tq_scan_", dir="/dev/shm" if os.path.isdir("/dev/shm") else None)
    out = {}
    try:
        pool = tq.PagePool(16 << 20, 64)  # 1 GiB of pinned pages
        value_bytes = n_dim * 16 + n_fact * 24
        for codec in ("snappy", "NONE"):
            dpath, fpath = os.path.join(tmp, f"dim_{codec}.parquet"), os.path.join(tmp, f"fact_{codec}.parquet")
            file_bytes = _write_parquet(dpath, dim, codec) + _write_parquet(fpath, fact, codec)
            ds = pipeline.ParquetScan(dpath, list(dim), pool)
            fs = pipeline.ParquetScan(fpath, list(fact), pool)
            ja = pipeline.JoinAgg(q, n_dim, 0.5)
            stream = torch.cuda.current_stream()
            side = torch.cuda.Stream()  # the two files are decoded at once, one per stream

            def step():
                t0 = time.perf_counter()
                dpl, fpl = ds.preload(), fs.preload()  # both files' reads start at once
                dpl.work_bytes()
                fpl.work_bytes()
                t1 = time.perf_counter()
                a, b = _events()
                a.record(stream)
                side.wait_stream(stream)
                dd, _ = ds.decode(dpl, side)
                ff, _ = fs.decode(fpl)
                stream.wait_stream(side)
                b.record(stream)
                ja.run(dd, ff)
                torch.cuda.synchronize()
                t2 = time.perf_counter()
                dpl.free()
                fpl.free()
                return (t1 - t0) * 1e3, a.elapsed_time(b), (t2 - t0) * 1e3

            for _ in range(max(2, args.warmup // 8)):
                step()
            ds.check()
            fs.check()
            got = ja.result()
            equal = (got["keys"][:, 0].tolist() == want["keys"][:, 0].tolist() and
                     got["count"].tolist() == want["count"].tolist() and got["sums"].tolist() == want["sums"].tolist())
            def step_pipelined():
                # row group by row group, the next one's bytes read while this one decodes
                t0 = time.perf_counter()
                side.wait_stream(stream)
                dd, _ = ds.read_pipelined(side)
                ff, _ = fs.read_pipelined()
                stream.wait_stream(side)
                ja.run(dd, ff)
                torch.cuda.synchronize()
                return (time.perf_counter() - t0) * 1e3

            k = min(args.steps, 10)
            step_pipelined()
            piped = float(np.median([step_pipelined() for _ in range(k)]))
            got2 = ja.result()
            equal = equal and got2["sums"].tolist() == want["sums"].tolist()
            runs = [step() for _ in range(k)]
            pre = float(np.median([r[0] for r in runs]))
            dec = float(np.median([r[1] for r in runs]))
            tot = float(np.median([r[2] for r in runs]))
            out[codec] = {"file_bytes": file_bytes, "value_bytes": value_bytes, "ms_preload": round(pre, 3),
                          "ms_copy_and_decode": round(dec, 3), "ms_step": round(tot, 3),
                          "ms_step_row_groups_pipelined": round(piped, 3),
                          "file_gbs_preload": round(file_bytes / pre / 1e6, 2),
                          "decoded_gbs": round(value_bytes / dec / 1e6, 2),
                          "result_equals_oracle": equal}
            log(codec, out[codec])
            pool_free = pool.free_pages()
            assert pool_free == 64, pool_free
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
    s = out["snappy"]
    return _base("Parquet scan + join-aggregate: decoded GB/s (file bytes preloaded, copied, decoded on the GPU)",
                 s["value_bytes"] / s["ms_step"] / 1e6, "GB/s", args, s["ms_step"], min(args.steps, 10),
                 "scan: dim 1.5M + fact 6M rows as Parquet (1 MiB pages, pyarrow dictionary default), Snappy; "
                 "preload -> decode (the two files on two streams) -> join+aggregate per step",
                 {"codecs": out, "roofline": None, "cpu_baseline": None})
