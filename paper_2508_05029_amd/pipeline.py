"""Query pipelines over the C ABI: filter + group-by, and join + aggregate.

A pipeline turns a query description (column names, predicates, product
expressions, a group key) into the index-based descriptors of the C ABI,
owns the device buffers it needs (allocated once, through torch) and enqueues
the library calls on a stream. It does no arithmetic of its own.
"""
from __future__ import annotations

import ctypes
from typing import Dict, List, Optional, Sequence

import numpy as np
import torch

from . import tq

I64_MIN = -(2 ** 63)


def to_device(table: Dict[str, np.ndarray], device="cuda") -> Dict[str, torch.Tensor]:
    return {k: torch.from_numpy(np.ascontiguousarray(v)).to(device) for k, v in table.items()}


def _col_index(names: List[str], name: str) -> int:
    return names.index(name)


def plan_preds(names, preds) -> List[tuple]:
    return [(_col_index(names, p.col), p.lo, p.hi) for p in preds]


def plan_exprs(names, exprs) -> List[List[tuple]]:
    return [[(-1 if f.col is None else _col_index(names, f.col), f.sign, f.add) for f in e] for e in exprs]


def referenced(preds, exprs, extra=()) -> List[str]:
    names: List[str] = []
    for c in list(extra) + [p.col for p in preds] + [f.col for e in exprs for f in e]:
        if c is not None and c not in names:
            names.append(c)
    return names


class GroupByResult:
    def __init__(self, domain: int, nsum: int, device):
        self.keys = torch.empty(domain, dtype=torch.int64, device=device)
        self.count = torch.empty(domain, dtype=torch.int64, device=device)
        self.sums = torch.empty(domain * max(nsum, 1), dtype=torch.int64, device=device)
        self.avg = torch.empty(domain * max(nsum, 1), dtype=torch.float64, device=device)
        self.ngroups = torch.zeros(1, dtype=torch.int64, device=device)
        self.nsum = nsum

    def host(self) -> dict:
        g = int(self.ngroups.item())
        return {"keys": self.keys[:g].cpu().numpy(), "count": self.count[:g].cpu().numpy(),
                "sums": self.sums[: g * self.nsum].cpu().numpy().reshape(g, self.nsum),
                "avg": self.avg[: g * self.nsum].cpu().numpy().reshape(g, self.nsum)}


class FilterGroupBy:
    """sigma + pi + gamma in one pass: tq_groupby_init / tq_groupby_agg / tq_groupby_finalize."""

    def __init__(self, query, device="cuda"):
        self.q = query
        self.names = referenced(query.preds, query.sums, query.key.cols)
        self.preds = plan_preds(self.names, query.preds)
        self.exprs = plan_exprs(self.names, query.sums)
        self.key = tq.gkey([_col_index(self.names, c) for c in query.key.cols], query.key.mult)
        self.domain = query.key.domain
        self.nsum = len(query.sums)
        self.state = torch.empty(tq.groupby_state_bytes(self.domain, self.nsum), dtype=torch.uint8, device=device)
        self.out = GroupByResult(self.domain, self.nsum, device)

    def run(self, table: Dict[str, torch.Tensor], nrows: Optional[int] = None, stream=None):
        cols = [table[c] for c in self.names]
        n = cols[0].numel() if nrows is None else nrows
        tq.groupby_init(self.state, self.domain, self.nsum, stream)
        tq.groupby_agg(self.state, self.domain, cols, n, self.preds, self.key, self.exprs, stream)
        tq.groupby_finalize(self.state, self.out.keys, self.out.count, self.out.sums, self.out.avg,
                            self.out.ngroups, stream)

    def result(self, stream=None) -> dict:
        tq.check(self.state, stream)
        r = self.out.host()
        k = r["keys"]
        if len(self.q.key.cols) == 2:
            r["keys"] = np.stack([k // self.q.key.mult, k % self.q.key.mult], axis=1)
        else:
            r["keys"] = k.reshape(-1, 1)
        return r


class JoinAgg:
    """sigma(dim) -> build -> probe(fact) with the group-by fused -> finalize."""

    def __init__(self, query, n_build_max: int, load_factor: float = 0.5, device="cuda", unique: bool = True):
        self.q = query
        self.lf = load_factor
        self.flags = tq.TQ_UNIQUE_KEYS if unique else 0
        self.bnames = referenced(query.build_preds, [])
        self.bpreds = plan_preds(self.bnames, query.build_preds)
        self.pnames = referenced(query.probe_preds, query.sums)
        self.ppreds = plan_preds(self.pnames, query.probe_preds)
        self.exprs = plan_exprs(self.pnames, query.sums)
        self.domain = query.domain
        self.nsum = len(query.sums)
        self.table = torch.empty(tq.join_table_bytes(n_build_max, load_factor), dtype=torch.uint8, device=device)
        tq.join_table_init(self.table)
        self.state = torch.empty(tq.groupby_state_bytes(self.domain, self.nsum), dtype=torch.uint8, device=device)
        self.out = GroupByResult(self.domain, self.nsum, device)

    def build(self, dim: Dict[str, torch.Tensor], n: Optional[int] = None, skip: int = 0, stream=None):
        keys = dim[self.q.build_key]
        n = keys.numel() if n is None else n
        tq.join_build(self.table, keys, dim[self.q.build_payload], n, [dim[c] for c in self.bnames], self.bpreds,
                      self.lf, skip, self.flags, stream)

    def probe(self, fact: Dict[str, torch.Tensor], n: Optional[int] = None, stream=None):
        keys = fact[self.q.probe_key]
        n = keys.numel() if n is None else n
        tq.join_probe(self.table, keys, n, [fact[c] for c in self.pnames], self.ppreds,
                      agg=(self.state, self.domain, self.exprs), stream=stream)

    def init_state(self, stream=None):
        tq.groupby_init(self.state, self.domain, self.nsum, stream)

    def finalize(self, stream=None, reset=False):
        """reset=True leaves the state empty, so the next query needs no init_state()."""
        tq.groupby_finalize(self.state, self.out.keys, self.out.count, self.out.sums, self.out.avg,
                            self.out.ngroups, stream, reset=reset)

    def run(self, dim, fact, stream=None):
        self.init_state(stream)
        self.build(dim, stream=stream)
        self.probe(fact, stream=stream)
        self.finalize(stream)

    def result(self, stream=None) -> dict:
        tq.check(self.table, stream)
        tq.check(self.state, stream)
        r = self.out.host()
        r["keys"] = r["keys"].reshape(-1, 1)
        r["join_rows"] = int(r["count"].sum())  # every match lands in exactly one group
        return r


class OocJoinAgg:
    """The out-of-core join + aggregate over page-pool tables (tq_ooc_join_agg).

    keep_all: carry every fact column through the exchange (as a generic
    exchange that does not know which columns the join needs would); else only
    the key and the columns the sums read. exchange: "auto" (the Adaptive
    Exchange chooses one table or hash partitioning from an estimate taken on
    the first dimension batches), "partitioned" or "single"."""

    def __init__(self, query, dim_table, fact_table, budget_bytes: int, log2_fanout: int = 8,
                 load_factor: float = 0.5, chunk_bytes: int = 4 << 20, nslots: int = 3, keep_all: bool = True,
                 unique: bool = True, exchange: str = "auto", device="cuda"):
        self.q = query
        self.dim, self.fact = dim_table, fact_table
        dn, fn = dim_table.names, fact_table.names
        self._preds = tq.preds([(dn.index(p.col), p.lo, p.hi) for p in query.build_preds])
        self._sums = tq.exprs([[(-1 if f.col is None else fn.index(f.col), f.sign, f.add) for f in e]
                               for e in query.sums])
        keep = (1 << len(fn)) - 1 if keep_all else 0
        keep |= 1 << fn.index(query.probe_key)
        for e in query.sums:
            for f in e:
                if f.col is not None:
                    keep |= 1 << fn.index(f.col)
        self.plan = tq.OocPlan(dn.index(query.build_key), dn.index(query.build_payload),
                               ctypes.cast(self._preds, ctypes.POINTER(tq.PredS)), len(query.build_preds),
                               fn.index(query.probe_key), keep, ctypes.cast(self._sums, ctypes.POINTER(tq.ExprS)),
                               len(query.sums), query.domain, log2_fanout, load_factor,
                               tq.TQ_UNIQUE_KEYS if unique else 0, chunk_bytes, nslots,
                               tq.EXCHANGE_MODES[exchange])
        self.budget = tq.Budget(budget_bytes)
        self.domain, self.nsum = query.domain, len(query.sums)
        # the group-by state and its outputs live outside the budgeted workspace
        self.state = torch.empty(tq.groupby_state_bytes(self.domain, self.nsum), dtype=torch.uint8, device=device)
        self.out = GroupByResult(self.domain, self.nsum, device)
        self.work = torch.empty(budget_bytes, dtype=torch.uint8, device=device)
        self.copy_stream = torch.cuda.Stream()
        self.stats = None

    def run(self):
        stream = torch.cuda.current_stream()
        tq.groupby_init(self.state, self.domain, self.nsum, stream)
        self.stats = tq.ooc_join_agg(self.dim.pool, self.dim.c_batches(), self.fact.c_batches(), self.plan,
                                     self.budget, self.work, self.state, self.copy_stream, stream)
        tq.groupby_finalize(self.state, self.out.keys, self.out.count, self.out.sums, self.out.avg, self.out.ngroups,
                            stream)
        return self.stats

    def result(self) -> dict:
        tq.check(self.state)
        r = self.out.host()
        r["keys"] = r["keys"].reshape(-1, 1)
        r["join_rows"] = int(r["count"].sum())
        return r


def _align(x: int, a: int = 256) -> int:
    return (x + a - 1) // a * a


class BatchedJoinAgg:
    """Many join + group-by instances of one query shape (tq_batched_*).

    instances: list of (dim table, fact table, domain) as numpy dicts;
    params: per instance (load_factor, build_tile, probe_tile), e.g. from the
    autotuner. All device memory is one torch allocation carved into columns,
    tables, states and outputs."""

    def __init__(self, query, instances, params, device="cuda", unique: bool = True):
        self.q = query
        self.dnames = referenced(query.build_preds, [], [query.build_key, query.build_payload])
        self.fnames = referenced([], query.sums, [query.probe_key])
        assert len(self.dnames) <= 4 and len(self.fnames) <= 4
        Q = tq.BatchQuery()
        d0, f0, _ = instances[0]
        for i, c in enumerate(self.dnames):
            Q.dim_types[i] = tq._TYPE[torch.from_numpy(d0[c][:0]).dtype]
        Q.ndim = len(self.dnames)
        for j, p in enumerate(query.build_preds):
            Q.preds[j] = tq.PredS(self.dnames.index(p.col), p.lo, p.hi)
        Q.np = len(query.build_preds)
        for i, c in enumerate(self.fnames):
            Q.fact_types[i] = tq._TYPE[torch.from_numpy(f0[c][:0]).dtype]
        Q.nfact = len(self.fnames)
        for j, e in enumerate(query.sums):
            Q.sums[j].nf = len(e)
            for k, f in enumerate(e):
                Q.sums[j].f[k] = tq.FactorS(-1 if f.col is None else self.fnames.index(f.col), f.sign, f.add)
        Q.nsum = len(query.sums)
        Q.join_flags = tq.TQ_UNIQUE_KEYS if unique else 0
        self.Q = Q
        nsum = Q.nsum
        # carve one allocation
        plan, total = [], 0

        def take(nbytes):
            nonlocal total
            off = total
            total = _align(total + max(int(nbytes), 1))
            return off

        for (d, f, domain), (lf, bt, pt) in zip(instances, params):
            nd, nf = len(d[self.dnames[0]]), len(f[self.fnames[0]])
            e = {"dcols": [take(d[c].nbytes) for c in self.dnames], "fcols": [take(f[c].nbytes) for c in self.fnames],
                 "table": take(tq.join_table_bytes(nd, lf)), "tbytes": tq.join_table_bytes(nd, lf),
                 "state": take(tq.batched_state_bytes(domain, nsum)), "sbytes": tq.batched_state_bytes(domain, nsum),
                 "keys": take(domain * 8), "count": take(domain * 8), "sums": take(domain * nsum * 8),
                 "avg": take(domain * nsum * 8), "ng": take(8), "nd": nd, "nf": nf, "domain": domain,
                 "lf": lf, "bt": bt, "pt": pt}
            plan.append(e)
        self.arena = torch.empty(total, dtype=torch.uint8, device=device)
        base = self.arena.data_ptr()
        self.insts = (tq.Instance * len(instances))()
        uploads = []  # (arena offset, column): only the columns come from the host;
        # tables, states and outputs are set up on the device
        for i, ((d, f, domain), e) in enumerate(zip(instances, plan)):
            I = self.insts[i]
            for j, c in enumerate(self.dnames):
                uploads.append((e["dcols"][j], d[c]))
                I.dim_cols[j] = base + e["dcols"][j]
            for j, c in enumerate(self.fnames):
                uploads.append((e["fcols"][j], f[c]))
                I.fact_cols[j] = base + e["fcols"][j]
            I.n_dim, I.n_fact, I.domain = e["nd"], e["nf"], domain
            I.d_table, I.table_bytes = base + e["table"], e["tbytes"]
            I.d_state, I.state_bytes = base + e["state"], e["sbytes"]
            I.d_keys, I.d_count, I.d_sums = base + e["keys"], base + e["count"], base + e["sums"]
            I.d_avg, I.d_ngroups = base + e["avg"], base + e["ng"]
            I.load_factor, I.build_tile, I.probe_tile = e["lf"], e["bt"], e["pt"]
        self._upload(uploads)
        self.plan = plan
        self.n = len(instances)
        self.nsum = nsum
        self.input_bytes = sum(len(self.dnames) * 8 * e["nd"] + len(self.fnames) * 8 * e["nf"] for e in plan)
        self.work = torch.empty(max(1, tq.batched_work_bytes(self.insts)), dtype=torch.uint8, device=device)
        tq.batched_prepare(self.Q, self.insts, self.work)

    def _upload(self, uploads, stage_bytes=64 << 20):
        """Copies the columns into the arena through one reusable pinned
        buffer (a pinned copy of the whole arena would be tens of GB)."""
        stage = torch.empty(stage_bytes, dtype=torch.uint8, pin_memory=True)
        sb = stage.data_ptr()
        batch, fill = [], 0

        def flush():
            for off, n, at in batch:
                self.arena[off:off + n].copy_(stage[at:at + n], non_blocking=True)
            torch.cuda.synchronize()  # the buffer is refilled next
            batch.clear()

        for off, col in uploads:
            a = np.ascontiguousarray(col)
            n, pos = a.nbytes, 0
            while pos < n:
                k = min(n - pos, stage_bytes - fill)
                ctypes.memmove(sb + fill, a.ctypes.data + pos, k)
                batch.append((off + pos, k, fill))
                fill, pos = fill + k, pos + k
                if fill == stage_bytes:
                    flush()
                    fill = 0
        if batch:
            flush()

    def set_params(self, params, device="cuda"):
        """New (load_factor, build_tile, probe_tile) per instance; the tables were
        sized for the load factors given at construction, so a load factor may
        only grow."""
        for i, (lf, bt, pt) in enumerate(params):
            I = self.insts[i]
            if tq.join_table_bytes(I.n_dim, lf) > I.table_bytes:
                raise ValueError("the table was sized for a larger load factor")
            I.load_factor, I.build_tile, I.probe_tile = lf, bt, pt
        need = tq.batched_work_bytes(self.insts)
        if need > self.work.numel():
            self.work = torch.empty(need, dtype=torch.uint8, device=device)
        tq.batched_prepare(self.Q, self.insts, self.work)

    def run(self, stream=None):
        tq.batched_run(self.Q, self.work, self.n, stream)

    def run_per_instance(self, stream=None):
        tq.batched_run_per_instance(self.Q, self.insts, stream)

    def check(self, stream=None):
        tq.batched_check(self.work, stream)

    def results(self, which=None):
        """Outputs of the instances in `which` (default all), copied per instance."""
        torch.cuda.synchronize()
        out = []
        for i in (range(self.n) if which is None else which):
            e = self.plan[i]
            g = int(self.arena[e["ng"]:e["ng"] + 8].cpu().numpy().view(np.int64)[0])
            ns = self.nsum

            def grab(off, nbytes, dt):
                return self.arena[off:off + nbytes].cpu().numpy().view(dt)
            out.append({"keys": grab(e["keys"], 8 * g, np.int64).reshape(-1, 1),
                        "count": grab(e["count"], 8 * g, np.int64),
                        "sums": grab(e["sums"], 8 * g * ns, np.int64).reshape(g, ns),
                        "avg": grab(e["avg"], 8 * g * ns, np.float64).reshape(g, ns)})
        return out


class ServingSetup:
    """Base tables for the three request shapes and the request -> window mapping.

    shape 0: a filter + group-by table in device memory (n0 rows)
    shape 1: a dimension (n_dim rows) and a fact table (n1 rows) in device memory
    shape 2: the same dimension, and a fact table in page-pool batches (n2 rows)
    A request of n fact rows reads a seeded window of its shape's base tables;
    join requests read a dimension window of n / 4 rows."""

    def __init__(self, n0, n_dim, n1, n2, batch_rows, pool, seed=None, device="cuda", load_factor=0.5, nslots=3,
                 estimate=True, dim_sorted_by=None):
        from .datagen import workloads as wl
        from .hosttable import HostTable
        seed = wl.SERVE_SEED if seed is None else seed
        self.wl = wl
        self.fg = wl.filter_groupby_tables(n0, seed=seed + 10)
        self.dim, self.fact = wl.join_agg_tables(n_dim, n1, seed=seed + 11)
        if dim_sorted_by is not None:  # a dimension whose windows keep very different fractions
            order = np.argsort(self.dim[dim_sorted_by], kind="stable")
            self.dim = {k: v[order] for k, v in self.dim.items()}
        self.hdim, self.hfact = wl.ooc_tables_numpy(n2, n_dim, seed=seed + 12)
        self.fg_dev = to_device(self.fg, device)
        self.dim_dev = to_device(self.dim, device)
        self.fact_dev = to_device(self.fact, device)
        self.batch_rows = batch_rows
        self.host = HostTable(pool, wl.OOC_FACT_COLS, n2, batch_rows)
        self.host.fill_numpy(self.hfact)
        self.n0, self.n_dim, self.n1, self.n2 = n0, n_dim, n1, n2
        q0, q1 = wl.FILTER_GROUPBY_QUERY, wl.JOIN_AGG_QUERY
        self.q0, self.q1 = q0, q1
        T = tq.ServeTables()
        names0 = referenced(q0.preds, q0.sums, q0.key.cols)
        for i, c in enumerate(names0):
            T.fg_cols[i] = tq.col(self.fg_dev[c])
        T.fg_ncol = len(names0)
        for j, (c, lo, hi) in enumerate(plan_preds(names0, q0.preds)):
            T.fg_preds[j] = tq.PredS(c, lo, hi)
        T.fg_np = len(q0.preds)
        T.fg_key = tq.gkey([names0.index(c) for c in q0.key.cols], q0.key.mult)
        for j, e in enumerate(plan_exprs(names0, q0.sums)):
            T.fg_sums[j].nf = len(e)
            for k, (c, s, a) in enumerate(e):
                T.fg_sums[j].f[k] = tq.FactorS(c, s, a)
        T.fg_nsum, T.fg_domain = len(q0.sums), q0.key.domain
        dnames = referenced(q1.build_preds, [], [q1.build_key, q1.build_payload])
        for i, c in enumerate(dnames):
            T.dim_cols[i] = tq.col(self.dim_dev[c])
        T.dim_ncol = len(dnames)
        for j, p in enumerate(q1.build_preds):
            T.dim_preds[j] = tq.PredS(dnames.index(p.col), p.lo, p.hi)
        T.dim_np = len(q1.build_preds)
        fnames = referenced([], q1.sums, [q1.probe_key])
        for i, c in enumerate(fnames):
            T.fact_cols[i] = tq.col(self.fact_dev[c])
            T.fact_map[i] = self.host.col_index(c)
        T.fact_ncol = len(fnames)
        for j, e in enumerate(plan_exprs(fnames, q1.sums)):
            T.join_sums[j].nf = len(e)
            for k, (c, s, a) in enumerate(e):
                T.join_sums[j].f[k] = tq.FactorS(c, s, a)
        T.join_nsum, T.join_domain, T.load_factor = len(q1.sums), q1.domain, load_factor
        self._batches = self.host.c_batches()
        T.pool = pool.h
        T.fact_batches = ctypes.cast(self._batches[0], ctypes.c_void_p)
        T.n_fact_batches = len(self.host.batches)
        T.nslots = nslots
        T.estimate = 1 if estimate else 0
        T.fg_rows, T.dim_rows, T.fact_rows = n0, n_dim, n1
        self.T = T

    def requests(self, reqs, time_scale=1.0):
        """tq_request array for workload Request objects (shape, n_fact, arrival)."""
        out = (tq.Request * max(1, len(reqs)))()
        rng = np.random.default_rng(12345)
        for i, r in enumerate(reqs):
            q = out[i]
            q.shape, q.arrival_s = r.shape, r.arrival_s * time_scale
            if r.shape == 0:
                n = min(r.n_fact, self.n0)
                q.fact_first, q.n_fact = int(rng.integers(0, self.n0 - n + 1)) // 16 * 16, n
            elif r.shape == 1:
                n = min(r.n_fact, self.n1)
                q.fact_first, q.n_fact = int(rng.integers(0, self.n1 - n + 1)) // 16 * 16, n
            else:
                nb = min(max(1, -(-r.n_fact // self.batch_rows)), len(self.host.batches))
                q.fact_first, q.n_fact = int(rng.integers(0, len(self.host.batches) - nb + 1)), nb
                n = nb * self.batch_rows
            if r.shape != 0:
                nd = max(1, min(n // 4, self.n_dim))
                q.dim_first, q.n_dim = int(rng.integers(0, self.n_dim - nd + 1)) // 16 * 16, nd
        return out


class NullableGroupByResult:
    """Outputs of tq_groupby_finalize_nullable: domain + 1 groups (the last key is NULL)."""

    def __init__(self, domain: int, nsum: int, device):
        g = domain + 1
        self.domain = domain
        self.keys = torch.empty(g, dtype=torch.int64, device=device)
        self.count = torch.empty(g, dtype=torch.int64, device=device)
        self.sums = torch.empty(g * max(nsum, 1), dtype=torch.int64, device=device)
        self.nonnull = torch.empty(g * max(nsum, 1), dtype=torch.int64, device=device)
        self.avg = torch.empty(g * max(nsum, 1), dtype=torch.float64, device=device)
        self.ngroups = torch.zeros(1, dtype=torch.int64, device=device)
        self.nsum = nsum

    def host(self) -> dict:
        g = int(self.ngroups.item())
        k = self.keys[:g].cpu().numpy()
        ns = self.nsum
        return {"keys": np.where(k == self.domain, 0, k), "key_null": k == self.domain,
                "count": self.count[:g].cpu().numpy(),
                "sums": self.sums[: g * ns].cpu().numpy().reshape(g, ns),
                "nonnull": self.nonnull[: g * ns].cpu().numpy().reshape(g, ns),
                "avg": self.avg[: g * ns].cpu().numpy().reshape(g, ns)}


class NullableFilterGroupBy:
    """sigma + pi + gamma under NULL semantics (one key column). `valid` maps a
    column name to a device validity bitmap (uint8 tensor); others have no NULLs."""

    def __init__(self, query, device="cuda"):
        assert len(query.key.cols) == 1
        self.q = query
        self.names = referenced(query.preds, query.sums, query.key.cols)
        self.preds = plan_preds(self.names, query.preds)
        self.exprs = plan_exprs(self.names, query.sums)
        self.key = tq.gkey([_col_index(self.names, query.key.cols[0])], 1)
        self.domain = query.key.domain
        self.nsum = len(query.sums)
        self.state = torch.empty(tq.groupby_state_bytes_nullable(self.domain, self.nsum), dtype=torch.uint8,
                                 device=device)
        self.out = NullableGroupByResult(self.domain, self.nsum, device)

    def run(self, table, valid, nrows=None, stream=None):
        cols = [table[c] for c in self.names]
        vals = [valid.get(c) if valid else None for c in self.names]
        n = cols[0].numel() if nrows is None else nrows
        tq.groupby_init_nullable(self.state, self.domain, self.nsum, stream)
        tq.groupby_agg_nullable(self.state, self.domain, cols, vals, n, self.preds, self.key, self.exprs, stream)
        o = self.out
        tq.groupby_finalize_nullable(self.state, o.keys, o.count, o.sums, o.nonnull, o.avg, o.ngroups, stream)

    def result(self, stream=None) -> dict:
        tq.check(self.state, stream)
        return self.out.host()


class NullableJoinAgg:
    """join + aggregate under NULL semantics: NULL keys match nothing, a NULL
    build payload is the NULL group, a NULL probe value skips the sums reading it."""

    def __init__(self, query, n_build_max: int, load_factor: float = 0.5, device="cuda", unique: bool = True):
        self.q = query
        self.lf = load_factor
        self.flags = tq.TQ_UNIQUE_KEYS if unique else 0
        self.bnames = referenced(query.build_preds, [])
        self.bpreds = plan_preds(self.bnames, query.build_preds)
        self.pnames = referenced(query.probe_preds, query.sums)
        self.ppreds = plan_preds(self.pnames, query.probe_preds)
        self.exprs = plan_exprs(self.pnames, query.sums)
        self.domain = query.domain
        self.nsum = len(query.sums)
        self.table = torch.empty(tq.join_table_bytes(n_build_max, load_factor), dtype=torch.uint8, device=device)
        tq.join_table_init(self.table)
        self.state = torch.empty(tq.groupby_state_bytes_nullable(self.domain, self.nsum), dtype=torch.uint8,
                                 device=device)
        self.out = NullableGroupByResult(self.domain, self.nsum, device)

    def run(self, dim, dvalid, fact, fvalid, stream=None):
        dv = dvalid or {}
        fv = fvalid or {}
        q = self.q
        keys = dim[q.build_key]
        tq.groupby_init_nullable(self.state, self.domain, self.nsum, stream)
        tq.join_build_nullable(self.table, keys, dv.get(q.build_key), dim[q.build_payload], dv.get(q.build_payload),
                               keys.numel(), [dim[c] for c in self.bnames], [dv.get(c) for c in self.bnames],
                               self.bpreds, self.lf, 0, self.flags, stream)
        pk = fact[q.probe_key]
        tq.join_probe_nullable(self.table, pk, fv.get(q.probe_key), pk.numel(), [fact[c] for c in self.pnames],
                               [fv.get(c) for c in self.pnames], self.ppreds, (self.state, self.domain, self.exprs),
                               stream)
        o = self.out
        tq.groupby_finalize_nullable(self.state, o.keys, o.count, o.sums, o.nonnull, o.avg, o.ngroups, stream)

    def result(self, stream=None) -> dict:
        tq.check(self.table, stream)
        tq.check(self.state, stream)
        r = self.out.host()
        r["join_rows"] = int(r["count"].sum())
        return r


class StringJoinAgg:
    """join + aggregate on a dictionary-encoded string key. The dimension's key
    column holds int32 codes into `build_dict`, the fact's into `probe_dict`
    (each an (offsets, data) pair of device tensors; the build dictionary's
    entries are distinct). tq_dict_unify maps the probe dictionary onto the
    build one, tq_dict_keys turns both code columns into int64 join keys, and
    the join runs as NullableJoinAgg (NULL codes match nothing)."""

    def __init__(self, query, n_build_max: int, n_probe_max: int, n_build_dict_max: int, n_probe_dict_max: int,
                 load_factor: float = 0.5, device="cuda"):
        self.q = query
        self.join = NullableJoinAgg(query, n_build_max, load_factor, device)
        self.dtable = torch.empty(tq.join_table_bytes(max(n_build_dict_max, 1), 0.5), dtype=torch.uint8,
                                  device=device)
        self.scratch = torch.empty(tq.dict_unify_scratch_bytes(n_build_dict_max), dtype=torch.uint8, device=device)
        self.remap = torch.empty(max(n_probe_dict_max, 1), dtype=torch.int32, device=device)
        self.bkeys = torch.empty(max(n_build_max, 1), dtype=torch.int64, device=device)
        self.pkeys = torch.empty(max(n_probe_max, 1), dtype=torch.int64, device=device)

    def run(self, build_dict, probe_dict, dim, dvalid, fact, fvalid, stream=None):
        q = self.q
        dv, fv = dvalid or {}, fvalid or {}
        npd = probe_dict[0].numel() - 1
        remap = self.remap[:npd]
        tq.dict_unify(self.dtable, build_dict, probe_dict, self.scratch, remap, stream)
        nb = dim[q.build_key].numel()
        nf = fact[q.probe_key].numel()
        bk, pk = self.bkeys[:nb], self.pkeys[:nf]
        tq.dict_keys(dim[q.build_key], dv.get(q.build_key), nb, None, bk, stream)
        tq.dict_keys(fact[q.probe_key], fv.get(q.probe_key), nf, remap, pk, stream)
        self.join.run(dict(dim, **{q.build_key: bk}), dv, dict(fact, **{q.probe_key: pk}), fv, stream)

    def result(self, stream=None) -> dict:
        tq.check(self.dtable, stream)
        return self.join.result(stream)


class ParquetScan:
    """Scan of a Parquet file's columns into device tensors: tq_parquet_preload
    (byte ranges merged and read into pool pages by a host thread), then
    tq_parquet_decode (pages copied to the device and decoded there). The
    work buffer grows to the largest preload seen; outputs are new tensors.
    read_pipelined decodes successive row groups on `pipe_streams` streams in
    turn (the caller's and its own), each with its own work buffer, so that
    one row group's kernels run beside the next one's copies and kernels."""

    def __init__(self, path: str, columns, pool, merge_gap: int = 1 << 20, device="cuda", pipe_streams: int = 4):
        self.file = tq.ParquetFile(path)
        meta = self.file.columns()
        names = [m[0] for m in meta]
        self.cols = [names.index(c) for c in columns]
        self.meta = [meta[c] for c in self.cols]
        self.names = list(columns)
        self.pool = pool
        self.merge_gap = merge_gap
        self.device = device
        self.work = None
        if pipe_streams < 1:
            raise ValueError("pipe_streams must be at least 1")
        self.pipe_streams = [torch.cuda.Stream(device=device) for _ in range(pipe_streams - 1)]
        self.pipe_works = [None] * (pipe_streams - 1)  # each allocated on its stream
        self.last_works = []  # the work buffers of the last read, for check()

    def preload(self, rg0: int = 0, rg1=None):
        rg1 = self.file.num_row_groups if rg1 is None else rg1
        return self.file.preload(self.pool, rg0, rg1, self.cols, self.merge_gap)

    def decode(self, pl, stream=None):
        """Decodes a preload; returns ({name: values}, {name: validity bitmap or None})."""
        need = pl.work_bytes()
        if self.work is None or self.work.numel() < need:
            self.work = torch.empty(need, dtype=torch.uint8, device=self.device)
        n = pl.rows
        data, valid, outs = {}, {}, []
        for name, (_, t, nullable) in zip(self.names, self.meta):
            d = torch.empty(max(n, 1), dtype=torch.int64 if t == tq.TQ_I64 else torch.int32, device=self.device)
            v = torch.empty(max(((n + 31) // 32) * 4, 4), dtype=torch.uint8, device=self.device) if nullable else None
            data[name], valid[name] = d[:n], v
            outs.append((d, v))
        pl.decode(self.work, outs, stream)
        self.last_works = [self.work]
        return data, valid

    def read_pipelined(self, stream=None):
        """Every row group into one set of columns, the next row group's bytes
        read ahead (its preload started) while the current one is decoded:
        the host reads overlap the copies and kernels. Row groups must start
        on multiples of 32 rows when a column is nullable (bitmap words)."""
        nrg = self.file.num_row_groups
        n = self.file.num_rows
        data, valid = {}, {}
        for name, (_, t, nullable) in zip(self.names, self.meta):
            data[name] = torch.empty(max(n, 1), dtype=torch.int64 if t == tq.TQ_I64 else torch.int32,
                                     device=self.device)
            valid[name] = (torch.empty(max(((n + 31) // 32) * 4, 4), dtype=torch.uint8, device=self.device)
                           if nullable else None)
        if nrg == 0:
            return {k: v[:0] for k, v in data.items()}, valid
        main = torch.cuda.current_stream(self.device) if stream is None else stream
        side = self.pipe_streams[:max(0, min(len(self.pipe_streams), nrg - 1))]
        for s_ in side:
            s_.wait_stream(main)  # the outputs were allocated on the caller's stream
        nxt = self.preload(0, 1)
        row = 0
        self.last_works = []
        for g in range(nrg):
            cur = nxt
            nxt = self.preload(g + 1, g + 2) if g + 1 < nrg else None
            need = cur.work_bytes()
            k = g % (len(side) + 1)
            st = main if k == 0 else side[k - 1]
            if k == 0:
                if self.work is None or self.work.numel() < need:
                    self.work = torch.empty(need, dtype=torch.uint8, device=self.device)
                work = self.work
            else:
                if self.pipe_works[k - 1] is None or self.pipe_works[k - 1].numel() < need:
                    with torch.cuda.stream(st):  # freed and reused in this stream's order
                        self.pipe_works[k - 1] = None
                        self.pipe_works[k - 1] = torch.empty(need, dtype=torch.uint8, device=self.device)
                work = self.pipe_works[k - 1]
            rows = cur.rows
            if any(v is not None for v in valid.values()) and row % 32:
                raise ValueError("a row group of a nullable column starts off a 32-row boundary")
            outs = [(data[name][row:row + rows], None if valid[name] is None else valid[name][row // 8:])
                    for name in self.names]
            cur.decode(work, outs, st)
            if all(w is not work for w in self.last_works):
                self.last_works.append(work)
            cur.free()
            row += rows
        for s_ in side:
            main.wait_stream(s_)
        for name in self.names:  # used on the side streams: not reused before their work is done
            for s_ in side:
                data[name].record_stream(s_)
                if valid[name] is not None:
                    valid[name].record_stream(s_)
        return {k: v[:n] for k, v in data.items()}, valid

    def read(self, rg0: int = 0, rg1=None, stream=None):
        pl = self.preload(rg0, rg1)
        try:
            return self.decode(pl, stream)
        finally:
            pl.free()

    def check(self, stream=None):
        """Raises the error a kernel of the last decode or read latched."""
        for w in self.last_works:
            tq.check(w, stream)


class StringGroupBy:
    """GROUP BY a plain (not dictionary-encoded) string column: tq_dict_encode
    gives every distinct string a code, the group-by runs on the codes, and
    the result's keys are the first rows of their strings."""

    def __init__(self, n_max: int, sums, device="cuda"):
        self.scratch = torch.empty(tq.dict_encode_scratch_bytes(n_max), dtype=torch.uint8, device=device)
        self.codes = torch.empty(max(n_max, 1), dtype=torch.int32, device=device)
        self.first = torch.empty(max(n_max, 1), dtype=torch.int32, device=device)
        self.ndict = torch.zeros(1, dtype=torch.int64, device=device)
        self.sums = sums
        self.device = device

    def run(self, column, values: Dict[str, torch.Tensor], stream=None):
        """column: (offsets, data); values: the columns the sums read. Returns
        the group-by result with 'first_row' (the smallest row of each group's
        string) in place of keys."""
        from .datagen.workloads import FilterGroupByQuery, GroupKey
        n = column[0].numel() - 1
        tq.dict_encode(column, self.scratch, self.codes[:n], self.first[:n], self.ndict, stream)
        nd = int(self.ndict.item())  # the domain of the codes
        if nd < 0:
            raise tq.TqError(tq.TQ_EINVAL, "more than 16 distinct strings share one hash")
        q = FilterGroupByQuery(preds=[], key=GroupKey(("__code",), 1, max(nd, 1)), sums=self.sums,
                               avg_of=list(range(len(self.sums))))
        fg = FilterGroupBy(q, self.device)
        fg.run(dict(values, __code=self.codes[:n]), n, stream)
        r = fg.result(stream)
        r["first_row"] = self.first[:max(nd, 1)].cpu().numpy()[r["keys"][:, 0]]
        return r
