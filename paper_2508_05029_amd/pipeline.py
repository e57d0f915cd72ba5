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

    def finalize(self, stream=None):
        tq.groupby_finalize(self.state, self.out.keys, self.out.count, self.out.sums, self.out.avg,
                            self.out.ngroups, stream)

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
    the key and the columns the sums read."""

    def __init__(self, query, dim_table, fact_table, budget_bytes: int, log2_fanout: int = 8,
                 load_factor: float = 0.5, chunk_bytes: int = 4 << 20, nslots: int = 3, keep_all: bool = True,
                 unique: bool = True, device="cuda"):
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
                               tq.TQ_UNIQUE_KEYS if unique else 0, chunk_bytes, nslots)
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
