"""Synthetic workloads: table recipes and query descriptions as plain data.

The paper measures on TPC-H / TPC-DS Parquet files; none of those suites is
reproduced here. These seeded tables stand in for them with the column types,
value ranges and join shapes that the five workload descriptions fix:

  filter_groupby   1M-row fact table, date filter, group by two flags
  join_agg         1.5M-row dimension x 6M-row fact, date window, group by dim group
  ooc_join_agg     600M-row fact / 150M-row dimension streamed from pinned pages
  batched          4,096 uneven join+group-by instances, Zipf(1.1) group skew
  serving          Poisson arrivals of requests of the three shapes above
  string keys      dictionary-encoded string join keys (two dictionaries)

A query is described by predicates (inclusive integer ranges, conjunctive),
product expressions of affine factors, and a group key. The descriptions are
data; evaluating them is the job of the oracle and of the GPU path.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

from . import (log2_uniform, log_uniform, permutation, sequence, uniform, zipf, zipf_cdf,
               exponential, unit)

SEED_BASE = 2508050290
I64_MIN = -(2 ** 63)
I64_MAX = 2 ** 63 - 1


@dataclass(frozen=True)
class Pred:
    """lo <= col <= hi (inclusive, on the value widened to int64)."""
    col: str
    lo: int
    hi: int


@dataclass(frozen=True)
class Factor:
    """sign * col + add; col None means the constant ``add``."""
    col: Optional[str]
    sign: int = 1
    add: int = 0


Expr = Tuple[Factor, ...]  # product of factors, int64 arithmetic mod 2^64


@dataclass(frozen=True)
class GroupKey:
    """key = c0 * mult + c1 (or c0 alone); keys must lie in [0, domain)."""
    cols: Tuple[str, ...]
    mult: int
    domain: int


@dataclass
class FilterGroupByQuery:
    preds: List[Pred]
    key: GroupKey
    sums: List[Expr]
    avg_of: List[int]  # indices into sums whose AVG is reported


@dataclass
class JoinAggQuery:
    build_key: str
    build_payload: str  # group id carried by the build side
    build_preds: List[Pred]
    probe_key: str
    probe_preds: List[Pred]
    sums: List[Expr]  # over probe-side columns
    domain: int  # group ids lie in [0, domain)
    avg_of: List[int] = field(default_factory=list)


def col(name: str) -> Factor:
    return Factor(name, 1, 0)


# ---------------------------------------------------------------------------
# filter + group-by over a 1M-row fact table

FG_DATE_MAX = 2436

FILTER_GROUPBY_QUERY = FilterGroupByQuery(
    preds=[Pred("date", I64_MIN, FG_DATE_MAX)],
    key=GroupKey(("flagA", "flagB"), 2, 6),
    sums=[
        (col("qty"),),
        (col("price"),),
        (col("price"), Factor("disc", -1, 100)),
        (col("price"), Factor("disc", -1, 100), Factor("tax", 1, 100)),
        (col("disc"),),
    ],
    avg_of=[0, 1, 4],
)

FACT_COLUMNS = {  # name -> (dtype, lo, hi)
    "date": (np.int32, 0, 2525),
    "qty": (np.int64, 1, 50),
    "price": (np.int64, 90_000, 10_500_000),
    "disc": (np.int64, 0, 10),
    "tax": (np.int64, 0, 8),
    "flagA": (np.uint8, 0, 2),
    "flagB": (np.uint8, 0, 1),
}


def filter_groupby_tables(n: int = 1_000_000, seed: int = SEED_BASE + 0) -> Dict[str, np.ndarray]:
    t = {"key": sequence(n)}
    for j, (name, (dt, lo, hi)) in enumerate(FACT_COLUMNS.items()):
        t[name] = uniform(n, lo, hi, dt, seed, 1 + j)
    return t


# ---------------------------------------------------------------------------
# dimension x fact join + aggregate

JA_WINDOW = (730, 1094)  # 365 days out of 0..2405
JA_GROUPS = 25

JOIN_AGG_QUERY = JoinAggQuery(
    build_key="key", build_payload="group",
    build_preds=[Pred("date", *JA_WINDOW)],
    probe_key="fk", probe_preds=[],
    sums=[(col("price"), Factor("disc", -1, 100))],
    domain=JA_GROUPS,
    avg_of=[0],
)


def dim_tables(n_dim: int, seed: int, int64_cols: bool = False, groups: int = JA_GROUPS,
               zipf_s: Optional[float] = None, stream0: int = 0) -> Dict[str, np.ndarray]:
    """Dimension: key = keyed permutation of [0, n_dim), group, date over 2,406 days."""
    gt = np.int64 if int64_cols else np.int32
    d = {"key": permutation(n_dim, seed, stream0 + 0)}
    if zipf_s is None:
        d["group"] = uniform(n_dim, 0, groups - 1, gt, seed, stream0 + 1)
    else:
        d["group"] = zipf(n_dim, groups, zipf_s, seed, stream0 + 1).astype(gt, copy=False)
    d["date"] = uniform(n_dim, 0, 2405, gt, seed, stream0 + 2)
    return d


def fact_tables(n_fact: int, n_dim: int, seed: int, extra: bool = False, stream0: int = 3) -> Dict[str, np.ndarray]:
    """Fact: fk uniform over the dimension keys, price and discount as above."""
    f = {"fk": uniform(n_fact, 0, n_dim - 1, np.int64, seed, stream0 + 0),
         "price": uniform(n_fact, 90_000, 10_500_000, np.int64, seed, stream0 + 1),
         "disc": uniform(n_fact, 0, 10, np.int64, seed, stream0 + 2)}
    if extra:
        f["qty"] = uniform(n_fact, 1, 50, np.int64, seed, stream0 + 3)
        f["tax"] = uniform(n_fact, 0, 8, np.int64, seed, stream0 + 4)
        f["date"] = uniform(n_fact, 0, 2525, np.int32, seed, stream0 + 5)
    return f


def join_agg_tables(n_dim: int = 1_500_000, n_fact: int = 6_000_000, seed: int = SEED_BASE + 1):
    return dim_tables(n_dim, seed), fact_tables(n_fact, n_dim, seed)


# ---------------------------------------------------------------------------
# out-of-core: 600M x 150M, generated batch by batch straight into pinned pages

OOC_FACT_ROWS = 600_000_000
OOC_DIM_ROWS = 150_000_000
OOC_FACT_COLS = [("fk", np.int64), ("price", np.int64), ("disc", np.int64), ("qty", np.int64),
                 ("tax", np.int64), ("date", np.int32)]
OOC_DIM_COLS = [("key", np.int64), ("group", np.int32), ("date", np.int32)]
OOC_SEED = SEED_BASE + 2


def ooc_fill_fact(name: str, addr: int, first: int, count: int, n_dim: int, seed: int = OOC_SEED):
    """Write rows [first, first+count) of fact column ``name`` to raw memory."""
    from . import uniform_into
    spec = {"fk": (np.int64, 0, n_dim - 1, 3), "price": (np.int64, 90_000, 10_500_000, 4),
            "disc": (np.int64, 0, 10, 5), "qty": (np.int64, 1, 50, 6), "tax": (np.int64, 0, 8, 7),
            "date": (np.int32, 0, 2525, 8)}[name]
    dt, lo, hi, stream = spec
    uniform_into(addr, dt, count, lo, hi, seed, stream, first)


def ooc_fill_dim(name: str, addr: int, first: int, count: int, n_dim: int, seed: int = OOC_SEED):
    from . import permutation_into, uniform_into
    if name == "key":
        permutation_into(addr, count, n_dim, seed, 0, first, 0)
    elif name == "group":
        uniform_into(addr, np.int32, count, 0, JA_GROUPS - 1, seed, 1, first)
    else:
        uniform_into(addr, np.int32, count, 0, 2405, seed, 2, first)


def ooc_tables_numpy(n_fact: int, n_dim: int, seed: int = OOC_SEED):
    """The same tables as the pinned-page generator, as numpy arrays (small sizes)."""
    f = {}
    for name, dt in OOC_FACT_COLS:
        a = np.empty(n_fact, dtype=dt)
        ooc_fill_fact(name, a.ctypes.data, 0, n_fact, n_dim, seed)
        f[name] = a
    d = {}
    for name, dt in OOC_DIM_COLS:
        a = np.empty(n_dim, dtype=dt)
        ooc_fill_dim(name, a.ctypes.data, 0, n_dim, n_dim, seed)
        d[name] = a
    return d, f


# ---------------------------------------------------------------------------
# batched: 4,096 uneven instances

BATCH_INSTANCES = 4096
BATCH_SEED = SEED_BASE + 3
ZIPF_S = 1.1


@dataclass
class InstanceShape:
    n_fact: int
    n_dim: int
    groups: int


def batched_shapes(count: int = BATCH_INSTANCES, seed: int = BATCH_SEED, fact_lo: float = 3.0,
                   fact_hi: float = 6.0) -> List[InstanceShape]:
    """n_fact = floor(10^(3 + 3U)) in [1e3, 1e6]; n_dim = n_fact // 4;
    groups = floor(4 * 2^(14 U')) in [4, 65536]."""
    nf = log_uniform(count, fact_lo, fact_hi, int(round(10 ** fact_lo)), int(round(10 ** fact_hi)), seed, 0)
    g = log2_uniform(count, 4.0, 14.0, 4, 65536, seed, 1)
    return [InstanceShape(int(a), max(1, int(a) // 4), int(b)) for a, b in zip(nf, g)]


def batched_instance_tables(i: int, shape: InstanceShape, seed: int = BATCH_SEED):
    s = seed + 7919 * (i + 1)
    d = dim_tables(shape.n_dim, s, int64_cols=True, groups=shape.groups, zipf_s=ZIPF_S)
    f = fact_tables(shape.n_fact, shape.n_dim, s)
    return d, f


def batched_query(groups: int) -> JoinAggQuery:
    return JoinAggQuery(build_key="key", build_payload="group", build_preds=[Pred("date", *JA_WINDOW)],
                        probe_key="fk", probe_preds=[],
                        sums=[(col("price"), Factor("disc", -1, 100))], domain=groups, avg_of=[0])


# ---------------------------------------------------------------------------
# serving: mixed requests

SERVE_SEED = SEED_BASE + 4


@dataclass
class Request:
    rid: int
    shape: int  # 0 filter+group-by, 1 in-device join, 2 host-streamed join
    n_fact: int
    arrival_s: float


def serving_requests(count: int, qps: float, seed: int = SERVE_SEED, fact_lo: float = 4.0,
                     fact_hi: float = 8.0) -> List[Request]:
    shapes = np.minimum((unit(count, seed, 0) * 3).astype(np.int64), 2)
    nf = log_uniform(count, fact_lo, fact_hi, int(round(10 ** fact_lo)), int(round(10 ** fact_hi)), seed, 1)
    gaps = exponential(count, qps, seed, 2)
    t = np.cumsum(gaps)
    return [Request(i, int(shapes[i]), int(nf[i]), float(t[i])) for i in range(count)]


# ---------------------------------------------------------------------------
# dictionary-encoded string keys

def strings_of(ids: np.ndarray, seed: int, stream: int, max_prefix: int = 20) -> Tuple[np.ndarray, np.ndarray]:
    """Arrow string column (int32 offsets, uint8 bytes) for entity ids: a
    lower-case prefix of 0..max_prefix letters drawn per id, '#', then the id
    in decimal. Distinct ids give distinct strings (the text after the last
    '#' is the id); equal ids give equal strings. Lengths 2..max_prefix + 20."""
    ids = np.asarray(ids, dtype=np.int64)
    n = len(ids)
    # draws indexed by id (not by position), so one id always spells one string
    top = int(ids.max()) + 1 if n else 1
    plen = uniform(top, 0, max_prefix, np.int64, seed, stream)
    letters = uniform(top * max_prefix, 97, 122, np.uint8, seed, stream + 1).reshape(top, max_prefix) \
        if max_prefix else np.zeros((top, 0), np.uint8)
    parts = [letters[x, :plen[x]].tobytes() + b"#" + str(x).encode() for x in ids.tolist()]
    offsets = np.zeros(n + 1, np.int32)
    offsets[1:] = np.cumsum([len(b) for b in parts], dtype=np.int64)
    data = np.frombuffer(b"".join(parts), dtype=np.uint8).copy() if n else np.zeros(0, np.uint8)
    return offsets, data


@dataclass
class StringJoinTables:
    build_dict: Tuple[np.ndarray, np.ndarray]  # distinct strings
    probe_dict: Tuple[np.ndarray, np.ndarray]  # distinct strings, a quarter of them absent from build_dict
    dim: Dict[str, np.ndarray]                 # key: int32 codes into build_dict (one row per entry)
    fact: Dict[str, np.ndarray]                # fk: int32 codes into probe_dict


def string_join_tables(n_dim: int, n_fact: int, seed: int = SEED_BASE + 5,
                       groups: int = 25) -> StringJoinTables:
    """join_agg's shape with string keys encoded against two dictionaries. The
    build dictionary spells entity ids [0, n_dim) in a keyed order, the probe
    dictionary ids [n_dim / 4, n_dim * 5 / 4) in another, so a quarter of the
    probe entries match nothing; the dimension's key codes are a permutation
    of the build dictionary, the fact's uniform over the probe dictionary."""
    q = n_dim // 4
    bids = permutation(n_dim, seed, 0)
    pids = permutation(n_dim, seed, 1) + q
    d = {"key": permutation(n_dim, seed, 2).astype(np.int32),
         "group": uniform(n_dim, 0, groups - 1, np.int32, seed, 3),
         "date": uniform(n_dim, 0, 2405, np.int32, seed, 4)}
    f = {"fk": uniform(n_fact, 0, max(n_dim - 1, 0), np.int32, seed, 5),
         "price": uniform(n_fact, 90_000, 10_500_000, np.int64, seed, 6),
         "disc": uniform(n_fact, 0, 10, np.int64, seed, 7)}
    return StringJoinTables(strings_of(bids, seed, 8), strings_of(pids, seed, 8), d, f)
