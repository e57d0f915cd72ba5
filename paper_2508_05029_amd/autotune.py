"""Autotuner for the batched join + group-by: tile sizes and load factor per
size bucket.

Instances are bucketed by fact-row decade and by whether their group domain
fits the dense LDS partials. For each bucket, a sample of its instances is
timed under candidate parameters by coordinate descent (load factor, then
probe tile, then build tile), each timing the median of a few runs of the
batched launches. Results are independent of these parameters (the tests
sweep them), so tuning only changes speed. Choices are cached in a JSON file
keyed by device and bucket.
"""
from __future__ import annotations

import json
import math
import os
from typing import Callable, Dict, List, Optional, Sequence, Tuple

import torch

from . import pipeline

DEFAULT = (0.5, 4096, 16384)
LOAD_FACTORS = (0.25, 0.5, 0.75)
PROBE_TILES = (4096, 16384, 65536)
BUILD_TILES = (1024, 4096, 16384)
DENSE_GROUPS = 2048  # group domains up to this size aggregate in dense LDS partials (1 sum)


def bucket_of(n_fact: int, groups: int) -> str:
    dec = int(math.floor(math.log10(max(n_fact, 1))))
    return f"f1e{dec}-{'dense' if groups <= DENSE_GROUPS else 'hash'}"


def _time_run(job: "pipeline.BatchedJoinAgg", reps: int) -> float:
    ts = []
    for _ in range(reps + 1):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        job.run()
        b.record()
        b.synchronize()
        ts.append(a.elapsed_time(b))
    ts = sorted(ts[1:])
    return ts[len(ts) // 2]


def tune_batched(query, instances: Sequence[Tuple[dict, dict, int]], cache_path: Optional[str] = None,
                 sample: int = 48, reps: int = 3, log: Callable[[str], None] = lambda s: None) -> Dict[str, tuple]:
    """Best (load_factor, build_tile, probe_tile) per bucket of `instances`."""
    device = torch.cuda.get_device_name(0)
    cache = {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as f:
            cache = json.load(f).get(device, {})
    buckets: Dict[str, List[int]] = {}
    for i, (d, f, g) in enumerate(instances):
        buckets.setdefault(bucket_of(len(f["fk"]), g), []).append(i)
    best: Dict[str, tuple] = {}
    for b, idx in sorted(buckets.items()):
        if b in cache:
            best[b] = tuple(cache[b])
            continue
        pick = [instances[i] for i in idx[:sample]]
        job = pipeline.BatchedJoinAgg(query, pick, [(min(LOAD_FACTORS),) + DEFAULT[1:]] * len(pick))
        cur = list(DEFAULT)
        for axis, values in ((0, LOAD_FACTORS), (2, PROBE_TILES), (1, BUILD_TILES)):
            scores = []
            for v in values:
                cand = list(cur)
                cand[axis] = v
                job.set_params([tuple(cand)] * len(pick))
                scores.append((_time_run(job, reps), v))
            cur[axis] = min(scores)[1]
            log(f"tune {b}: axis {axis} -> {cur[axis]} ({', '.join(f'{v}:{t:.3f}ms' for t, v in scores)})")
        best[b] = tuple(cur)
        del job
        torch.cuda.empty_cache()
    if cache_path:
        allc = {}
        if os.path.exists(cache_path):
            with open(cache_path) as f:
                allc = json.load(f)
        allc.setdefault(device, {}).update({k: list(v) for k, v in best.items()})
        with open(cache_path, "w") as f:
            json.dump(allc, f, indent=1)
    return best


def params_for(instances: Sequence[Tuple[dict, dict, int]], table: Dict[str, tuple]) -> List[tuple]:
    return [table.get(bucket_of(len(f["fk"]), g), DEFAULT) for d, f, g in instances]
