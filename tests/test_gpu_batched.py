"""GPU: thousands-of-instances batching. Every instance of the batched
launches equals the oracle and the one-launch-per-instance path; results do
not depend on tile sizes or load factors; a captured hipGraph replays
correctly."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_2508_05029_amd import pipeline  # noqa: E402
from paper_2508_05029_amd.datagen import workloads as wl  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def make_instances(count, fact_hi=4.5, seed=wl.BATCH_SEED + 100):
    shapes = wl.batched_shapes(count, seed, fact_lo=3.0, fact_hi=fact_hi)
    out = []
    for i, s in enumerate(shapes):
        d, f = wl.batched_instance_tables(i, s, seed)
        out.append((d, f, s.groups))
    return out


def check_all(job, insts, which=None):
    which = range(len(insts)) if which is None else which
    got = job.results(which)
    for k, i in enumerate(which):
        d, f, G = insts[i]
        want = oracle.join_agg(d, f, wl.batched_query(G))
        g = got[k]
        assert g["keys"].tolist() == want["keys"].tolist(), i
        assert g["count"].tolist() == want["count"].tolist(), i
        assert g["sums"].tolist() == want["sums"].tolist(), i
        assert np.all(np.abs(g["avg"][:, 0] - want["avg"][:, 0]) <= 1e-12 * np.abs(want["avg"][:, 0])), i


@pytest.mark.parametrize("tiles", [(4096, 4096, 0.5), (1024, 65536, 0.25), (65536, 1024, 0.9)])
def test_batched_launches_match_oracle(tiles):
    bt, pt, lf = tiles
    say(f"batched tiles={tiles}")
    insts = make_instances(48)
    job = pipeline.BatchedJoinAgg(wl.batched_query(8), insts, [(lf, bt, pt)] * len(insts))
    job.run()
    job.check()
    check_all(job, insts)


def test_per_instance_path_matches_oracle():
    insts = make_instances(24)
    job = pipeline.BatchedJoinAgg(wl.batched_query(8), insts, [(0.5, 8192, 8192)] * len(insts))
    job.run_per_instance()
    torch.cuda.synchronize()
    check_all(job, insts)


def test_mixed_per_instance_parameters_and_graph_replay():
    insts = make_instances(32, fact_hi=5.0, seed=wl.BATCH_SEED + 200)
    params = [((0.25, 0.5, 0.75)[i % 3], (1024, 8192)[i % 2], (2048, 16384, 65536)[i % 3]) for i in range(len(insts))]
    job = pipeline.BatchedJoinAgg(wl.batched_query(8), insts, params)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        job.run()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        job.run()
    for rep in range(3):
        # eager work and a sync between replays
        torch.zeros(1, device="cuda").add_(1)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        job.check()
        check_all(job, insts)


def test_group_key_outside_domain_is_reported():
    """One instance whose dimension payloads (the group keys) all lie outside
    its domain: tq_batched_check reports TQ_EDOMAIN, as the stand-alone path's
    tq_check would, and every other instance still equals the oracle."""
    from paper_2508_05029_amd import tq
    insts = make_instances(12)
    bad = 5
    d, f, G = insts[bad]
    d = dict(d)
    d["group"] = np.full_like(d["group"], G)
    insts[bad] = (d, f, G)
    want_bad = oracle.join_agg(d, f, wl.batched_query(G))
    assert want_bad["join_rows"] > 0  # some probe row matches, so the bad key is reached
    job = pipeline.BatchedJoinAgg(wl.batched_query(8), insts, [(0.5, 4096, 4096)] * len(insts))
    job.run()
    with pytest.raises(tq.TqError) as e:
        job.check()
    assert e.value.status == tq.TQ_EDOMAIN
    check_all(job, insts, [i for i in range(len(insts)) if i != bad])


def test_batched_sums_wrap_mod_2_64_like_the_oracle():
    """Prices near 2^62 in every instance: products and per-group sums wrap mod
    2^64 in the batched launches exactly as in the oracle."""
    from paper_2508_05029_amd.datagen import uniform
    insts = []
    for i, (d, f, G) in enumerate(make_instances(24, seed=wl.BATCH_SEED + 300)):
        f = dict(f)
        f["price"] = uniform(len(f["price"]), 2 ** 61, 2 ** 62, np.int64, 83 + i, 0)
        insts.append((d, f, G))
    assert any(oracle.join_agg(d, f, wl.batched_query(G))["overflow"].any() for d, f, G in insts)
    job = pipeline.BatchedJoinAgg(wl.batched_query(8), insts, [(0.5, 4096, 8192)] * len(insts))
    job.run()
    job.check()
    check_all(job, insts)


@pytest.mark.parametrize("window", [(0, 1 << 30), (-5, -1), (100, 100)])
def test_build_keeps_every_row_none_or_few(window):
    """The build items compact the rows they keep per wave before inserting
    them: every dimension row kept (the queue fills on every step), none, or
    one date's rows, with 1088-row build tiles whose last wave is partial."""
    import dataclasses
    say(f"batched build window={window}")

    def query(G):
        return dataclasses.replace(wl.batched_query(G), build_preds=[wl.Pred("date", *window)])

    insts = make_instances(24, seed=wl.BATCH_SEED + 400)
    job = pipeline.BatchedJoinAgg(query(8), insts, [(0.5, 1088, 4096)] * len(insts))
    job.run()
    job.check()
    got = job.results(range(len(insts)))
    kept = 0
    for i, (d, f, G) in enumerate(insts):
        want = oracle.join_agg(d, f, query(G))
        kept += want["join_rows"]
        assert got[i]["keys"].tolist() == want["keys"].tolist(), i
        assert got[i]["count"].tolist() == want["count"].tolist(), i
        assert got[i]["sums"].tolist() == want["sums"].tolist(), i
    assert (kept > 0) == (window[1] >= 0)
