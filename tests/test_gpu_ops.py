"""GPU parity: every C-ABI operator against the CPU oracle on the same seeded inputs.

Integers are compared bit for bit; AVG within 1e-12 relative (both sides do
one IEEE double division, so they normally agree exactly). Where the output
order is unspecified (compacted rows, pairs, rows inside a partition) the
outputs are compared as sorted multisets.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_2508_05029_amd import pipeline, tq  # noqa: E402
from paper_2508_05029_amd.datagen import uniform, permutation, zipf  # noqa: E402
from paper_2508_05029_amd.datagen import workloads as wl  # noqa: E402
from paper_2508_05029_amd.datagen.workloads import Factor, Pred  # noqa: E402

DEV = "cuda"


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def assert_groups_equal(got, want, avg_of=None):
    assert got["keys"].tolist() == want["keys"].tolist()
    assert got["count"].tolist() == want["count"].tolist()
    assert got["sums"].tolist() == want["sums"].tolist()
    cols = range(want["avg"].shape[1]) if avg_of is None else avg_of
    for j in cols:
        a, b = got["avg"][:, j], want["avg"][:, j]
        assert np.all(np.abs(a - b) <= 1e-12 * np.abs(b)), (a, b)


# ---------------------------------------------------------------- filter + group-by

@pytest.mark.parametrize("n", [0, 1, 3, 4, 5, 1000, 4097, 100_003, 1_000_000])
def test_filter_groupby_matches_oracle(n):
    say(f"filter_groupby n={n}")
    t = wl.filter_groupby_tables(n)
    q = wl.FILTER_GROUPBY_QUERY
    fg = pipeline.FilterGroupBy(q)
    fg.run(pipeline.to_device(t))
    got = fg.result()
    want = oracle.filter_groupby(t, q)
    assert_groups_equal(got, want, q.avg_of)


def test_filter_groupby_is_repeatable_and_accumulates():
    t = wl.filter_groupby_tables(50_000)
    q = wl.FILTER_GROUPBY_QUERY
    fg = pipeline.FilterGroupBy(q)
    d = pipeline.to_device(t)
    fg.run(d)
    a = fg.result()
    fg.run(d)
    b = fg.result()
    assert a["sums"].tolist() == b["sums"].tolist()
    # two batches into one state equal one pass over both
    tq.groupby_init(fg.state, fg.domain, fg.nsum)
    cols = [d[c] for c in fg.names]
    half = 24_000  # a multiple of 16 rows keeps the second slice 16-byte aligned for every width
    tq.groupby_agg(fg.state, fg.domain, [c[:half] for c in cols], half, fg.preds, fg.key, fg.exprs)
    tq.groupby_agg(fg.state, fg.domain, [c[half:] for c in cols], 50_000 - half, fg.preds, fg.key, fg.exprs)
    out = fg.out
    tq.groupby_finalize(fg.state, out.keys, out.count, out.sums, out.avg, out.ngroups)
    c = out.host()
    assert c["sums"].tolist() == a["sums"].tolist()


@pytest.mark.parametrize("domain,skew", [(25, None), (4000, None), (65_536, 1.1), (100_000, None)])
def test_groupby_lds_modes_match_oracle(domain, skew):
    """Dense LDS partials, the LDS hot-key hash table, and its global overflow."""
    say(f"groupby domain={domain} skew={skew}")
    n = 300_000
    g = zipf(n, domain, skew, 4, 0) if skew else uniform(n, 0, domain - 1, np.int64, 4, 0)
    v = uniform(n, -10**12, 10**12, np.int64, 4, 1)
    w = uniform(n, 0, 100, np.int32, 4, 2)
    t = {"g": g, "v": v, "w": w}
    q = wl.FilterGroupByQuery(preds=[Pred("w", 5, 95)], key=wl.GroupKey(("g",), 1, domain),
                              sums=[(Factor("v"),), (Factor("v"), Factor("w", -1, 7))], avg_of=[0, 1])
    fg = pipeline.FilterGroupBy(q)
    fg.run(pipeline.to_device(t))
    got = fg.result()
    want = oracle.filter_groupby(t, q)
    assert_groups_equal(got, want)


@pytest.mark.parametrize("domain", [6, 4000, 100_000])
def test_finalize_reset_leaves_the_state_empty(domain):
    """tq_groupby_finalize_reset: queries one after another on one state, with no
    tq_groupby_init between them, each equal to the oracle (private rows for the small
    domain, one shared table for the larger ones)."""
    say(f"finalize_reset domain={domain}")
    q = wl.FilterGroupByQuery(preds=[Pred("w", 5, 95)], key=wl.GroupKey(("g",), 1, domain),
                              sums=[(Factor("v"),), (Factor("v"), Factor("w", -1, 7))], avg_of=[0, 1])
    fg = pipeline.FilterGroupBy(q)
    tq.groupby_init(fg.state, fg.domain, fg.nsum)
    for rep, n in enumerate((300_000, 70_001, 5)):
        g = uniform(n, 0, domain - 1, np.int64, 40 + rep, 0)
        v = uniform(n, -10**12, 10**12, np.int64, 40 + rep, 1)
        w = uniform(n, 0, 100, np.int32, 40 + rep, 2)
        t = {"g": g, "v": v, "w": w}
        d = pipeline.to_device(t)
        tq.groupby_agg(fg.state, fg.domain, [d[c] for c in fg.names], n, fg.preds, fg.key, fg.exprs)
        out = fg.out
        tq.groupby_finalize(fg.state, out.keys, out.count, out.sums, out.avg, out.ngroups, reset=True)
        assert_groups_equal(fg.result(), oracle.filter_groupby(t, q))
    # and for the fused join probe: two steps on one table and state, reset between them
    dim, fact = wl.join_agg_tables(150_000, 600_000, seed=47)
    q = wl.JOIN_AGG_QUERY
    want = oracle.join_agg(dim, fact, q)
    ja = pipeline.JoinAgg(q, 150_000, 0.5)
    ja.init_state()
    dd, fd = pipeline.to_device(dim), pipeline.to_device(fact)
    for _ in range(2):
        ja.build(dd)
        ja.probe(fd)
        ja.finalize(reset=True)
        got = ja.result()
        assert got["join_rows"] == want["join_rows"]
        assert_groups_equal(got, want, q.avg_of)


@pytest.mark.parametrize("domain", [25, 4000, 100_000])
def test_groupby_wraps_mod_2_64_like_the_oracle(domain):
    """Values near +-2^62: the products and the per-group sums leave the int64
    range and wrap mod 2^64, on the GPU exactly as in the oracle (dense LDS
    partials, the LDS hot-key table, and global atomics)."""
    say(f"groupby wrap domain={domain}")
    n = 200_003
    t = {"g": uniform(n, 0, domain - 1, np.int64, 81, 0),
         "v": uniform(n, 2 ** 62 - 2 ** 40, 2 ** 62, np.int64, 81, 1),
         "u": uniform(n, -(2 ** 62), 2 ** 62, np.int64, 81, 2),
         "w": uniform(n, 0, 100, np.int32, 81, 3)}
    sums = [(Factor("v"),), (Factor("v"), Factor("w", -1, 7)), (Factor("u"), Factor("v"), Factor("w", 1, 3))]
    q = wl.FilterGroupByQuery(preds=[Pred("w", 1, 99)], key=wl.GroupKey(("g",), 1, domain), sums=sums,
                              avg_of=[0, 1, 2])
    fg = pipeline.FilterGroupBy(q)
    fg.run(pipeline.to_device(t))
    got = fg.result()
    want = oracle.filter_groupby(t, q)
    assert oracle.project(t, sums[1])[1].any() and oracle.project(t, sums[2])[1].any()  # products wrap
    # the exact sums leave the int64 range: SUM(v) of every group with 3 rows or more (v >= 2^62 - 2^40)
    assert want["overflow"].any() and want["overflow"][want["count"] >= 3, 0].all()
    assert_groups_equal(got, want)


def test_groupby_key_outside_domain_is_latched():
    t = {"g": np.array([0, 1, 7, 2], np.int64), "v": np.arange(4, dtype=np.int64)}
    q = wl.FilterGroupByQuery(preds=[], key=wl.GroupKey(("g",), 1, 4), sums=[(Factor("v"),)], avg_of=[])
    fg = pipeline.FilterGroupBy(q)
    fg.run(pipeline.to_device(t))
    with pytest.raises(tq.TqError) as e:
        fg.result()
    assert e.value.status == tq.TQ_EDOMAIN


# ---------------------------------------------------------------- filter + project

@pytest.mark.parametrize("n", [0, 7, 64, 1000, 65_537])
def test_filter_project_matches_oracle(n):
    rng = np.random.default_rng(n)
    t = {"a": rng.integers(-50, 50, n).astype(np.int64), "b": rng.integers(0, 256, n).astype(np.uint8),
         "c": rng.integers(-1000, 1000, n).astype(np.int32)}
    preds = [Pred("a", -20, 30), Pred("b", 0, 200)]
    exprs = [(Factor("a"), Factor("c", -1, 100)), (Factor("b", 1, 1), Factor("c"), Factor(None, 1, 3)), (Factor("c"),)]
    names = ["a", "b", "c"]
    d = pipeline.to_device(t)
    out = [torch.empty(max(n, 1), dtype=torch.int64, device=DEV) for _ in exprs]
    sel = torch.empty(max(n, 1), dtype=torch.int64, device=DEV)
    cnt = torch.zeros(1, dtype=torch.int64, device=DEV)
    scratch = torch.empty(tq.filter_project_scratch_bytes(n), dtype=torch.uint8, device=DEV)
    tq.filter_project([d[c] for c in names], n, pipeline.plan_preds(names, preds),
                      pipeline.plan_exprs(names, exprs), out, sel, cnt, scratch)
    m = int(cnt.item())
    mask = oracle.filter_mask(t, preds)
    assert m == int(mask.sum())
    rows = sel[:m].cpu().numpy()
    assert rows.tolist() == np.nonzero(mask)[0].tolist()  # stable: ascending row order
    for j, e in enumerate(exprs):
        want = oracle.project(t, e)[0][mask.astype(bool)]
        assert out[j][:m].cpu().numpy().tolist() == want.tolist()


# ---------------------------------------------------------------- join

def _pairs(build_keys, probe_keys, lf=0.5, unique=False, capacity=None):
    nb, np_ = len(build_keys), len(probe_keys)
    bk = torch.from_numpy(np.asarray(build_keys, np.int64)).to(DEV)
    pk = torch.from_numpy(np.asarray(probe_keys, np.int64)).to(DEV)
    pay = torch.arange(nb, dtype=torch.int64, device=DEV)
    table = torch.empty(tq.join_table_bytes(nb, lf), dtype=torch.uint8, device=DEV)
    tq.join_table_init(table)
    tq.join_build(table, bk, pay, nb, load_factor=lf, flags=tq.TQ_UNIQUE_KEYS if unique else 0)
    total, _, _ = oracle.join_pairs(bk.cpu().numpy(), pk.cpu().numpy(), with_pairs=False)
    cap = max(total, 1) if capacity is None else capacity
    rows = torch.empty(cap, dtype=torch.int64, device=DEV)
    bro = torch.empty(cap, dtype=torch.int64, device=DEV)
    cnt = torch.zeros(1, dtype=torch.int64, device=DEV)
    tq.join_probe(table, pk, np_, out_row=rows, out_payload=bro, capacity=cap, out_count=cnt)
    tq.check(table)
    m = int(cnt.item())
    k = min(m, cap)
    rl = rows[:k].cpu().tolist()
    assert rl == sorted(rl)  # pairs come out in probe-row order
    got = sorted(zip(rl, bro[:k].cpu().tolist()))
    return m, got


@pytest.mark.parametrize("lf", [0.25, 0.5, 0.9])
def test_join_pairs_many_to_many(lf):
    rng = np.random.default_rng(3)
    bk, pk = rng.integers(0, 3000, 10_000), rng.integers(-100, 3500, 40_000)
    m, got = _pairs(bk, pk, lf)
    total, pr, br = oracle.join_pairs(bk, pk)
    assert m == total
    assert got == list(zip(pr.tolist(), br.tolist()))


def test_join_pairs_heavy_duplicates():
    # one key repeated 6,000 times: its chain runs over some 750 buckets
    rng = np.random.default_rng(5)
    bk = np.concatenate([np.full(6000, 7, np.int64), rng.integers(10, 200_000, 30_000)])
    rng.shuffle(bk)
    pk = np.concatenate([np.array([7, 7, 8], np.int64), rng.integers(0, 210_000, 20_000)])
    m, got = _pairs(bk, pk, 0.5)
    total, pr, br = oracle.join_pairs(bk, pk)
    assert m == total and m > 12_000
    assert got == list(zip(pr.tolist(), br.tolist()))


def test_join_pairs_extreme_keys_and_empty_sides():
    I64_MIN, I64_MAX = -(2 ** 63), 2 ** 63 - 1
    bk = [I64_MAX, I64_MIN, I64_MIN + 1, -1, 0, 5, 5]
    pk = [5, -1, I64_MAX, 7, I64_MIN, I64_MIN + 1, 0, 5]
    m, got = _pairs(bk, pk)
    total, pr, br = oracle.join_pairs(np.array(bk), np.array(pk))
    assert m == total and got == list(zip(pr.tolist(), br.tolist()))
    assert _pairs([], [1, 2, 3])[0] == 0
    assert _pairs([1, 2, 3], [])[0] == 0


def test_join_pairs_capacity_overflow_reports_total():
    bk = np.arange(100)
    pk = np.concatenate([np.arange(100)] * 3)
    m, got = _pairs(bk, pk, capacity=50)
    assert m == 300 and len(got) == 50


def test_join_same_slot_collisions():
    # keys that share their top hash bits land on the same home slot
    keys = (np.arange(2000, dtype=np.int64) << 40)
    m, got = _pairs(keys, keys[::-1].copy(), lf=0.9, unique=True)
    total, pr, br = oracle.join_pairs(keys, keys[::-1].copy())
    assert m == total == 2000 and got == list(zip(pr.tolist(), br.tolist()))


def _table_header(table):
    """(regions, alt, log2g, log2cap, bloom_log2w) from the table header:
    whether the last build filled the table region by region in LDS, whether a
    fallback insert built it into the scratch's alternate arrays, the probe's
    wrap span, and the size of the Bloom filter a region build leaves."""
    h = table[:72].cpu().numpy()
    i32 = lambda o: int(h[o:o + 4].view(np.int32)[0])  # noqa: E731
    return i32(52), i32(56), i32(48), i32(16), i32(64)


@pytest.mark.parametrize("case", ["regions", "multipass", "multipass_16", "cas_large_table", "cas_region_overflow",
                                  "cas_domain_overflow", "host_fallback"])
def test_join_build_paths(case):
    """Each build path gives the oracle's pairs, and the header says which ran:
    regions (filled in LDS; up to 2^19 slots one domain per region, up to 2^23
    several domains of 2048 slots filled one after the other; probing wraps
    inside a domain), or the global CAS insert (wrapping over the whole
    table): into the alternate arrays when the table is too large for LDS
    domains or some domain receives more rows than it can hold with a free
    slot, or into the main arrays (with a counting pass first) when the rows'
    segments do not fit the scratch area."""
    rng = np.random.default_rng(11)
    filt = ()
    if case == "regions":
        bk = rng.permutation(100_000).astype(np.int64)
        nb_table, want_regions = len(bk), 1
    elif case == "multipass":
        bk = rng.permutation(600_000).astype(np.int64)  # 2^21 slots at 0.5: four domains per region
        nb_table, want_regions = len(bk), 1
    elif case == "multipass_16":
        bk = rng.permutation(3_000_000).astype(np.int64)  # 2^23 slots: sixteen domains per region
        nb_table, want_regions = len(bk), 1
    elif case == "cas_large_table":
        bk = rng.permutation(5_000_000).astype(np.int64)  # 2^24 slots at 0.5
        nb_table, want_regions = len(bk), 0
    elif case == "cas_domain_overflow":
        # one key 3000 times: its domain cannot hold them
        bk = np.concatenate([np.full(3000, 7, np.int64), rng.permutation(600_000).astype(np.int64) + 10])
        rng.shuffle(bk)
        nb_table, want_regions = len(bk), 0
    elif case == "cas_region_overflow":
        bk = np.concatenate([np.full(3000, 7, np.int64), rng.integers(10, 400_000, 17_000)])
        rng.shuffle(bk)
        nb_table, want_regions = len(bk), 0
    else:
        # a selective filter over many rows into a table sized for the survivors
        bk = rng.permutation(40_000).astype(np.int64)
        filt = (bk % 40 == 0)
        nb_table, want_regions = int(filt.sum()), 0
    pk = np.concatenate([bk[:5000], rng.integers(-1000, 700_000, 30_000)])
    n = len(bk)
    say(f"build path {case} n={n}")
    d_bk = torch.from_numpy(bk).to(DEV)
    pay = torch.arange(n, dtype=torch.int64, device=DEV)
    table = torch.empty(tq.join_table_bytes(nb_table, 0.5), dtype=torch.uint8, device=DEV)
    tq.join_table_init(table)
    if len(filt):
        f = torch.from_numpy(filt.astype(np.int32)).to(DEV)
        tq.join_build(table, d_bk, pay, n, filt_cols=[f], ps=[(0, 1, 1)], load_factor=0.5)
        keep = np.nonzero(filt)[0]
    else:
        tq.join_build(table, d_bk, pay, n, load_factor=0.5)
        keep = np.arange(n)
    tq.check(table)
    regions, alt, log2g, log2cap, bloom_log2w = _table_header(table)
    assert regions == want_regions
    assert alt == (1 if case.startswith("cas") else 0)  # the fallback insert uses the alternate arrays
    assert log2cap == {"multipass": 21, "multipass_16": 23, "cas_large_table": 24,
                       "cas_domain_overflow": 21}.get(case, log2cap)
    assert log2g == (min(log2cap, 19) - 11 if regions else log2cap - 3)
    # two filter bits per slot, 512 to 2^19 words of 32 bits (past 32768 words a probe reads it
    # from device memory instead of LDS); only a region build (up to 2^23 slots) has one
    assert bloom_log2w == (max(log2cap - 4, 9) if regions else 0)
    total, pr, br = oracle.join_pairs(bk[keep], pk)
    cap = max(total, 1)
    rows = torch.empty(cap, dtype=torch.int64, device=DEV)
    bro = torch.empty(cap, dtype=torch.int64, device=DEV)
    cnt = torch.zeros(1, dtype=torch.int64, device=DEV)
    tq.join_probe(table, torch.from_numpy(pk).to(DEV), len(pk), out_row=rows, out_payload=bro, capacity=cap,
                  out_count=cnt)
    tq.check(table)
    assert int(cnt.item()) == total
    got = sorted(zip(rows[:total].cpu().tolist(), bro[:total].cpu().tolist()))
    # the oracle's build rows are indices into bk[keep]; the payload is the row of bk
    assert got == sorted(zip(pr.tolist(), keep[br].tolist()))


def test_join_build_repeated_into_one_table():
    """Builds of different sizes into one buffer, each probed: the build's
    tickets and counts start clean every time, whichever path ran before."""
    rng = np.random.default_rng(12)
    table = torch.empty(tq.join_table_bytes(600_000, 0.5), dtype=torch.uint8, device=DEV)
    tq.join_table_init(table)
    for n in (50_000, 600_000, 3, 0, 200_000, 1):
        bk = rng.permutation(max(n, 1) * 2)[:n].astype(np.int64)
        pk = rng.integers(0, max(n, 1) * 2, 20_000).astype(np.int64)
        say(f"repeated build n={n}")
        pay = torch.arange(max(n, 1), dtype=torch.int64, device=DEV)
        tq.join_build(table, torch.from_numpy(bk).to(DEV) if n else pay, pay, n, load_factor=0.5)
        total, pr, br = oracle.join_pairs(bk, pk)
        cap = max(total, 1)
        rows = torch.empty(cap, dtype=torch.int64, device=DEV)
        bro = torch.empty(cap, dtype=torch.int64, device=DEV)
        cnt = torch.zeros(1, dtype=torch.int64, device=DEV)
        tq.join_probe(table, torch.from_numpy(pk).to(DEV), len(pk), out_row=rows, out_payload=bro, capacity=cap,
                      out_count=cnt)
        tq.check(table)
        assert int(cnt.item()) == total
        got = sorted(zip(rows[:total].cpu().tolist(), bro[:total].cpu().tolist()))
        assert got == sorted(zip(pr.tolist(), br.tolist()))


def test_build_after_a_failed_build_starts_clean():
    """A build that latches TQ_EFULL, then one that fits, into the same buffer:
    the second build clears the error and its table matches the oracle. Both
    build paths fail and recover: the region build (rows that fit the scratch
    segments, too many of them passing the filter) and the counting CAS build
    (more rows than the scratch holds)."""
    rng = np.random.default_rng(31)
    table = torch.empty(tq.join_table_bytes(1000, 0.5), dtype=torch.uint8, device=DEV)  # 2048 slots
    tq.join_table_init(table)
    pk = rng.integers(0, 20_000, 30_000).astype(np.int64)
    # (rows, kept by the filter): region path too full; CAS path that fits; CAS path too full; region path that fits
    for n, keep_every, fits in ((2000, 1, False), (3000, 6, True), (10_000, 1, False), (500, 1, True)):
        bk = rng.permutation(20_000)[:n].astype(np.int64)
        f = (np.arange(n) % keep_every == 0).astype(np.int32)
        say(f"build n={n} kept={int(f.sum())} fits={fits}")
        pay = torch.arange(n, dtype=torch.int64, device=DEV)
        tq.join_build(table, torch.from_numpy(bk).to(DEV), pay, n, filt_cols=[torch.from_numpy(f).to(DEV)],
                      ps=[(0, 1, 1)], load_factor=0.5)
        if not fits:
            with pytest.raises(tq.TqError) as e:
                tq.check(table)
            assert e.value.status == tq.TQ_EFULL
            continue
        tq.check(table)
        keep = np.nonzero(f)[0]
        total, pr, br = oracle.join_pairs(bk[keep], pk)
        cap = max(total, 1)
        rows = torch.empty(cap, dtype=torch.int64, device=DEV)
        bro = torch.empty(cap, dtype=torch.int64, device=DEV)
        cnt = torch.zeros(1, dtype=torch.int64, device=DEV)
        tq.join_probe(table, torch.from_numpy(pk).to(DEV), len(pk), out_row=rows, out_payload=bro, capacity=cap,
                      out_count=cnt)
        tq.check(table)
        assert int(cnt.item()) == total > 0
        got = sorted(zip(rows[:total].cpu().tolist(), bro[:total].cpu().tolist()))
        assert got == sorted(zip(pr.tolist(), keep[br].tolist()))


def test_join_table_too_small_latches_full():
    table = torch.empty(tq.join_table_bytes(100, 0.5), dtype=torch.uint8, device=DEV)
    tq.join_table_init(table)
    keys = torch.arange(10_000, dtype=torch.int64, device=DEV)
    tq.join_build(table, keys, keys, 10_000, load_factor=0.5)
    with pytest.raises(tq.TqError) as e:
        tq.check(table)
    assert e.value.status == tq.TQ_EFULL


@pytest.mark.parametrize("lf,unique", [(0.5, True), (0.25, False), (0.9, True), (0.1, True)])
def test_join_agg_full_size_matches_oracle(lf, unique):
    say(f"join_agg 1.5M x 6M lf={lf} unique={unique}")
    dim, fact = wl.join_agg_tables()
    q = wl.JOIN_AGG_QUERY
    ja = pipeline.JoinAgg(q, len(dim["key"]), lf, unique=unique)
    ja.run(pipeline.to_device(dim), pipeline.to_device(fact))
    got = ja.result()
    want = oracle.join_agg(dim, fact, q)
    assert got["join_rows"] == want["join_rows"]
    assert_groups_equal(got, want, q.avg_of)


def _join_agg_case(dim, fact, q, lf, unique):
    ja = pipeline.JoinAgg(q, len(dim["key"]), lf, unique=unique)
    ja.run(pipeline.to_device(dim), pipeline.to_device(fact))
    got = ja.result()
    want = oracle.join_agg(dim, fact, q)
    assert got["join_rows"] == want["join_rows"]
    assert_groups_equal(got, want, q.avg_of)
    return want["join_rows"]


@pytest.mark.parametrize("lf", [0.5, 0.9])
def test_join_agg_duplicate_build_keys(lf):
    # many-to-many: every build key appears several times; full buckets are common at 0.9
    nd, nf = 60_000, 300_000
    dim = {"key": uniform(nd, 0, 14_999, np.int64, 71, 0), "group": uniform(nd, 0, 24, np.int32, 71, 1),
           "date": uniform(nd, 700, 1100, np.int32, 71, 2)}
    fact = {"fk": uniform(nf, 0, 17_999, np.int64, 72, 0), "price": uniform(nf, 90_000, 10_500_000, np.int64, 72, 1),
            "disc": uniform(nf, 0, 10, np.int64, 72, 2)}
    say(f"duplicate build keys lf={lf}")
    assert _join_agg_case(dim, fact, wl.JOIN_AGG_QUERY, lf, unique=False) > nf


@pytest.mark.parametrize("bits,unique,n_dim,share", [(1, True, 150_000, False), (3, True, 150_000, False),
                                                     (4, False, 40_000, False), (2, True, 1_000_000, False),
                                                     (3, True, 400_000, True)])
def test_join_partitions_one_after_another_equal_the_whole_join(bits, unique, n_dim, share):
    """TQ_SELECT_PARTITION: 2^bits builds, each keeping one hash partition of the
    dimension rows, each followed by a probe of the whole fact table into one
    group-by state, give the whole join's result (the split of a join too large
    for its memory). share: the table holds only a partition's share of the rows
    (its build then takes the global-atomic path)."""
    say(f"partition builds bits={bits} unique={unique} n_dim={n_dim} share={share}")
    q = wl.JOIN_AGG_QUERY
    dim, fact = wl.join_agg_tables(n_dim, 4 * n_dim, seed=91 + bits)
    if not unique:
        dim["key"] = dim["key"] % (n_dim // 3)
    want = oracle.join_agg(dim, fact, q)
    dd, fd = pipeline.to_device(dim), pipeline.to_device(fact)
    # (about 15% of the dimension rows pass the date filter; a share is an eighth of those, with room)
    rows = n_dim if not share else int(n_dim * 0.16 / (1 << bits) * 1.5) + 1024
    ja = pipeline.JoinAgg(q, rows, 0.5, unique=unique)
    ja.init_state()
    for part in range(1 << bits):
        tq.join_build(ja.table, dd[q.build_key], dd[q.build_payload], n_dim, [dd[c] for c in ja.bnames], ja.bpreds,
                      0.5, bits, ja.flags | tq.TQ_SELECT_PARTITION | tq.TQ_PARTITION(part))
        ja.probe(fd)
    ja.finalize()
    got = ja.result()
    assert got["join_rows"] == want["join_rows"]
    assert_groups_equal(got, want, q.avg_of)
    # materialised pairs: the union over the partitions equals the join
    bk = dim["key"][:20_000]
    pk = fact["fk"][:50_000]
    total, pr, br = oracle.join_pairs(bk, pk)
    bkd, pkd = torch.from_numpy(bk).to(DEV), torch.from_numpy(pk).to(DEV)
    pay = torch.arange(len(bk), dtype=torch.int64, device=DEV)
    table = torch.empty(tq.join_table_bytes(len(bk), 0.5), dtype=torch.uint8, device=DEV)
    tq.join_table_init(table)
    pairs = []
    for part in range(1 << bits):
        tq.join_build(table, bkd, pay, len(bk), skip=bits,
                      flags=(tq.TQ_UNIQUE_KEYS if unique else 0) | tq.TQ_SELECT_PARTITION | tq.TQ_PARTITION(part))
        cap = max(total, 1)
        rws = torch.empty(cap, dtype=torch.int64, device=DEV)
        bro = torch.empty(cap, dtype=torch.int64, device=DEV)
        cnt = torch.zeros(1, dtype=torch.int64, device=DEV)
        tq.join_probe(table, pkd, len(pk), out_row=rws, out_payload=bro, capacity=cap, out_count=cnt)
        tq.check(table)
        m = int(cnt.item())
        assert m <= cap
        pairs += list(zip(rws[:m].cpu().tolist(), bro[:m].cpu().tolist()))
    assert sorted(pairs) == list(zip(pr.tolist(), br.tolist()))


@pytest.mark.parametrize("unique", [True, False])
def test_join_agg_equal_tags_and_long_chains(unique):
    # keys whose low 40 bits are zero share one tag, so every probe of a bucket
    # sees several candidates; at load factor 0.9 chains run over many buckets
    nd = 3000
    keys = (np.arange(nd, dtype=np.int64) + 1) << 40
    dim = {"key": keys, "group": (np.arange(nd) % 25).astype(np.int32), "date": np.full(nd, 800, np.int32)}
    nf = 50_003
    pick = uniform(nf, 0, nd + 499, np.int64, 73, 0)  # about 1 in 7 misses
    fact = {"fk": (pick + 1) << 40, "price": uniform(nf, 90_000, 10_500_000, np.int64, 73, 1),
            "disc": uniform(nf, 0, 10, np.int64, 73, 2)}
    say(f"equal tags unique={unique}")
    _join_agg_case(dim, fact, wl.JOIN_AGG_QUERY, 0.9, unique)


def test_join_agg_two_sums_and_probe_filter():
    dim, fact = wl.join_agg_tables(200_000, 900_001, seed=74)
    q0 = wl.JOIN_AGG_QUERY
    q = wl.JoinAggQuery(build_key=q0.build_key, build_payload=q0.build_payload, build_preds=q0.build_preds,
                        probe_key=q0.probe_key, probe_preds=[Pred("disc", 2, 8)],
                        sums=[q0.sums[0], [Factor("price", 1, 0)]], domain=q0.domain, avg_of=[0, 1])
    _join_agg_case(dim, fact, q, 0.5, True)


@pytest.mark.parametrize("n_fact", [400_000, 6_000_000])
def test_join_agg_wraps_mod_2_64_like_the_oracle(n_fact):
    """Prices near 2^62: price * (100 - discount) and the per-group sums wrap
    mod 2^64 in the fused probe exactly as in the oracle."""
    say(f"join_agg wrap n_fact={n_fact}")
    dim, fact = wl.join_agg_tables(n_fact // 4, n_fact, seed=82)
    fact["price"] = uniform(n_fact, 2 ** 61, 2 ** 62, np.int64, 82, 5)
    q0 = wl.JOIN_AGG_QUERY
    q = wl.JoinAggQuery(build_key=q0.build_key, build_payload=q0.build_payload, build_preds=q0.build_preds,
                        probe_key=q0.probe_key, probe_preds=[], sums=[q0.sums[0], [Factor("price", 1, 0)]],
                        domain=q0.domain, avg_of=[0, 1])
    want_rows = _join_agg_case(dim, fact, q, 0.5, True)
    assert want_rows > 0
    assert oracle.project(fact, q.sums[0])[1].any()  # the product wraps
    want = oracle.join_agg(dim, fact, q)
    assert want["overflow"][:, 1].all()  # so does every group's SUM(price) (prices >= 2^61, thousands of rows)


@pytest.mark.parametrize("nd,nf", [(1, 1), (3, 10), (100, 5), (4097, 20_001)])
def test_join_agg_small_and_ragged(nd, nf):
    dim, fact = wl.join_agg_tables(nd, nf, seed=17 + nd)
    dim["date"][: max(1, nd // 2)] = 800  # make sure some dimension rows pass
    q = wl.JOIN_AGG_QUERY
    ja = pipeline.JoinAgg(q, nd, 0.5)
    ja.run(pipeline.to_device(dim), pipeline.to_device(fact))
    got = ja.result()
    want = oracle.join_agg(dim, fact, q)
    assert got["join_rows"] == want["join_rows"]
    assert_groups_equal(got, want, q.avg_of)


# ---------------------------------------------------------------- hash partition

@pytest.mark.parametrize("n,bits,skip", [(0, 4, 0), (1, 0, 0), (5000, 1, 0), (100_001, 8, 0), (300_000, 10, 0),
                                         (70_000, 6, 8)])
def test_hash_partition_matches_oracle(n, bits, skip):
    say(f"partition n={n} bits={bits} skip={skip}")
    keys = uniform(n, -(2 ** 62), 2 ** 62, np.int64, 9, 0)
    p64 = uniform(n, -10**15, 10**15, np.int64, 9, 1)
    p32 = uniform(n, -10**9, 10**9, np.int32, 9, 2)
    p8 = uniform(n, 0, 255, np.uint8, 9, 3)
    d = [torch.from_numpy(a).to(DEV) for a in (keys, p64, p32, p8)]
    out = [torch.empty(max(n, 1), dtype=t.dtype, device=DEV) for t in d]
    offs = torch.empty((1 << bits) + 1, dtype=torch.int64, device=DEV)
    scratch = torch.empty(max(1, tq.hash_partition_scratch_bytes(n, bits)), dtype=torch.uint8, device=DEV)
    tq.hash_partition(d[0], d[1:], n, bits, skip, out[0], out[1:], offs, scratch)
    torch.cuda.synchronize()
    # the oracle partitions by the top bits; with skip the id is taken from the bits below
    pid = oracle.partition_ids(keys, bits + skip) & ((1 << bits) - 1) if skip else oracle.partition_ids(keys, bits)
    counts = np.bincount(pid, minlength=1 << bits) if n else np.zeros(1 << bits, np.int64)
    want_offs = np.concatenate([[0], np.cumsum(counts)])
    got_offs = offs.cpu().numpy()
    assert got_offs.tolist() == want_offs.tolist()
    host = [o[:n].cpu().numpy() for o in out]
    src = [keys, p64, p32, p8]
    for p in range(1 << bits):
        a, b = got_offs[p], got_offs[p + 1]
        rows = np.nonzero(pid == p)[0]
        # rows travel together: sort both sides by key then compare every column
        go = np.lexsort((host[1][a:b], host[0][a:b]))
        wo = np.lexsort((p64[rows], keys[rows]))
        for j in range(4):
            assert host[j][a:b][go].tolist() == src[j][rows][wo].tolist()


def test_partition_then_join_equals_unpartitioned():
    """Join partition by partition (with the table slot bits below the
    partition bits) and compare with the plain join result."""
    dim, fact = wl.join_agg_tables(200_000, 800_000, seed=23)
    q = wl.JOIN_AGG_QUERY
    want = oracle.join_agg(dim, fact, q)
    dd, fd = pipeline.to_device(dim), pipeline.to_device(fact)
    bits = 4
    nb = 1 << bits

    def part(keys, pay):
        n = keys.numel()
        ok = torch.empty_like(keys)
        op = [torch.empty_like(t) for t in pay]
        offs = torch.empty(nb + 1, dtype=torch.int64, device=DEV)
        sc = torch.empty(tq.hash_partition_scratch_bytes(n, bits), dtype=torch.uint8, device=DEV)
        tq.hash_partition(keys, pay, n, bits, 0, ok, op, offs, sc)
        return ok, op, offs.cpu().tolist()

    dk, (dg, dt), doff = part(dd["key"], [dd["group"], dd["date"]])
    fk, (fp, fdc), foff = part(fd["fk"], [fd["price"], fd["disc"]])
    ja = pipeline.JoinAgg(q, 200_000, 0.5)
    ja.init_state()
    for p in range(nb):
        a, b = doff[p], doff[p + 1]
        # 16-byte alignment of the slices: copy each partition to fresh buffers
        dpart = {"key": dk[a:b].clone(), "group": dg[a:b].clone(), "date": dt[a:b].clone()}
        c, e = foff[p], foff[p + 1]
        fpart = {"fk": fk[c:e].clone(), "price": fp[c:e].clone(), "disc": fdc[c:e].clone()}
        ja.build(dpart, skip=bits)
        ja.probe(fpart)
    ja.finalize()
    got = ja.result()
    assert_groups_equal(got, want, q.avg_of)


# ---------------------------------------------------------------- measurement kernels

def test_read_peak_and_fill():
    x = torch.empty(1 << 20, dtype=torch.int64, device=DEV)
    tq.fill(x, 0x01010101)
    assert int(x[123].item()) == 0x0101010101010101
    part = torch.zeros(tq.read_peak_scratch_bytes() // 8, dtype=torch.int64, device=DEV)
    tq.read_peak(x, part)
    # the partial checksums wrap mod 2^64 (int64 adds), so compare modulo 2^64
    got = sum(int(x) for x in part.cpu().tolist()) % (1 << 64)
    assert got == ((1 << 20) * 0x0101010101010101) % (1 << 64)
