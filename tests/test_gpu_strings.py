"""GPU: dictionary-encoded string keys. tq_dict_unify maps one dictionary
onto another by byte equality; joins on string keys encoded against two
dictionaries, and group-by on a string column, against the oracle, which
compares the decoded strings themselves. Integers bit-exact."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_2508_05029_amd import pipeline, tq  # noqa: E402
from paper_2508_05029_amd.datagen import uniform  # noqa: E402
from paper_2508_05029_amd.datagen import workloads as wl  # noqa: E402
from paper_2508_05029_amd.datagen.workloads import Factor  # noqa: E402

DEV = "cuda"


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def arrow(strings):
    off = np.zeros(len(strings) + 1, np.int32)
    off[1:] = np.cumsum([len(s) for s in strings])
    data = np.frombuffer(b"".join(strings), np.uint8).copy() if strings else np.zeros(0, np.uint8)
    return off, data


def on_dev(sc):
    off, data = sc
    # an empty byte buffer still gets one byte, so that its pointer is not NULL
    return torch.from_numpy(off).to(DEV), torch.from_numpy(data if len(data) else np.zeros(1, np.uint8)).to(DEV)


def bitmap(n, density, seed, stream):
    present = uniform(n, 0, 999, np.int64, seed, stream) >= int(density * 1000)
    return np.packbits(present.astype(np.uint8), bitorder="little")


def gpu_unify(build, probe):
    nb, npr = len(build[0]) - 1, len(probe[0]) - 1
    table = torch.empty(tq.join_table_bytes(max(nb, 1), 0.5), dtype=torch.uint8, device=DEV)
    scratch = torch.empty(tq.dict_unify_scratch_bytes(nb), dtype=torch.uint8, device=DEV)
    remap = torch.full((max(npr, 1),), -7, dtype=torch.int32, device=DEV)
    tq.dict_unify(table, on_dev(build), on_dev(probe), scratch, remap[:npr])
    tq.check(table)
    return remap[:npr].cpu().numpy()


def tricky(n, seed):
    rng = np.random.default_rng(seed)
    out = {b"", b"a", b"ab", b"abc", b"abd", b"bbc", b"\x00", b"\x00\x00", b"\xff", b"\x80a", b"x" * 300}
    while len(out) < n:
        L = int(rng.integers(0, 40))
        out.add(bytes(rng.integers(0, 256, L).astype(np.uint8)) if rng.random() < 0.5
                else bytes(rng.choice(list(b"ab\x00\xff"), L).astype(np.uint8)))
    return sorted(out)


@pytest.mark.parametrize("nb,npr", [(0, 5), (5, 0), (1, 1), (700, 900), (3000, 2500)])
def test_dict_unify_matches_oracle_on_tricky_strings(nb, npr):
    say(f"dict_unify tricky nb={nb} np={npr}")
    pool = tricky(max(nb, npr) + 500, nb + npr)
    rng = np.random.default_rng(nb * 7 + npr)
    build = [pool[i] for i in rng.permutation(len(pool))[:nb]]
    probe = [pool[i] for i in rng.permutation(len(pool))[:npr]]
    b, p = arrow(build), arrow(probe)
    assert gpu_unify(b, p).tolist() == oracle.dict_unify(b, p).tolist()


@pytest.mark.parametrize("n", [1000, 200_000])
def test_dict_unify_matches_oracle_on_the_workload_dictionaries(n):
    say(f"dict_unify workload n={n}")
    T = wl.string_join_tables(n, 10)
    got = gpu_unify(T.build_dict, T.probe_dict)
    want = oracle.dict_unify(T.build_dict, T.probe_dict)
    assert got.tolist() == want.tolist()
    assert (got < 0).sum() == n // 4


@pytest.mark.parametrize("nd,nf,density", [(150_000, 600_000, 0.1), (1000, 5000, 0.0), (3, 10, 0.3)])
def test_string_join_agg_matches_oracle(nd, nf, density):
    say(f"string join nd={nd} nf={nf} density={density}")
    T = wl.string_join_tables(nd, nf, seed=71)
    dvalid = {"key": bitmap(nd, density, 72, 0)} if density else None
    fvalid = {"fk": bitmap(nf, density, 72, 1)} if density else None
    q = wl.JOIN_AGG_QUERY
    want = oracle.join_agg_strings(T.build_dict, T.dim, dvalid, T.probe_dict, T.fact, fvalid, q)
    sj = pipeline.StringJoinAgg(q, nd, nf, nd, nd)
    dv = None if dvalid is None else {k: torch.from_numpy(v).to(DEV) for k, v in dvalid.items()}
    fv = None if fvalid is None else {k: torch.from_numpy(v).to(DEV) for k, v in fvalid.items()}
    sj.run(on_dev(T.build_dict), on_dev(T.probe_dict), pipeline.to_device(T.dim), dv, pipeline.to_device(T.fact), fv)
    got = sj.result()
    assert got["join_rows"] == want["join_rows"]
    for k in ("keys", "key_null", "count", "sums", "nonnull"):
        assert got[k].tolist() == want[k].tolist(), k


def test_group_by_a_string_column_groups_by_its_codes():
    """GROUP BY a dictionary-encoded string: the group-by runs on the codes
    (domain = dictionary size) and the output keys decode to the strings; the
    oracle groups the decoded strings."""
    nd, nf = 50_000, 400_000
    T = wl.string_join_tables(nd, nf, seed=73)
    q = wl.FilterGroupByQuery(preds=[], key=wl.GroupKey(("fk",), 1, nd), sums=[(Factor("price"),)], avg_of=[0])
    fg = pipeline.FilterGroupBy(q)
    fg.run(pipeline.to_device(T.fact))
    got = fg.result()
    strings = oracle.decode(T.probe_dict, got["keys"][:, 0])
    by_string = {s: (int(c), int(v)) for s, c, v in zip(strings, got["count"], got["sums"][:, 0])}
    fact_strings = oracle.decode(T.probe_dict, T.fact["fk"])
    ids = {}
    for s in fact_strings:
        ids.setdefault(s, len(ids))
    want = oracle.groupby([np.array([ids[s] for s in fact_strings], np.int64)], [T.fact["price"]])
    inv = {v: k for k, v in ids.items()}
    expect = {inv[int(k)]: (int(c), int(v)) for k, c, v in zip(want["keys"][:, 0], want["count"], want["sums"][:, 0])}
    assert by_string == expect


def test_dict_unify_rejects_bad_arguments():
    b = on_dev(arrow([b"a", b"b"]))
    table = torch.empty(tq.join_table_bytes(2, 0.5), dtype=torch.uint8, device=DEV)
    small = torch.empty(tq.dict_unify_scratch_bytes(2) - 1, dtype=torch.uint8, device=DEV)
    remap = torch.empty(2, dtype=torch.int32, device=DEV)
    with pytest.raises(tq.TqError):
        tq.dict_unify(table, b, b, small, remap)
    st = tq.lib().tq_dict_keys(None, None, 5, None, 0, None, tq._stream(None))
    assert st == tq.TQ_EINVAL


def test_join_on_plain_string_columns():
    """Plain (unencoded) string key columns with a unique build side: each row
    is its own dictionary entry, so the codes are the row numbers."""
    nd, nf = 20_000, 100_000
    T = wl.string_join_tables(nd, nf, seed=74)
    dim_s = arrow(oracle.decode(T.build_dict, T.dim["key"]))
    fact_s = arrow(oracle.decode(T.probe_dict, T.fact["fk"]))
    dim = dict(T.dim, key=np.arange(nd, dtype=np.int32))
    fact = dict(T.fact, fk=np.arange(nf, dtype=np.int32))
    q = wl.JOIN_AGG_QUERY
    want = oracle.join_agg_strings(dim_s, dim, None, fact_s, fact, None, q)
    sj = pipeline.StringJoinAgg(q, nd, nf, nd, nf)
    sj.run(on_dev(dim_s), on_dev(fact_s), pipeline.to_device(dim), None, pipeline.to_device(fact), None)
    got = sj.result()
    assert got["join_rows"] == want["join_rows"] > 0
    for k in ("keys", "count", "sums"):
        assert got[k].tolist() == want[k].tolist(), k


def gpu_encode(sc):
    n = len(sc[0]) - 1
    scratch = torch.empty(tq.dict_encode_scratch_bytes(n), dtype=torch.uint8, device=DEV)
    codes = torch.full((max(n, 1),), -5, dtype=torch.int32, device=DEV)
    first = torch.full((max(n, 1),), -5, dtype=torch.int32, device=DEV)
    nd = torch.zeros(1, dtype=torch.int64, device=DEV)
    tq.dict_encode(on_dev(sc), scratch, codes[:n], first[:n], nd)
    torch.cuda.synchronize()
    return codes[:n].cpu().numpy(), first.cpu().numpy(), int(nd.item())


def check_encoding(sc):
    codes, first, nd = gpu_encode(sc)
    want = oracle.first_occurrence(sc)
    assert nd == len(np.unique(want))
    assert codes.min(initial=0) >= 0 and codes.max(initial=-1) < nd
    # equal codes exactly for equal strings, and each code's first row is its smallest
    assert first[codes].tolist() == want.tolist()


@pytest.mark.parametrize("case", ["empty", "one", "all_equal", "all_distinct", "tricky", "zipf"])
def test_dict_encode_matches_first_occurrence(case):
    say(f"dict_encode {case}")
    rng = np.random.default_rng(41)
    if case == "empty":
        strs = []
    elif case == "one":
        strs = [b"abc"]
    elif case == "all_equal":
        strs = [b"same string"] * 70_000
    elif case == "all_distinct":
        strs = tricky(5000, 42)
    elif case == "tricky":
        pool = tricky(300, 43)
        strs = [pool[i] for i in rng.integers(0, len(pool), 20_000)]
    else:
        pool = [s for s in oracle.decode(wl.string_join_tables(2000, 1).build_dict, np.arange(2000))]
        cdf = np.cumsum(1.0 / np.arange(1, 2001) ** 1.1)
        idx = np.searchsorted(cdf / cdf[-1], rng.random(300_000))
        strs = [pool[i] for i in idx]
    check_encoding(arrow(strs))


def test_group_by_a_plain_string_column():
    """GROUP BY over strings that are not dictionary-encoded: encoded on the
    GPU, grouped on the codes; the oracle groups the strings themselves."""
    n = 200_000
    T = wl.string_join_tables(20_000, n, seed=75)
    strs = oracle.decode(T.probe_dict, T.fact["fk"])  # 200K strings, many repeated
    col = arrow(strs)
    sg = pipeline.StringGroupBy(n, [(Factor("price"),)])
    got = sg.run(on_dev(col), {"price": torch.from_numpy(T.fact["price"]).to(DEV)})
    by = {strs[int(r)]: (int(c), int(v)) for r, c, v in zip(got["first_row"], got["count"], got["sums"][:, 0])}
    want = {}
    for s, v in zip(strs, T.fact["price"].tolist()):
        c, t = want.get(s, (0, 0))
        want[s] = (c + 1, t + v)
    assert by == want
