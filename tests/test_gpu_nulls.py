"""GPU: NULLs (Arrow validity bitmaps) through filter + group-by and join +
aggregate, against the oracle's SQL semantics: a predicate over NULL drops the
row, NULL keys form one group (listed last) or match nothing in a join, sums
skip NULL values and report their own non-NULL counts, COUNT(*) counts every
row. Integers bit-exact, AVG within 1e-12."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_2508_05029_amd import pipeline, tq  # noqa: E402
from paper_2508_05029_amd.datagen import uniform  # noqa: E402
from paper_2508_05029_amd.datagen import workloads as wl  # noqa: E402
from paper_2508_05029_amd.datagen.workloads import Factor, Pred  # noqa: E402

DEV = "cuda"


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def bitmap(n, density, seed, stream):
    """An Arrow validity bitmap with about `density` of the rows NULL."""
    present = uniform(n, 0, 999, np.int64, seed, stream) >= int(density * 1000)
    return np.packbits(present.astype(np.uint8), bitorder="little")


def same(got, want):
    assert got["key_null"].tolist() == want["key_null"].tolist()
    assert got["keys"].tolist() == want["keys"].tolist()
    assert got["count"].tolist() == want["count"].tolist()
    assert got["nonnull"].tolist() == want["nonnull"].tolist()
    assert got["sums"].tolist() == want["sums"].tolist()
    a, b = got["avg"], want["avg"]
    assert np.all(np.abs(a - b) <= 1e-12 * np.abs(b)), (a, b)


def dev(bits):
    return None if bits is None else torch.from_numpy(bits).to(DEV)


@pytest.mark.parametrize("n,domain,density", [(0, 6, 0.3), (1, 6, 0.0), (5, 6, 1.0), (100_003, 6, 0.2),
                                              (300_000, 4000, 0.5), (200_000, 100_000, 0.1), (70_001, 3, 0.0)])
def test_nullable_filter_groupby_matches_oracle(n, domain, density):
    say(f"nullable filter+group-by n={n} domain={domain} density={density}")
    t = {"g": uniform(n, 0, domain - 1, np.int64, 61, 0), "v": uniform(n, -(2 ** 62), 2 ** 62, np.int64, 61, 1),
         "w": uniform(n, 0, 100, np.int32, 61, 2), "x": uniform(n, 0, 255, np.uint8, 61, 3)}
    valid = {"g": bitmap(n, density, 62, 0), "v": bitmap(n, density, 62, 1), "w": bitmap(n, density, 62, 2),
             "x": None if density == 0.0 else bitmap(n, density, 62, 3)}
    q = wl.FilterGroupByQuery(preds=[Pred("w", 5, 95)], key=wl.GroupKey(("g",), 1, domain),
                              sums=[(Factor("v"),), (Factor("v"), Factor("w", -1, 7)), (Factor("x"), Factor(None, 0, 3))],
                              avg_of=[0, 1, 2])
    fg = pipeline.NullableFilterGroupBy(q)
    fg.run(pipeline.to_device(t) if n else {k: torch.from_numpy(v).to(DEV) for k, v in t.items()},
           {k: dev(v) for k, v in valid.items()}, n)
    same(fg.result(), oracle.filter_groupby_nullable(t, valid, q))


@pytest.mark.parametrize("nd,nf,density,share", [(150_000, 600_000, 0.2, False), (40_000, 160_000, 0.5, False),
                                                 (3, 10, 0.3, False), (150_000, 600_000, 0.2, True)])
def test_nullable_join_agg_matches_oracle(nd, nf, density, share):
    say(f"nullable join nd={nd} nf={nf} density={density} share={share}")
    dim, fact = wl.join_agg_tables(nd, nf, seed=63)
    dvalid = {"key": bitmap(nd, density, 64, 0), "group": bitmap(nd, density, 64, 1), "date": bitmap(nd, density, 64, 2)}
    fvalid = {"fk": bitmap(nf, density, 65, 0), "price": bitmap(nf, density, 65, 1), "disc": bitmap(nf, density, 65, 2)}
    q = wl.JOIN_AGG_QUERY
    want = oracle.join_agg_nullable(dim, dvalid, fact, fvalid, q)
    # share: a table for a fraction of the rows, below the region build's segment room (global-atomic build path)
    ja = pipeline.NullableJoinAgg(q, nd if not share else nd // 5, 0.5)
    ja.run(pipeline.to_device(dim), {k: dev(v) for k, v in dvalid.items()}, pipeline.to_device(fact),
           {k: dev(v) for k, v in fvalid.items()})
    got = ja.result()
    assert got["join_rows"] == want["join_rows"]
    same(got, want)


def test_nullable_without_bitmaps_equals_the_plain_path():
    dim, fact = wl.join_agg_tables(100_000, 400_000, seed=66)
    q = wl.JOIN_AGG_QUERY
    plain = pipeline.JoinAgg(q, 100_000, 0.5)
    dd, fd = pipeline.to_device(dim), pipeline.to_device(fact)
    plain.run(dd, fd)
    a = plain.result()
    ja = pipeline.NullableJoinAgg(q, 100_000, 0.5)
    ja.run(dd, None, fd, None)
    b = ja.result()
    assert not b["key_null"].any()
    assert b["keys"].tolist() == a["keys"][:, 0].tolist()
    assert b["count"].tolist() == a["count"].tolist() and b["sums"].tolist() == a["sums"].tolist()
    assert (b["nonnull"] == b["count"][:, None]).all()


def test_bitmaps_need_the_nullable_entry_points():
    """A column with a validity bitmap passed to an entry point without NULL
    semantics is rejected before anything runs."""
    n = 1000
    t = pipeline.to_device({"g": np.zeros(n, np.int64), "v": np.ones(n, np.int64)})
    bits = torch.ones((n + 7) // 8, dtype=torch.uint8, device=DEV)
    state = torch.empty(tq.groupby_state_bytes(4, 1), dtype=torch.uint8, device=DEV)
    tq.groupby_init(state, 4, 1)
    key = tq.gkey([0], 1)
    status = tq.lib().tq_groupby_agg(state.data_ptr(), 4, tq.cols([t["g"], t["v"]], [None, bits]), 2, n,
                                     tq.preds([]), 0, tq.ctypes.byref(key), tq.exprs([[(1, 1, 0)]]), 1,
                                     tq._stream(None))
    assert status == tq.TQ_EINVAL
