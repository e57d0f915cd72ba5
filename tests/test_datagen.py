"""The seeded generators: determinism, ranges, bijectivity, batch independence."""
import numpy as np

from paper_2508_05029_amd import datagen as dg
from paper_2508_05029_amd.datagen import workloads as wl


def test_uniform_range_and_determinism():
    a = dg.uniform(100_000, 90_000, 10_500_000, np.int64, 7, 3)
    b = dg.uniform(100_000, 90_000, 10_500_000, np.int64, 7, 3)
    assert (a == b).all()
    assert a.min() >= 90_000 and a.max() <= 10_500_000
    c = dg.uniform(100_000, 0, 2, np.uint8, 7, 4)
    assert set(np.unique(c).tolist()) == {0, 1, 2}
    counts = np.bincount(c)
    assert abs(counts / len(c) - 1 / 3).max() < 0.01


def test_batches_equal_the_whole_column():
    whole = dg.uniform(10_000, 0, 2405, np.int32, 5, 2)
    part = np.empty(3000, np.int32)
    dg.uniform_into(part.ctypes.data, np.int32, 3000, 0, 2405, 5, 2, first=4000)
    assert (part == whole[4000:7000]).all()


def test_permutation_is_a_bijection():
    for n in [1, 2, 3, 1000, 65537]:
        p = dg.permutation(n, 11, 0)
        assert sorted(p.tolist()) == list(range(n))


def test_zipf_top_share():
    G, n = 64, 200_000
    z = dg.zipf(n, G, 1.1, 3, 0)
    cdf = dg.zipf_cdf(G, 1.1)
    share = (z == 0).mean()
    assert abs(share - cdf[0]) < 0.01
    assert z.min() >= 0 and z.max() < G


def test_workload_shapes():
    t = wl.filter_groupby_tables(1000)
    assert t["date"].dtype == np.int32 and t["flagA"].dtype == np.uint8
    dim, fact = wl.join_agg_tables(1500, 6000)
    assert sorted(dim["key"].tolist()) == list(range(1500))
    assert fact["fk"].max() < 1500
    shapes = wl.batched_shapes(64)
    assert all(1000 <= s.n_fact <= 1_000_000 and 4 <= s.groups <= 65536 for s in shapes)
    reqs = wl.serving_requests(50, 100.0)
    assert all(r.shape in (0, 1, 2) for r in reqs)
    assert all(reqs[i].arrival_s < reqs[i + 1].arrival_s for i in range(49))
