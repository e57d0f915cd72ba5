"""Parquet files for the scan tests, written by pyarrow from seeded columns."""
import numpy as np

from paper_2508_05029_amd.datagen import uniform  # noqa: F401 (also used by the tests)

pa = None
pq = None


def _arrow():
    global pa, pq
    if pa is None:
        import pyarrow
        import pyarrow.parquet
        pa, pq = pyarrow, pyarrow.parquet
    return pa, pq


def columns(n, seed, null_density=0.1):
    """Seeded columns of several kinds: (name, values, present mask or None, dictionary?)."""
    present = lambda s: uniform(n, 0, 999, np.int64, seed, s) >= int(null_density * 1000)
    return [
        ("key", uniform(n, -2 ** 62, 2 ** 62, np.int64, seed, 0), None, False),       # required int64, PLAIN
        ("grp", uniform(n, 0, 24, np.int32, seed, 1), present(11), True),             # optional int32, dictionary
        ("fk", uniform(n, 0, max(n // 4, 1), np.int64, seed, 2), present(12), True),  # dictionary then PLAIN
        ("price", uniform(n, 90_000, 10_500_000, np.int64, seed, 3), None, False),    # required int64
        ("date", uniform(n, 0, 2525, np.int32, seed, 4), present(14), False),         # optional int32, PLAIN
        ("all_null", np.zeros(n, np.int64), np.zeros(n, bool), True),                 # optional, every row NULL
    ]


def write(path, cols, row_group_size=None, data_page_size=None, version="1.0", compression="NONE",
          dictionary_pagesize_limit=None):
    pa, pq = _arrow()
    fields, arrays = [], []
    for name, vals, mask, _ in cols:
        t = pa.int64() if vals.dtype == np.int64 else pa.int32()
        fields.append(pa.field(name, t, nullable=mask is not None))
        arrays.append(pa.array(vals, t, mask=None if mask is None else ~mask))
    table = pa.Table.from_arrays(arrays, schema=pa.schema(fields))
    kw = {}
    if dictionary_pagesize_limit is not None:
        kw["dictionary_pagesize_limit"] = dictionary_pagesize_limit
    pq.write_table(table, path, compression=compression, row_group_size=row_group_size,
                   data_page_size=data_page_size, data_page_version=version,
                   use_dictionary=[name for name, _, _, d in cols if d], **kw)
    return path
