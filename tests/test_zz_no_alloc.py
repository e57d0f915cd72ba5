"""The partition entry point that allocates nothing (tq_hash_partition_noalloc):
its outputs against those of tq_hash_partition (caller scratch) and the oracle,
on two calls in a row through the C ABI, the second one smaller, so that what
the first call left in the fixed scratch area must not leak into the second."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_2508_05029_amd import tq  # noqa: E402
from paper_2508_05029_amd.datagen import uniform  # noqa: E402

DEV = "cuda"


def _inputs(n, seed):
    keys = uniform(n, -(2 ** 62), 2 ** 62, np.int64, seed, 0)
    p64 = uniform(n, -10**15, 10**15, np.int64, seed, 1)
    p32 = uniform(n, -10**9, 10**9, np.int32, seed, 2)
    p8 = uniform(n, 0, 255, np.uint8, seed, 3)
    return [keys, p64, p32, p8]


def _run(fn, host, bits, skip):
    n = len(host[0])
    d = [torch.from_numpy(a).to(DEV) for a in host]
    out = [torch.full((max(n, 1),), 7, dtype=t.dtype, device=DEV) for t in d]
    offs = torch.full(((1 << bits) + 1,), -1, dtype=torch.int64, device=DEV)
    fn(d, out, offs)
    torch.cuda.synchronize()
    return offs.cpu().numpy(), [o[:n].cpu().numpy() for o in out]


def _by_partition(offs, cols, bits):
    """The rows sorted by (partition, then every column): the order inside a
    partition is unspecified, so two outputs are compared in this form."""
    part = np.repeat(np.arange(1 << bits), np.diff(offs))
    order = np.lexsort(tuple(reversed(cols)) + (part,))
    return [c[order].tolist() for c in cols]


@pytest.mark.parametrize("calls", [[(1_000_003, 8, 0, 31), (70_001, 6, 3, 32)],
                                   [(4096 * 200, 10, 0, 33), (1, 0, 0, 34)]])
def test_noalloc_partition_equals_scratch_partition(calls):
    for n, bits, skip, seed in calls:
        print(f"noalloc partition n={n} bits={bits} skip={skip} seed={seed}", flush=True)
        sys.stdout.flush()
        host = _inputs(n, seed)
        assert tq.hash_partition_scratch_bytes(n, bits) <= tq.PARTITION_STATIC_SCRATCH_BYTES
        scratch = torch.empty(max(1, tq.hash_partition_scratch_bytes(n, bits)), dtype=torch.uint8, device=DEV)
        ref_offs, ref_cols = _run(lambda d, o, f: tq.hash_partition(d[0], d[1:], n, bits, skip, o[0], o[1:], f, scratch),
                                  host, bits, skip)
        got_offs, got_cols = _run(lambda d, o, f: tq.hash_partition_noalloc(d[0], d[1:], n, bits, skip, o[0], o[1:], f),
                                  host, bits, skip)
        assert got_offs.tolist() == ref_offs.tolist()
        assert _by_partition(got_offs, got_cols, bits) == _by_partition(ref_offs, ref_cols, bits)
        # and the partition definition itself (the oracle's ids: the top bits, below `skip` ones)
        pid = oracle.partition_ids(host[0], bits + skip) & ((1 << bits) - 1) if (skip and bits) else \
            oracle.partition_ids(host[0], bits)
        want_offs = np.concatenate([[0], np.cumsum(np.bincount(pid, minlength=1 << bits))])
        assert got_offs.tolist() == want_offs.tolist()


def test_noalloc_partition_rejects_sizes_beyond_the_area():
    n, bits = 5_000_000, 10
    assert tq.hash_partition_scratch_bytes(n, bits) > tq.PARTITION_STATIC_SCRATCH_BYTES
    keys = torch.zeros(n, dtype=torch.int64, device=DEV)
    out = torch.empty_like(keys)
    offs = torch.empty((1 << bits) + 1, dtype=torch.int64, device=DEV)
    with pytest.raises(tq.TqError) as e:
        tq.hash_partition_noalloc(keys, [], n, bits, 0, out, [], offs)
    assert e.value.status == tq.TQ_EINVAL
