"""Tables resident in host page-pool pages, as batches over page chains.

A batch holds `rows_per_batch` rows of every column; its columns follow each
other in the byte stream of its page chain (256-byte aligned, possibly
straddling pages), as laid out by tq_batch_layout. Filling and reading split
each column at page boundaries (a boundary never cuts a value: pages and
column offsets are multiples of 256 bytes).
"""
from __future__ import annotations

import ctypes
from typing import Callable, Dict, List, Sequence, Tuple

import numpy as np

from . import tq

_TYPE = {np.dtype(np.uint8): tq.TQ_U8, np.dtype(np.int32): tq.TQ_I32, np.dtype(np.int64): tq.TQ_I64}


class HostTable:
    def __init__(self, pool: tq.PagePool, columns: Sequence[Tuple[str, type]], nrows: int, rows_per_batch: int):
        self.pool = pool
        self.names = [c for c, _ in columns]
        self.dtypes = [np.dtype(d) for _, d in columns]
        self.types = [_TYPE[d] for d in self.dtypes]
        self.nrows = nrows
        self.batches: List[Tuple[int, int, List[int], List[int]]] = []  # (first row, rows, offsets, page ids)
        try:
            for start in range(0, nrows, rows_per_batch):
                n = min(rows_per_batch, nrows - start)
                offs, _nbytes, npages = tq.batch_layout(n, self.types, pool.page_bytes)
                ids = pool.alloc(npages)
                self.batches.append((start, n, offs, ids))
        except Exception:
            self.free()
            raise

    def col_index(self, name: str) -> int:
        return self.names.index(name)

    def pieces(self, b: int, c: int):
        """(host address, first global row, rows) segments of column c of batch b."""
        start, n, offs, ids = self.batches[b]
        w = self.dtypes[c].itemsize
        pb = self.pool.page_bytes
        pos, row, left = offs[c], 0, n
        while left > 0:
            page, within = divmod(pos, pb)
            take = min(left, (pb - within) // w)
            yield self.pool.page(ids[page]) + within, start + row, take
            pos += take * w
            row += take
            left -= take

    def fill(self, fn: Callable[[str, int, int, int], None]):
        """fn(column name, host address, first row, rows) writes the values."""
        for b in range(len(self.batches)):
            for c, name in enumerate(self.names):
                for addr, first, count in self.pieces(b, c):
                    fn(name, addr, first, count)

    def fill_numpy(self, arrays: Dict[str, np.ndarray]):
        def put(name, addr, first, count):
            a = np.ascontiguousarray(arrays[name][first:first + count], dtype=self.dtypes[self.col_index(name)])
            ctypes.memmove(addr, a.ctypes.data, a.nbytes)
        self.fill(put)

    def read_column(self, name: str) -> np.ndarray:
        c = self.col_index(name)
        out = np.empty(self.nrows, dtype=self.dtypes[c])
        for b in range(len(self.batches)):
            for addr, first, count in self.pieces(b, c):
                ctypes.memmove(out[first:first + count].ctypes.data, addr, count * self.dtypes[c].itemsize)
        return out

    def c_batches(self):
        """(ctypes array of tq_batch, objects that must stay alive while it is used)."""
        arr = (tq.Batch * max(1, len(self.batches)))()
        keep = []
        for i, (_start, n, offs, ids) in enumerate(self.batches):
            p = (ctypes.c_int32 * max(1, len(ids)))(*ids)
            o = (ctypes.c_int64 * len(offs))(*offs)
            t = (ctypes.c_int32 * len(self.types))(*self.types)
            keep += [p, o, t]
            arr[i] = tq.Batch(len(ids), p, n, len(self.types), o, t)
        if not self.batches:
            arr = (tq.Batch * 0)()
        return arr, keep

    def max_batch_bytes(self) -> int:
        return max((len(ids) for _, _, _, ids in self.batches), default=0) * self.pool.page_bytes

    def free(self):
        for _, _, _, ids in self.batches:
            self.pool.free(ids)
        self.batches = []
