"""A minimal Parquet writer and Snappy encoder for tests: one required INT64
column, one row group, PLAIN data pages whose Snappy bodies are built element
by element, so that a test can place copies where the reference compressor
never does (further back than 64 KiB, across 64 KiB output fragments). The
format is written from its published Thrift definitions; pyarrow reading the
file back confirms that it is valid Parquet and valid Snappy."""
import struct


# ---------------------------------------------------------------- Thrift compact protocol

def _varint(n):
    out = bytearray()
    while True:
        b = n & 0x7F
        n >>= 7
        if n:
            out.append(b | 0x80)
        else:
            out.append(b)
            return bytes(out)


def _zz(n):
    return _varint((n << 1) ^ (n >> 63))


class _Struct:
    """Fields are (id, type, value); types: 'i32', 'i64', 'bin', 'list_i32', 'list_bin', 'list_struct', 'struct'."""

    def __init__(self, *fields):
        self.fields = fields

    def encode(self):
        out = bytearray()
        last = 0
        codes = {"i32": 5, "i64": 6, "bin": 8, "list_i32": 9, "list_bin": 9, "list_struct": 9, "struct": 12}
        for fid, t, v in self.fields:
            code = codes[t]
            d = fid - last
            out += bytes([(d << 4) | code]) if 0 < d <= 15 else bytes([code]) + _zz(fid)
            last = fid
            if t in ("i32", "i64"):
                out += _zz(v)
            elif t == "bin":
                b = v.encode() if isinstance(v, str) else v
                out += _varint(len(b)) + b
            elif t == "struct":
                out += v.encode()
            else:
                et = {"list_i32": 5, "list_bin": 8, "list_struct": 12}[t]
                out += bytes([(len(v) << 4) | et]) if len(v) < 15 else bytes([0xF0 | et]) + _varint(len(v))
                for x in v:
                    if t == "list_i32":
                        out += _zz(x)
                    elif t == "list_bin":
                        b = x.encode() if isinstance(x, str) else x
                        out += _varint(len(b)) + b
                    else:
                        out += x.encode()
        out.append(0)
        return bytes(out)


# ---------------------------------------------------------------- Snappy elements

def literal(data):
    n = len(data) - 1
    if n < 60:
        return bytes([n << 2]) + data
    nb = (n.bit_length() + 7) // 8
    return bytes([(59 + nb) << 2]) + n.to_bytes(nb, "little") + data


def copy(offset, length):
    """One copy element (length 1..64); 4-byte offsets when the offset needs them."""
    assert 1 <= length <= 64 and offset >= 1
    if offset < 65536:
        return bytes([((length - 1) << 2) | 2]) + struct.pack("<H", offset)
    return bytes([((length - 1) << 2) | 3]) + struct.pack("<I", offset)


def snappy_block(elements, out_len):
    return _varint(out_len) + b"".join(elements)


# ---------------------------------------------------------------- the file

def write(path, bodies, values_per_page, codec=1):
    """bodies[i]: the stored body of data page i (PLAIN int64 values, Snappy-
    compressed when codec == 1); values_per_page[i]: its value count."""
    out = bytearray(b"PAR1")
    data_off = len(out)
    total_u = total_c = 0
    for body, nv in zip(bodies, values_per_page):
        usize = nv * 8
        hdr = _Struct((1, "i32", 0), (2, "i32", usize), (3, "i32", len(body)),
                      (5, "struct", _Struct((1, "i32", nv), (2, "i32", 0), (3, "i32", 3), (4, "i32", 3)))).encode()
        out += hdr + body
        total_u += len(hdr) + usize
        total_c += len(hdr) + len(body)
    n = sum(values_per_page)
    meta = _Struct((1, "i32", 2), (2, "list_i32", [0]), (3, "list_bin", ["x"]), (4, "i32", codec), (5, "i64", n),
                   (6, "i64", total_u), (7, "i64", total_c), (9, "i64", data_off))
    chunk = _Struct((2, "i64", data_off), (3, "struct", meta))
    rg = _Struct((1, "list_struct", [chunk]), (2, "i64", total_u), (3, "i64", n))
    schema = [_Struct((4, "bin", "schema"), (5, "i32", 1)), _Struct((1, "i32", 2), (3, "i32", 0), (4, "bin", "x"))]
    fmd = _Struct((1, "i32", 1), (2, "list_struct", schema), (3, "i64", n), (4, "list_struct", [rg])).encode()
    out += fmd + struct.pack("<I", len(fmd)) + b"PAR1"
    with open(path, "wb") as f:
        f.write(out)
    return path
