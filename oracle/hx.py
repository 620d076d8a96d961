"""Huffman-X: the Huffman pipeline as a standalone lossless codec (oracle).

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
benchmark's CPU-baseline leg may import this module.

Algorithm 2 of the paper compresses a stream of keys losslessly: histogram,
sort by frequency, drop the zero-frequency keys, build the code, encode,
serialise (Section IV-B).  The paper evaluates it on its own as one of its
reduction kernels (Section VI-B) without fixing how a stream of arbitrary
integers becomes keys.  The reading used here:

* Byte streams (u8) and 16-bit streams (u16): every value is its own key
  (dictionaries of 256 and 65536 keys); nothing is escaped.
* Signed 32- and 64-bit streams (i32, i64) with a dictionary of D keys
  (2 <= D <= 65536) and a base b: a value v with b <= v <= b + D - 2 is key
  v - b; every other value is key D - 1 (the escape key) and is stored raw,
  after the coded section, in the order of its position.  The position of
  the k-th escaped value is the position of the k-th escape key.

Code construction, canonical codes and the chunked bit layout are those of
``huffman`` (the compressor's Huffman stage).  Byte layout (little-endian):

  off  type  field
    0  u32   magic 0x5848474D ("MGHX")
    4  u8    value type (0 u8, 1 u16, 2 i32, 3 i64)
    5  u8[3] zero
    8  u32   D, dictionary size (escape key included)
   12  u32   C, keys per chunk
   16  i64   b, base
   24  u64   n, number of values
   32  u64   number of escaped values
   40  u64   length of the coded section (0 when n = 0)
   48  u64   total stream bytes
   56  u64   zero

then the coded section (the Huffman stage's own stream: a 48-byte header
u32 0x3148474D, u32 C, u64 n, n_codes, n_chunks, n_words, total; the
codebook (u16 keys ascending, then their u8 code lengths); u64 chunk word
offsets; u32 coded words; each section starting on a multiple of 8 bytes),
then the escaped values (n_escaped values of the stream's type), the stream
padded with zeros to a multiple of 8 bytes.
"""
from __future__ import annotations

import struct

import numpy as np

from .huffman import canonical_codes, code_lengths, decode_chunks, encode_chunks, histogram

MAGIC = 0x5848474D
HUFF_MAGIC = 0x3148474D
HEADER_BYTES = 64
HUFF_HEADER_BYTES = 48
TYPES = {0: np.dtype("<u1"), 1: np.dtype("<u2"), 2: np.dtype("<i4"), 3: np.dtype("<i8")}
FULL_DICT = {0: 256, 1: 65536}
MAX_DICT = 65536


def _pad8(n: int) -> int:
    return (n + 7) // 8 * 8


def type_code(dtype) -> int:
    dt = np.dtype(dtype).newbyteorder("<")
    for k, v in TYPES.items():
        if v == dt:
            return k
    raise TypeError("value type must be uint8, uint16, int32 or int64")


def default_dict_base(t: int):
    """Dictionary and base used when the caller gives none: the full range
    for u8 and u16; 65536 keys centred on zero for i32 and i64."""
    if t in FULL_DICT:
        return FULL_DICT[t], 0
    return MAX_DICT, -(MAX_DICT // 2 - 1)


def check_params(t: int, D: int, b: int) -> None:
    if t in FULL_DICT:
        if D != FULL_DICT[t] or b != 0:
            raise ValueError("u8 and u16 streams use their full range as the dictionary")
        return
    if not 2 <= D <= MAX_DICT:
        raise ValueError("dictionary size must be in [2, 65536]")
    info = np.iinfo(TYPES[t])
    if not info.min <= b <= info.max:
        raise ValueError("base outside the value type")


def keys(values: np.ndarray, t: int, D: int, b: int):
    """(keys int64[n], escaped values in position order) of a value stream."""
    v = np.asarray(values)
    if t in FULL_DICT:
        return v.astype(np.int64), np.zeros(0, dtype=TYPES[t])
    hi = b + D - 2                      # last value with a key of its own (Python int)
    info = np.iinfo(TYPES[t])
    inside = v >= b
    if hi < info.max:
        inside &= v <= hi
    k = np.full(len(v), D - 1, dtype=np.int64)
    # v - b of an in-range value fits in [0, D - 2]; compute it without overflow
    k[inside] = (v[inside].astype(object) - b).astype(np.int64)
    return k, v[~inside].astype(TYPES[t])


def values_from_keys(k: np.ndarray, esc: np.ndarray, t: int, D: int, b: int) -> np.ndarray:
    """Inverse of ``keys``."""
    k = np.asarray(k, dtype=np.int64)
    if t in FULL_DICT:
        return k.astype(TYPES[t])
    out = np.zeros(len(k), dtype=TYPES[t])
    e = k == D - 1
    if int(e.sum()) != len(esc):
        raise ValueError("escape count does not match the escaped values")
    out[e] = esc
    out[~e] = (k[~e].astype(object) + b).astype(TYPES[t])
    return out


def huffman_section(sym: np.ndarray, C: int) -> bytes:
    """The Huffman stage's standalone stream for keys ``sym`` (Algorithm 2:
    histogram, code from the non-zero frequencies, encode, serialise)."""
    N = len(sym)
    ln = code_lengths(histogram(sym, MAX_DICT))
    codes = canonical_codes(ln)
    off, words = encode_chunks(sym, ln, codes, C)
    coded = np.nonzero(ln)[0]
    nc = len(coded)
    n_chunks = len(off) - 1
    o_off = _pad8(HUFF_HEADER_BYTES + 3 * nc)
    w_off = o_off + 8 * (n_chunks + 1)
    end = _pad8(w_off + 4 * len(words))
    out = bytearray(end)
    out[0:HUFF_HEADER_BYTES] = struct.pack("<II5Q", HUFF_MAGIC, C, N, nc, n_chunks, len(words), end)
    out[HUFF_HEADER_BYTES:HUFF_HEADER_BYTES + 2 * nc] = coded.astype("<u2").tobytes()
    out[HUFF_HEADER_BYTES + 2 * nc:HUFF_HEADER_BYTES + 3 * nc] = ln[coded].astype("u1").tobytes()
    out[o_off:w_off] = off.astype("<u8").tobytes()
    out[w_off:w_off + 4 * len(words)] = words.astype("<u4").tobytes()
    return bytes(out)


def decode_huffman_section(buf: bytes, n: int) -> np.ndarray:
    magic, C, N, nc, n_chunks, n_words, total = struct.unpack_from("<II5Q", buf, 0)
    if magic != HUFF_MAGIC or N != n or total > len(buf):
        raise ValueError("bad coded section")
    ln = np.zeros(MAX_DICT, dtype=np.int64)
    coded = np.frombuffer(buf, dtype="<u2", count=nc, offset=HUFF_HEADER_BYTES).astype(np.int64)
    ln[coded] = np.frombuffer(buf, dtype="u1", count=nc, offset=HUFF_HEADER_BYTES + 2 * nc)
    o_off = _pad8(HUFF_HEADER_BYTES + 3 * nc)
    off = np.frombuffer(buf, dtype="<u8", count=n_chunks + 1, offset=o_off)
    w_off = o_off + 8 * (n_chunks + 1)
    words = np.frombuffer(buf, dtype="<u4", count=n_words, offset=w_off)
    return decode_chunks(words, off, ln, n, C)


def compress(values, D: int | None = None, b: int | None = None, C: int = 1024) -> bytes:
    v = np.ascontiguousarray(values).reshape(-1)
    t = type_code(v.dtype)
    d0, b0 = default_dict_base(t)
    D = d0 if D is None else int(D)
    b = b0 if b is None else int(b)
    check_params(t, D, b)
    if not (64 <= C <= 65536 and C % 64 == 0):
        raise ValueError("chunk size must be a multiple of 64 in [64, 65536]")
    n = len(v)
    k, esc = keys(v, t, D, b)
    sec = huffman_section(k, C) if n else b""
    eb = esc.astype(TYPES[t]).tobytes()
    total = HEADER_BYTES + len(sec) + _pad8(len(eb))
    out = bytearray(total)
    out[0:HEADER_BYTES] = struct.pack("<IB3xIIqQQQQQ", MAGIC, t, D, C, b, n, len(esc), len(sec),
                                      total, 0)
    out[HEADER_BYTES:HEADER_BYTES + len(sec)] = sec
    out[HEADER_BYTES + len(sec):HEADER_BYTES + len(sec) + len(eb)] = eb
    return bytes(out)


def parse_header(buf: bytes) -> dict:
    if len(buf) < HEADER_BYTES:
        raise ValueError("stream shorter than its header")
    magic, t, D, C, b, n, n_esc, sec, total, _ = struct.unpack_from("<IB3xIIqQQQQQ", buf, 0)
    if magic != MAGIC or t not in TYPES:
        raise ValueError("bad magic or value type")
    return dict(type=t, D=D, C=C, base=b, n=n, n_escaped=n_esc, section=sec, total=total)


def decompress(buf: bytes) -> np.ndarray:
    h = parse_header(buf)
    t, n = h["type"], h["n"]
    check_params(t, h["D"], h["base"])
    if h["total"] != HEADER_BYTES + h["section"] + _pad8(h["n_escaped"] * TYPES[t].itemsize) \
            or h["total"] > len(buf):
        raise ValueError("inconsistent stream length")
    if n == 0:
        return np.zeros(0, dtype=TYPES[t])
    k = decode_huffman_section(buf[HEADER_BYTES:HEADER_BYTES + h["section"]], n)
    esc = np.frombuffer(buf, dtype=TYPES[t], count=h["n_escaped"],
                        offset=HEADER_BYTES + h["section"])
    return values_from_keys(k, esc, t, h["D"], h["base"])
