"""Compressed stream layout and the end-to-end oracle codec.

TEST INFRASTRUCTURE ONLY.

compress(u, e) follows Algorithm 1 of the paper end to end: build the
hierarchy, decompose level by level, quantise level-wise, Huffman-code
(Algorithm 2).  decompress inverts it.  The paper fixes no byte layout; the one
used (all fields little-endian) is:

  off  type      field
    0  u32       magic 0x3143474D ("MGC1")
    4  u16       version (1)
    6  u8        dtype (0 f32, 1 f64)
    7  u8        norm (0 L-inf, 1 L2)
    8  u8        bound mode (0 relative, 1 absolute)
    9  u8        ndim of the user's array (1..3)
   10  u8        flags (bit 0 constant field, bit 1 empty array)
   11  u8        D, number of axes longer than 1
   12  u32       L, number of levels
   16  u64[3]    shape (unused entries 0)
   40  f64       user error bound
   48  f64       tau, the absolute bound
   56  f64       tau', the budget the bins were derived for
   64  f64       value of a constant field
   72  u32       S, dictionary size
   76  u32       C, symbols per chunk
   80  u64       N, number of values
   88  u64       n_codes, symbols with a code
   96  u64       n_outliers
  104  u64       n_chunks
  112  u64       n_words, 32-bit words of coded bits
  120  u64       total stream bytes
  128  f64[L+1]  bins q_0 .. q_L

Then, unless the array is constant or empty, five sections, each starting at
the next multiple of 8 bytes: the codebook (u16 symbols ascending, then their
u8 code lengths), the chunk word offsets (u64[n_chunks+1]), the outlier
positions (u64[n_outliers], ascending), the outlier values (i64[n_outliers])
and the coded words (u32[n_words]).  The stream length is padded to 8 bytes.
"""
from __future__ import annotations

import struct

import numpy as np

from .hierarchy import Hierarchy
from .huffman import canonical_codes, code_lengths, decode_chunks, encode_chunks, histogram
from .quantize import (S_DEFAULT, dequantize, error_budget, from_symbols, level_bins,
                       quantize, to_symbols)
from .transform import decompose, recompose

MAGIC = 0x3143474D
VERSION = 1
HEADER_BYTES = 128
FLAG_CONSTANT = 1
FLAG_EMPTY = 2
_DTYPES = {np.dtype(np.float32): 0, np.dtype(np.float64): 1}
_NORMS = {"linf": 0, "l2": 1}
_MODES = {"rel": 0, "abs": 1}


def _pad8(n: int) -> int:
    return (n + 7) // 8 * 8


def section_offsets(L: int, n_codes: int, n_chunks: int, n_outliers: int, n_words: int):
    """Byte offsets of (codebook, offsets, outlier pos, outlier vals, words, end)."""
    cb = HEADER_BYTES + 8 * (L + 1)
    off = _pad8(cb + 3 * n_codes)
    opos = off + 8 * (n_chunks + 1)
    oval = opos + 8 * n_outliers
    words = oval + 8 * n_outliers
    end = _pad8(words + 4 * n_words)
    return cb, off, opos, oval, words, end


def _header(dtype, norm, mode, shape, flags, D, L, bound, tau, tau_eff, const, S, C,
            N, n_codes, n_out, n_chunks, n_words, total, q) -> bytes:
    shp = list(shape) + [0] * (3 - len(shape))
    b = struct.pack("<IHBBBBBBI3Q4dII6Q", MAGIC, VERSION, _DTYPES[np.dtype(dtype)],
                    _NORMS[norm], _MODES[mode], len(shape), flags, D, L, *shp,
                    bound, tau, tau_eff, const, S, C, N, n_codes, n_out, n_chunks,
                    n_words, total)
    assert len(b) == HEADER_BYTES
    return b + np.asarray(q, dtype="<f8").tobytes()


def parse_header(buf: bytes) -> dict:
    if len(buf) < HEADER_BYTES:
        raise ValueError("stream shorter than its header")
    f = struct.unpack_from("<IHBBBBBBI3Q4dII6Q", buf, 0)
    (magic, ver, dt, nm, md, ndim, flags, D, L, s0, s1, s2, bound, tau, tau_eff,
     const, S, C, N, n_codes, n_out, n_chunks, n_words, total) = f
    if magic != MAGIC or ver != VERSION:
        raise ValueError("bad magic or version")
    if dt not in (0, 1) or nm not in (0, 1) or md not in (0, 1) or not 1 <= ndim <= 3:
        raise ValueError("bad header field")
    if L > 64 or len(buf) < HEADER_BYTES + 8 * (L + 1):
        raise ValueError("truncated header")
    q = np.frombuffer(buf, dtype="<f8", count=L + 1, offset=HEADER_BYTES).copy()
    shape = (s0, s1, s2)[:ndim]
    return dict(dtype=np.float32 if dt == 0 else np.float64,
                norm=["linf", "l2"][nm], mode=["rel", "abs"][md], shape=shape,
                flags=flags, D=D, L=L, bound=bound, tau=tau, tau_eff=tau_eff,
                const=const, S=S, C=C, N=N, n_codes=n_codes, n_outliers=n_out,
                n_chunks=n_chunks, n_words=n_words, total=total, q=q)


def compress(u: np.ndarray, bound: float, norm: str = "linf", mode: str = "rel",
             C: int = 1024, S: int = S_DEFAULT) -> bytes:
    u = np.asarray(u)
    if np.dtype(u.dtype) not in _DTYPES:
        raise TypeError("only float32 and float64 arrays")
    if not 1 <= u.ndim <= 3:
        raise ValueError("ndim must be 1, 2 or 3")
    if not (np.isfinite(bound) and bound > 0):
        raise ValueError("error bound must be positive and finite")
    if norm not in _NORMS or mode not in _MODES:
        raise ValueError("bad norm or mode")
    h = Hierarchy(u.shape)
    common = (u.dtype, norm, mode, u.shape)
    if h.N == 0:
        return _header(*common, FLAG_EMPTY, h.D, 0, bound, 0.0, 0.0, 0.0, S, C, 0, 0, 0,
                       0, 0, HEADER_BYTES + 8, [0.0])
    if not np.all(np.isfinite(u)):
        raise ValueError("input holds NaN or Inf")
    umin, umax = float(u.min()), float(u.max())
    if umin == umax:
        return _header(*common, FLAG_CONSTANT, h.D, 0, bound, 0.0, 0.0, umin, S, C, h.N,
                       0, 0, 0, 0, HEADER_BYTES + 8, [0.0])
    tau, tau_eff = error_budget(u, bound, norm, mode)
    if not tau_eff > 0:
        raise ValueError("error bound below the resolution of the output type")
    q = level_bins(h, tau_eff, norm)
    k = quantize(decompose(u, h), h, q)
    sym, opos, oval = to_symbols(k, S)
    lengths = code_lengths(histogram(sym, S))
    codes = canonical_codes(lengths)
    offsets, words = encode_chunks(sym, lengths, codes, C)
    coded = np.nonzero(lengths)[0]
    n_chunks = len(offsets) - 1
    cb, off, o_pos, o_val, w_off, end = section_offsets(h.L, len(coded), n_chunks,
                                                         len(opos), len(words))
    out = bytearray(end)
    out[0:cb] = _header(*common, 0, h.D, h.L, bound, tau, tau_eff, 0.0, S, C, h.N,
                        len(coded), len(opos), n_chunks, len(words), end, q)
    out[cb:cb + 2 * len(coded)] = coded.astype("<u2").tobytes()
    out[cb + 2 * len(coded):cb + 3 * len(coded)] = lengths[coded].astype("u1").tobytes()
    out[off:o_pos] = offsets.astype("<u8").tobytes()
    out[o_pos:o_val] = opos.astype("<u8").tobytes()
    out[o_val:w_off] = oval.astype("<i8").tobytes()
    out[w_off:w_off + 4 * len(words)] = words.astype("<u4").tobytes()
    return bytes(out)


def decode_symbols(buf: bytes, hd: dict | None = None, chunks=None):
    """The stream's symbols and outliers (no dequantisation).

    With ``chunks`` only those chunks of symbols are decoded (others read 0).
    """
    hd = hd or parse_header(buf)
    cb, off, o_pos, o_val, w_off, end = section_offsets(
        hd["L"], hd["n_codes"], hd["n_chunks"], hd["n_outliers"], hd["n_words"])
    if len(buf) < end or hd["total"] != end:
        raise ValueError("truncated stream")
    nc = hd["n_codes"]
    syms = np.frombuffer(buf, "<u2", nc, cb).astype(np.int64)
    lens = np.frombuffer(buf, "u1", nc, cb + 2 * nc).astype(np.int64)
    lengths = np.zeros(hd["S"], dtype=np.int64)
    lengths[syms] = lens
    offsets = np.frombuffer(buf, "<u8", hd["n_chunks"] + 1, off)
    opos = np.frombuffer(buf, "<u8", hd["n_outliers"], o_pos)
    oval = np.frombuffer(buf, "<i8", hd["n_outliers"], o_val)
    words = np.frombuffer(buf, "<u4", hd["n_words"], w_off)
    sym = decode_chunks(words, offsets, lengths, hd["N"], hd["C"], chunks)
    return sym, opos, oval


def decompress(buf: bytes) -> np.ndarray:
    hd = parse_header(buf)
    shape, dt = hd["shape"], hd["dtype"]
    if hd["flags"] & FLAG_EMPTY:
        return np.zeros(shape, dtype=dt)
    if hd["flags"] & FLAG_CONSTANT:
        return np.full(shape, hd["const"], dtype=dt)
    h = Hierarchy(shape)
    if h.L != hd["L"] or h.N != hd["N"]:
        raise ValueError("header inconsistent with its shape")
    sym, opos, oval = decode_symbols(buf, hd)
    k = from_symbols(sym, opos, oval, hd["S"])
    coeffs = dequantize(k, h, hd["q"])
    return recompose(coeffs, h).astype(dt)
