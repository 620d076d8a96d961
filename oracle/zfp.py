"""Fixed-rate block transform coding (ZFP-X; oracle, test infrastructure).

TEST INFRASTRUCTURE ONLY.

Algorithm "ZFP Fix-Rate Compression" of the paper (Section IV-C) cuts the
array into blocks of 4^d values, aligns each block's values to its largest
exponent as fixed-point integers, applies a near-orthogonal decorrelating
transform, and keeps a fixed number of bits per block by truncating the
coefficients' bit planes.  The paper prints no constants; the readings used:

* blocks: 4 values along every axis (d = number of axes, 1..3), in row-major
  block order; a partial block at the high end of an axis repeats the axis'
  last value;
* alignment: e = the exponent of the block's largest magnitude
  (max|x| = f 2^e with 0.5 <= f < 1); each value becomes
  trunc(x 2^(q - e)) with q = P - 2 - d, where P = 32 (float32) or 64
  (float64) is the integer width; a block of zeros has no exponent;
* transform: per axis (the last axis first, then the others towards axis 0)
  two levels of the reversible integer Haar lifting on the 4 values of a
  line: (a, b) -> (s, t) with t = a - b and s = b + floor(t / 2), first on
  (v0, v1) and (v2, v3), then on their two s values; the line becomes
  (S, T, t0, t1), frequencies 0, 1, 2, 2.  A difference at most doubles the
  magnitudes and an average never grows them, so |coefficients| < 2^(P-2);
* order: coefficients sorted by the sum of their per-axis frequencies
  (stable in row-major position within the block);
* negabinary: u = ((i + M) xor M) mod 2^P with M = the P-bit pattern
  1010...10 (the base -2 digits of i), so that magnitude sits in the high
  planes and no sign bit is needed;
* bit-plane coding of the n = 4^d coefficients under a budget of
  maxbits = round(rate n) bits per block: one bit "block not zero", then
  (if not zero) the exponent e + bias (9 bits, bias 149, for float32; 12 bits,
  bias 1074, for float64), then planes from P - 1 down: the plane's bits of
  the m coefficients already found significant, verbatim; then, while
  coefficients remain, a group bit (does any remaining coefficient have a 1
  in this plane?) and, if so, the remaining coefficients' bits one by one up
  to and including the next 1 (the last coefficient's 1 is implied, not
  written), which makes that coefficient significant.  Coding stops when the
  budget is spent; the rest of the block's bits are zeros.  The decoder runs
  the same steps reading bits (missing planes read as zeros).

Stream (little-endian): u32 magic 0x465A474D, u8 dtype (0 float32, 1
float64), u8 ndim, u16 0, u32 maxbits, u32 0, u64 shape[3], f64 rate, u64
blocks, u64 total bytes (64-byte header); then the blocks' bits, block b at
bits [b maxbits, (b + 1) maxbits) of a sequence of u64 words in which bit j
is bit j mod 64 of word j / 64; zero padding to a multiple of 8 bytes.
"""
from __future__ import annotations

import struct

import numpy as np

MAGIC = 0x465A474D
HEADER_BYTES = 64
_DT = {np.dtype(np.float32): 0, np.dtype(np.float64): 1}


def params(dtype, ndim: int):
    """(P, q, exponent bits, exponent bias) of a dtype and block dimension."""
    P = 32 if np.dtype(dtype) == np.float32 else 64
    eb, bias = (9, 149) if P == 32 else (12, 1074)
    return P, P - 2 - ndim, eb, bias


def maxbits_of(rate: float, ndim: int) -> int:
    return int(round(rate * 4 ** ndim))


# ------------------------------------------------------------------ blocks
def blocks_of(u: np.ndarray) -> np.ndarray:
    """[n_blocks, 4^d] values in row-major block order, partial blocks padded
    by repeating each axis' last value."""
    d = u.ndim
    nb = [(n + 3) // 4 for n in u.shape]
    idx = [np.minimum(np.arange(4 * m), n - 1) for m, n in zip(nb, u.shape)]
    padded = u[np.ix_(*idx)]
    # split every axis into (block, 4) and bring the block indices first
    shp = []
    for m in nb:
        shp += [m, 4]
    b = padded.reshape(shp)
    order = list(range(0, 2 * d, 2)) + list(range(1, 2 * d, 2))
    return b.transpose(order).reshape(int(np.prod(nb)), 4 ** d)


def unblock(blk: np.ndarray, shape) -> np.ndarray:
    d = len(shape)
    nb = [(n + 3) // 4 for n in shape]
    b = blk.reshape(nb + [4] * d)
    order = []
    for k in range(d):
        order += [k, d + k]
    full = b.transpose(order).reshape([4 * m for m in nb])
    return full[tuple(slice(0, n) for n in shape)]


# --------------------------------------------------------------- alignment
def block_exponent(vals: np.ndarray) -> np.ndarray:
    """e per block (max|x| = f 2^e, 0.5 <= f < 1); 0 where the block is zero."""
    m = np.max(np.abs(vals.astype(np.float64)), axis=1)
    _, e = np.frexp(m)
    return np.where(m > 0, e, 0).astype(np.int64)


def to_fixed(vals: np.ndarray, e: np.ndarray, q: int) -> np.ndarray:
    """trunc(x 2^(q - e)) per value (exact: a power-of-two scaling in FP64)."""
    x = np.ldexp(vals.astype(np.float64), (q - e)[:, None])
    return np.trunc(x).astype(np.int64)


def from_fixed(ints: np.ndarray, e: np.ndarray, q: int) -> np.ndarray:
    return np.ldexp(ints.astype(np.float64), (e - q)[:, None])


# --------------------------------------------------------------- transform
def _lift(a, b):
    t = a - b
    return b + (t >> 1), t          # floor(t / 2) by an arithmetic shift


def _unlift(s, t):
    b = s - (t >> 1)
    return b + t, b


def _fwd_line(v):
    s0, t0 = _lift(v[0], v[1])
    s1, t1 = _lift(v[2], v[3])
    S, T = _lift(s0, s1)
    return [S, T, t0, t1]


def _inv_line(c):
    s0, s1 = _unlift(c[0], c[1])
    v0, v1 = _unlift(s0, c[2])
    v2, v3 = _unlift(s1, c[3])
    return [v0, v1, v2, v3]


def forward(ints: np.ndarray, d: int) -> np.ndarray:
    """Per-axis transform of [n_blocks, 4^d] integers, last axis first."""
    x = ints.reshape((-1,) + (4,) * d).copy()
    for ax in range(d, 0, -1):
        x = np.moveaxis(x, ax, -1)
        y = _fwd_line([x[..., k] for k in range(4)])
        x = np.moveaxis(np.stack(y, axis=-1), -1, ax)
    return x.reshape(ints.shape)


def inverse(coef: np.ndarray, d: int) -> np.ndarray:
    x = coef.reshape((-1,) + (4,) * d).copy()
    for ax in range(1, d + 1):
        x = np.moveaxis(x, ax, -1)
        y = _inv_line([x[..., k] for k in range(4)])
        x = np.moveaxis(np.stack(y, axis=-1), -1, ax)
    return x.reshape(coef.shape)


FREQ = (0, 1, 2, 2)


def order(d: int) -> np.ndarray:
    """Block positions sorted by total frequency (stable in position)."""
    pos = list(np.ndindex(*(4,) * d))
    key = [sum(FREQ[i] for i in p) for p in pos]
    return np.array(sorted(range(len(pos)), key=lambda k: (key[k], k)), dtype=np.int64)


# -------------------------------------------------------------- negabinary
def to_negabinary(i: np.ndarray, P: int) -> np.ndarray:
    mask = (1 << P) - 1
    M = int("10" * (P // 2), 2)
    return np.array([((int(v) + M) & mask) ^ M for v in i.ravel()], dtype=object).reshape(i.shape)


def from_negabinary(u, P: int) -> np.ndarray:
    mask = (1 << P) - 1
    M = int("10" * (P // 2), 2)
    out = []
    for v in np.asarray(u, dtype=object).ravel():
        x = ((int(v) ^ M) - M) & mask
        if x >> (P - 1):
            x -= 1 << P
        out.append(x)
    return np.array(out, dtype=np.int64).reshape(np.shape(u))


# ---------------------------------------------------------- bit-plane coder
def encode_planes(u, P: int, budget: int):
    """Bits (list of 0/1) of the n coefficients u (negabinary, P bits)
    under a budget of bits."""
    n = len(u)
    bits = []
    m = 0
    B = budget
    for k in range(P - 1, -1, -1):
        if B == 0:
            break
        x = 0
        for i in range(n):
            x |= ((int(u[i]) >> k) & 1) << i
        t = min(m, B)
        for i in range(t):
            bits.append((x >> i) & 1)
        B -= t
        if t < m:
            break
        x >>= m
        while m < n and B > 0:
            g = 1 if x else 0
            bits.append(g)
            B -= 1
            if not g:
                break
            while True:
                if m == n - 1:          # the last coefficient's one is implied
                    x >>= 1
                    m += 1
                    break
                if B == 0:
                    break
                b = x & 1
                bits.append(b)
                B -= 1
                x >>= 1
                m += 1
                if b:
                    break
    return bits


def decode_planes(read, n: int, P: int, budget: int):
    """Inverse of encode_planes; ``read()`` returns the next bit."""
    u = [0] * n
    m = 0
    B = budget
    for k in range(P - 1, -1, -1):
        if B == 0:
            break
        t = min(m, B)
        for i in range(t):
            u[i] |= read() << k
        B -= t
        if t < m:
            break
        while m < n and B > 0:
            g = read()
            B -= 1
            if not g:
                break
            while True:
                if m == n - 1:
                    u[m] |= 1 << k
                    m += 1
                    break
                if B == 0:
                    break
                b = read()
                B -= 1
                if b:
                    u[m] |= 1 << k
                m += 1
                if b:
                    break
    return u


# ------------------------------------------------------------------ codec
def compress(u: np.ndarray, rate: float) -> bytes:
    u = np.asarray(u)
    if np.dtype(u.dtype) not in _DT:
        raise TypeError("float32 or float64 arrays only")
    if not 1 <= u.ndim <= 3 or u.size == 0:
        raise ValueError("ndim must be 1..3 and the array non-empty")
    if not np.all(np.isfinite(u)):
        raise ValueError("input holds NaN or Inf")
    d = u.ndim
    P, q, eb, bias = params(u.dtype, d)
    n = 4 ** d
    mb = maxbits_of(rate, d)
    if mb < 1 + eb + 1 or rate > 2 * P:
        raise ValueError("rate out of range")
    blk = blocks_of(u)
    e = block_exponent(blk)
    zero = np.max(np.abs(blk.astype(np.float64)), axis=1) == 0
    coef = forward(to_fixed(blk, e, q), d)[:, order(d)]
    nblk = len(blk)
    total_bits = nblk * mb
    words = np.zeros((total_bits + 63) // 64, dtype=np.uint64)
    stream_bits = np.zeros(total_bits, dtype=np.uint8)
    for b in range(nblk):
        out = [0 if zero[b] else 1]
        if not zero[b]:
            v = int(e[b]) + bias
            out += [(v >> j) & 1 for j in range(eb)]
            out += encode_planes(to_negabinary(coef[b], P), P, mb - 1 - eb)
        stream_bits[b * mb:b * mb + len(out)] = out
    # bit j of the stream is bit j mod 64 of word j / 64
    padded = np.zeros(len(words) * 64, dtype=np.uint8)
    padded[:total_bits] = stream_bits
    words = np.packbits(padded.reshape(-1, 64)[:, ::-1], axis=1).view(">u8").ravel().astype(np.uint64)
    total = HEADER_BYTES + 8 * len(words)
    shp = list(u.shape) + [0] * (3 - d)
    head = struct.pack("<IBBHII3QdQQ", MAGIC, _DT[np.dtype(u.dtype)], d, 0, mb, 0, *shp,
                       float(rate), nblk, total)
    return head + words.astype("<u8").tobytes()


def parse_header(buf: bytes) -> dict:
    magic, dt, d, _, mb, _, s0, s1, s2, rate, nblk, total = struct.unpack_from(
        "<IBBHII3QdQQ", buf, 0)
    if magic != MAGIC:
        raise ValueError("not a ZFP-X stream")
    return dict(dtype=np.float32 if dt == 0 else np.float64, ndim=d, maxbits=mb,
                shape=(s0, s1, s2)[:d], rate=rate, blocks=nblk, total=total)


def decompress(buf: bytes) -> np.ndarray:
    h = parse_header(buf)
    d, mb, nblk = h["ndim"], h["maxbits"], h["blocks"]
    P, q, eb, bias = params(h["dtype"], d)
    n = 4 ** d
    words = np.frombuffer(buf, dtype="<u8", offset=HEADER_BYTES).astype(np.uint64)
    bits = np.unpackbits(words.astype(">u8").view(np.uint8).reshape(-1, 8), axis=1)
    bits = bits.reshape(-1, 64)[:, ::-1].ravel()
    coef = np.zeros((nblk, n), dtype=np.int64)
    e = np.zeros(nblk, dtype=np.int64)
    for b in range(nblk):
        pos = [b * mb]

        def read():
            v = int(bits[pos[0]])
            pos[0] += 1
            return v

        if not read():
            continue
        v = 0
        for j in range(eb):
            v |= read() << j
        e[b] = v - bias
        coef[b] = from_negabinary(decode_planes(read, n, P, mb - 1 - eb), P)
    ints = np.zeros_like(coef)
    ints[:, order(d)] = coef
    vals = from_fixed(inverse(ints, d), e, q)
    return unblock(vals.astype(h["dtype"]), h["shape"])
