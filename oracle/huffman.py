"""Huffman coding of the quantised symbols (oracle; test infrastructure).

Follows Algorithm 2 of the paper (histogram, sort by frequency, drop the
zero-frequency keys, build the code, encode, serialise).  The paper defers
the code construction to its citations and fixes no tie rule, length limit or
bit layout; the readings used here:

* Code lengths: the alphabet is the symbols with non-zero frequency, sorted by
  (frequency, symbol).  Two queues - the sorted leaves and the internal nodes
  in creation order - and at each step the smaller front is taken, a tie going
  to the leaf; two taken nodes make an internal node whose weight is their
  sum.  A symbol's length is its depth.  A one-symbol alphabet has length 1.
  If the longest code exceeds 32 bits every frequency f > 0 becomes ceil(f/2)
  and the lengths are rebuilt (repeated as needed).
* Canonical codes: order the coded symbols by (length, symbol); the first gets
  code 0 and code_{i+1} = (code_i + 1) << (len_{i+1} - len_i) (the canonical
  construction of RFC 1951).
* Bit layout: symbols are cut into chunks of C; inside a chunk the codes are
  appended most-significant bit first into 32-bit words (the first bit is
  bit 31 of the chunk's first word); every chunk starts on a word boundary;
  a table of n_chunks + 1 word offsets locates the chunks.
"""
from __future__ import annotations

from collections import deque

import numpy as np

MAX_LEN = 32


def histogram(sym: np.ndarray, S: int) -> np.ndarray:
    return np.bincount(sym.astype(np.int64), minlength=S).astype(np.int64)


def _two_queue_depths(weights):
    """Depth of each leaf; ``weights`` ascending (ties already ordered)."""
    n = len(weights)
    if n == 1:
        return [1]
    w = list(weights)
    parent = [0] * (2 * n - 1)
    internal = deque()
    li = 0
    for _ in range(n - 1):
        picked = []
        for _ in range(2):
            if li < n and (not internal or w[li] <= w[internal[0]]):
                picked.append(li)
                li += 1
            else:
                picked.append(internal.popleft())
        node = len(w)
        w.append(w[picked[0]] + w[picked[1]])
        parent[picked[0]] = node
        parent[picked[1]] = node
        internal.append(node)
    root = 2 * n - 2
    depth = [0] * (2 * n - 1)
    for node in range(root - 1, -1, -1):  # parents are created after children
        depth[node] = depth[parent[node]] + 1
    return depth[:n]


def code_lengths(freq: np.ndarray) -> np.ndarray:
    """Code length of every symbol (0 for symbols that do not occur)."""
    freq = np.asarray(freq, dtype=np.int64).copy()
    lengths = np.zeros(len(freq), dtype=np.int64)
    while True:
        syms = [int(s) for s in np.nonzero(freq)[0]]
        if not syms:
            return lengths
        syms.sort(key=lambda s: (int(freq[s]), s))
        depths = _two_queue_depths([int(freq[s]) for s in syms])
        if max(depths) <= MAX_LEN:
            for s, d in zip(syms, depths):
                lengths[s] = d
            return lengths
        freq = np.where(freq > 0, (freq + 1) // 2, 0)


def canonical_codes(lengths: np.ndarray) -> np.ndarray:
    """Canonical code of every coded symbol (uint64; 0 where length is 0)."""
    codes = np.zeros(len(lengths), dtype=np.uint64)
    order = sorted((int(lengths[s]), s) for s in np.nonzero(lengths)[0])
    code, prev_len = -1, None
    for ln, s in order:
        code = 0 if prev_len is None else (code + 1) << (ln - prev_len)
        prev_len = ln
        codes[s] = code
    return codes


def encode_chunks(sym: np.ndarray, lengths: np.ndarray, codes: np.ndarray, C: int):
    """Return (offsets uint64[n_chunks+1], words uint32[n_words])."""
    N = len(sym)
    n_chunks = (N + C - 1) // C
    if N == 0:
        return np.zeros(1, dtype=np.uint64), np.zeros(0, dtype=np.uint32)
    ln = lengths[sym].astype(np.int64)
    cd = codes[sym].astype(np.uint64)
    if np.any(ln == 0):
        raise ValueError("symbol without a code")
    chunk = np.arange(N) // C
    bits_per_chunk = np.bincount(chunk, weights=ln, minlength=n_chunks).astype(np.int64)
    words_per_chunk = (bits_per_chunk + 31) // 32
    offsets = np.zeros(n_chunks + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(words_per_chunk)
    # bit position of each code: chunk start + bits of the earlier codes in the chunk
    incl = np.cumsum(ln)
    chunk_first = np.arange(n_chunks) * C
    before_chunk = np.where(chunk_first > 0, incl[np.maximum(chunk_first - 1, 0)], 0)
    start = 32 * offsets[chunk] + (incl - ln - before_chunk[chunk])
    total_bits = 32 * int(offsets[-1])
    bits = np.zeros(total_bits, dtype=np.uint8)
    for b in range(MAX_LEN):
        m = ln > b
        if not np.any(m):
            break
        shift = (ln[m] - 1 - b).astype(np.uint64)
        bits[start[m] + b] = ((cd[m] >> shift) & np.uint64(1)).astype(np.uint8)
    words = np.packbits(bits, bitorder="big").view(">u4").astype(np.uint32)
    return offsets.astype(np.uint64), words


def decode_tables(lengths: np.ndarray):
    """Canonical decoding tables: first code, count and base index per length."""
    count = np.zeros(MAX_LEN + 2, dtype=np.int64)
    for s in np.nonzero(lengths)[0]:
        count[int(lengths[s])] += 1
    first = np.zeros(MAX_LEN + 2, dtype=np.int64)
    base = np.zeros(MAX_LEN + 2, dtype=np.int64)
    code = 0
    idx = 0
    for ln in range(1, MAX_LEN + 1):
        first[ln] = code          # first canonical code of this length
        base[ln] = idx            # its index in the (length, symbol) order
        idx += count[ln]
        code = (code + count[ln]) << 1
    order = np.array(sorted((int(lengths[s]), int(s)) for s in np.nonzero(lengths)[0]),
                     dtype=np.int64).reshape(-1, 2)
    return first, count, base, order[:, 1] if len(order) else np.zeros(0, dtype=np.int64)


def decode_chunks(words: np.ndarray, offsets: np.ndarray, lengths: np.ndarray,
                  N: int, C: int, chunks=None) -> np.ndarray:
    """Decode N symbols; all chunks advance together, one symbol per step.

    With ``chunks`` (chunk indices) only those chunks are decoded; the other
    entries of the result stay 0.
    """
    out = np.zeros(N, dtype=np.int64)
    if N == 0:
        return out
    first, count, base, sorted_syms = decode_tables(lengths)
    n_chunks = (N + C - 1) // C
    w = np.concatenate([words.astype(np.uint64), np.zeros(2, dtype=np.uint64)])
    bitpos = offsets[:n_chunks].astype(np.int64) * 32
    chunk_len = np.minimum(C, N - np.arange(n_chunks) * C)
    if chunks is not None:
        keep = np.zeros(n_chunks, dtype=bool)
        keep[np.asarray(chunks, dtype=np.int64)] = True
        chunk_len = np.where(keep, chunk_len, 0)
    for s in range(C):
        act = np.nonzero(chunk_len > s)[0]
        if len(act) == 0:
            break
        p = bitpos[act]
        hi = w[p >> 5]
        lo = w[(p >> 5) + 1]
        window = (((hi << np.uint64(32)) | lo) >> (np.uint64(32) - (p & 31).astype(np.uint64))) \
            & np.uint64(0xFFFFFFFF)
        sym = np.full(len(act), -1, dtype=np.int64)
        used = np.zeros(len(act), dtype=np.int64)
        for ln in range(1, MAX_LEN + 1):
            if count[ln] == 0:
                continue
            v = (window >> np.uint64(32 - ln)).astype(np.int64)
            hit = (sym < 0) & (v - first[ln] >= 0) & (v - first[ln] < count[ln])
            sym[hit] = sorted_syms[base[ln] + v[hit] - first[ln]]
            used[hit] = ln
        if np.any(sym < 0):
            raise ValueError("invalid code in stream")
        out[act * C + s] = sym
        bitpos[act] = p + used
    return out
