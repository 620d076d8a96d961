"""Pins of the oracle's Huffman stage.

* Kraft equality (a full binary tree) and prefix-freeness of the codes;
* optimality: the weighted code length equals that of an independent heapq
  Huffman and, for alphabets of at most 6 symbols, the minimum over every
  length vector that satisfies Kraft's inequality (brute force);
* the tie rule and the bit layout: hand-derived fixtures in tests/golden;
* length limit: a Fibonacci alphabet is flattened to at most 32 bits;
* lossless round trip over chunk sizes, ragged last chunk and edge cases.
"""
import heapq
import itertools
import json
import os

import numpy as np
import pytest

from oracle import huffman

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "huffman_ties.json")


def _heapq_cost(freq):
    h = [int(f) for f in freq if f > 0]
    if len(h) == 1:
        return h[0]
    heapq.heapify(h)
    cost = 0
    while len(h) > 1:
        a = heapq.heappop(h)
        b = heapq.heappop(h)
        cost += a + b
        heapq.heappush(h, a + b)
    return cost


def _random_freq(rng, S, n):
    freq = np.zeros(S, dtype=np.int64)
    syms = rng.choice(S, size=n, replace=False)
    freq[syms] = rng.integers(1, 1000, size=n) ** 2
    return freq


@pytest.mark.parametrize("seed", range(6))
def test_kraft_and_optimality(seed):
    rng = np.random.default_rng(seed)
    freq = _random_freq(rng, 4096, int(rng.integers(2, 900)))
    ln = huffman.code_lengths(freq)
    used = freq > 0
    assert np.all((ln > 0) == used)
    kraft = sum(2.0 ** -int(x) for x in ln[used])
    assert kraft == 1.0
    assert int(np.sum(freq * ln)) == _heapq_cost(freq)


def test_laplacian_like_alphabet_is_optimal():
    # quantised coefficients are roughly Laplacian around the centre symbol
    rng = np.random.default_rng(1)
    k = np.round(rng.laplace(0, 40, size=200000)).astype(np.int64)
    freq = np.bincount(k + 32768, minlength=65536)
    ln = huffman.code_lengths(freq)
    assert int(np.sum(freq * ln)) == _heapq_cost(freq)


@pytest.mark.parametrize("seed", range(30))
def test_bruteforce_small_alphabets(seed):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(2, 7))
    freq = rng.integers(1, 20, size=n)
    best = None
    for lens in itertools.product(range(1, n), repeat=n):
        if sum(2.0 ** -l for l in lens) <= 1.0:
            c = sum(int(f) * l for f, l in zip(freq, lens))
            best = c if best is None else min(best, c)
    ln = huffman.code_lengths(freq)
    assert int(np.sum(freq * ln)) == best


def test_single_symbol_and_empty():
    f = np.zeros(16, dtype=np.int64)
    assert np.all(huffman.code_lengths(f) == 0)
    f[5] = 7
    ln = huffman.code_lengths(f)
    assert ln[5] == 1 and ln.sum() == 1


def test_golden_tie_rule_and_codes():
    g = json.load(open(GOLDEN))
    for case in g["cases"]:
        ln = huffman.code_lengths(np.array(case["freq"]))
        assert ln.tolist() == case["lengths"], case["derivation"]
        assert huffman.canonical_codes(ln).tolist() == case["codes"]


def test_golden_bit_layout():
    g = json.load(open(GOLDEN))["bit_layout"]
    ln = np.array(g["lengths"])
    codes = huffman.canonical_codes(ln)
    sym = np.array(g["symbols"])
    for C, key in ((4, "C4"), (2, "C2")):
        off, words = huffman.encode_chunks(sym, ln, codes, C)
        assert off.tolist() == g[key]["offsets"]
        assert words.tolist() == g[key]["words"]
        assert huffman.decode_chunks(words, off, ln, len(sym), C).tolist() == sym.tolist()


def test_canonical_codes_are_prefix_free_and_ordered():
    rng = np.random.default_rng(7)
    freq = _random_freq(rng, 512, 300)
    ln = huffman.code_lengths(freq)
    codes = huffman.canonical_codes(ln)
    coded = [(int(ln[s]), s, int(codes[s])) for s in np.nonzero(ln)[0]]
    coded.sort()
    strings = [format(c, "0%db" % l) for l, _, c in coded]
    for a, b in zip(strings, strings[1:]):
        assert a < b                              # canonical order
    for i, a in enumerate(strings):
        for b in strings[i + 1:]:
            assert not b.startswith(a)            # prefix-free


def test_length_limit_flattening():
    fib = [1, 1]
    while len(fib) < 45:
        fib.append(fib[-1] + fib[-2])
    freq = np.array(fib, dtype=np.int64)
    # without a limit the two-queue tree is a 44-deep spine
    assert max(huffman._two_queue_depths(sorted(fib))) == 44
    ln = huffman.code_lengths(freq)
    assert ln.max() <= 32
    assert sum(2.0 ** -int(x) for x in ln) == 1.0


@pytest.mark.parametrize("N,C", [(1, 1024), (1000, 1024), (1024, 1024), (5000, 1024),
                                 (4097, 32), (333, 7)])
def test_roundtrip(N, C):
    rng = np.random.default_rng(N)
    sym = (32768 + np.round(rng.laplace(0, 3, size=N))).astype(np.int64)
    freq = huffman.histogram(sym, 65536)
    ln = huffman.code_lengths(freq)
    codes = huffman.canonical_codes(ln)
    off, words = huffman.encode_chunks(sym, ln, codes, C)
    assert len(off) == (N + C - 1) // C + 1
    assert int(off[-1]) == len(words)
    out = huffman.decode_chunks(words, off, ln, N, C)
    assert np.array_equal(out, sym)


def test_roundtrip_single_symbol_stream():
    sym = np.full(3000, 40000, dtype=np.int64)
    ln = huffman.code_lengths(huffman.histogram(sym, 65536))
    off, words = huffman.encode_chunks(sym, ln, huffman.canonical_codes(ln), 1024)
    assert len(words) == 32 + 32 + 30     # 1 bit per symbol: 1024/32, 1024/32, 952/32
    assert np.array_equal(huffman.decode_chunks(words, off, ln, 3000, 1024), sym)
