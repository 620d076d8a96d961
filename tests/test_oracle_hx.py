"""Pins of the Huffman-X oracle (the Huffman pipeline of Algorithm 2 used as a
standalone lossless codec, Section IV-B): hand-derived streams, the key and
escape rule, optimality of the code lengths, and exact round trips."""
import json
import os
import struct

import numpy as np
import pytest

from oracle import hx
from oracle.huffman import canonical_codes, code_lengths, histogram

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "hx_streams.json")))


def test_byte_stream_matches_hand_derived_layout():
    g = GOLDEN["bytes_aab"]
    buf = hx.compress(np.array(g["input_u8"], dtype=np.uint8))
    h = g["header"]
    assert len(buf) == h["total"]
    assert struct.unpack_from("<IB3xIIqQQQQQ", buf, 0) == (
        0x5848474D, h["type"], h["D"], h["C"], h["base"], h["n"], h["n_escaped"], h["section"],
        h["total"], 0)
    sec = buf[64:64 + h["section"]]
    assert struct.unpack_from("<II5Q", sec, 0) == (0x3148474D, 1024, 3, 2, 1, 1, 80)
    assert list(np.frombuffer(sec, "<u2", 2, 48)) == g["codebook_keys"]
    assert list(np.frombuffer(sec, "u1", 2, 52)) == g["codebook_lengths"]
    assert sec[54:56] == b"\0\0"
    assert list(np.frombuffer(sec, "<u8", 2, 56)) == g["offsets"]
    assert list(np.frombuffer(sec, "<u4", 1, 72)) == g["words"]
    assert sec[76:80] == b"\0" * 4
    assert bytes(hx.decompress(buf)) == bytes(g["input_u8"])


def test_int32_keys_escapes_and_words_match_hand_derivation():
    g = GOLDEN["int32_escapes"]
    v = np.array(g["input_i32"], dtype=np.int32)
    k, esc = hx.keys(v, 2, g["D"], g["base"])
    assert list(k) == g["keys"]
    assert list(esc) == g["escaped"]
    buf = hx.compress(v, D=g["D"], b=g["base"])
    hd = hx.parse_header(buf)
    assert hd["n_escaped"] == 5 and hd["D"] == 8 and hd["base"] == -4
    sec = buf[64:64 + hd["section"]]
    nc = struct.unpack_from("<Q", sec, 16)[0]
    keys = list(np.frombuffer(sec, "<u2", nc, 48))
    lens = list(np.frombuffer(sec, "u1", nc, 48 + 2 * nc))
    assert dict(zip(map(str, keys), lens)) == g["lengths"]
    n_chunks = struct.unpack_from("<Q", sec, 24)[0]
    w_off = (48 + 3 * nc + 7) // 8 * 8 + 8 * (n_chunks + 1)
    assert list(np.frombuffer(sec, "<u4", 1, w_off)) == g["words"]
    tail = np.frombuffer(buf, "<i4", 5, 64 + hd["section"])
    assert list(tail) == g["escaped"]
    assert np.array_equal(hx.decompress(buf), v)


def test_key_rule_at_the_dictionary_edges():
    # i64: values b .. b + D - 2 have keys; b - 1 and b + D - 1 escape
    b, D = -10, 16
    v = np.array([b - 1, b, b + D - 2, b + D - 1, 0], dtype=np.int64)
    k, esc = hx.keys(v, 3, D, b)
    assert list(k) == [D - 1, 0, D - 2, D - 1, 10]
    assert list(esc) == [b - 1, b + D - 1]
    # a base at the top of the range: the key window ends at the type's max
    top = np.iinfo(np.int64).max
    v = np.array([top, top - 1, np.iinfo(np.int64).min], dtype=np.int64)
    k, esc = hx.keys(v, 3, 4, top - 1)
    assert list(k) == [1, 0, 3]
    assert list(esc) == [np.iinfo(np.int64).min]
    # dictionary of two: one value has a key, everything else escapes
    v = np.array([5, 6, 5, 4], dtype=np.int32)
    k, esc = hx.keys(v, 2, 2, 5)
    assert list(k) == [0, 1, 0, 1] and list(esc) == [6, 4]


@pytest.mark.parametrize("dt", [np.uint8, np.uint16, np.int32, np.int64])
def test_round_trip_is_exact(dt):
    rng = np.random.default_rng(7)
    info = np.iinfo(dt)
    for n in (0, 1, 63, 64, 1000, 70001):
        x = rng.integers(info.min, info.max, size=n, dtype=dt, endpoint=True)
        if np.issubdtype(dt, np.signedinteger) and n > 4:
            x[: n // 2] = np.round(rng.laplace(0, 30, size=n // 2)).astype(dt)
            x[:2] = [info.min, info.max]
        for C in (64, 1024):
            y = hx.decompress(hx.compress(x, C=C))
            assert y.dtype == np.dtype(dt) and np.array_equal(x, y)


def test_all_values_escaped_and_none_escaped():
    x = np.arange(100000, 100500, dtype=np.int32)
    buf = hx.compress(x, D=16, b=0)
    assert hx.parse_header(buf)["n_escaped"] == 500
    assert np.array_equal(hx.decompress(buf), x)
    buf = hx.compress(x, D=1024, b=100000)
    assert hx.parse_header(buf)["n_escaped"] == 0
    assert np.array_equal(hx.decompress(buf), x)


def test_code_lengths_are_optimal_within_one_bit_of_entropy():
    # Huffman codes satisfy H <= mean length < H + 1, with equality in the
    # Kraft sum; a dropped merge or a wrong depth breaks one of them
    rng = np.random.default_rng(11)
    for scale in (0.7, 4.0, 60.0):
        k = np.abs(np.round(rng.laplace(0, scale, size=200000))).astype(np.int64)
        f = histogram(k, 65536)
        ln = code_lengths(f)
        p = f[f > 0] / f.sum()
        H = float(-(p * np.log2(p)).sum())
        mean = float((f * ln).sum() / f.sum())
        assert H - 1e-12 <= mean < H + 1
        if (f > 0).sum() > 1:
            assert abs(float((2.0 ** -ln[f > 0]).sum()) - 1.0) < 1e-12
        codes = canonical_codes(ln)
        used = [(int(ln[s]), int(codes[s])) for s in np.nonzero(f)[0]]
        # prefix-free: no code is a prefix of another
        used.sort()
        for (la, ca), (lb, cb) in zip(used, used[1:]):
            assert (cb >> (lb - la)) != ca


def test_byte_stream_size_tracks_entropy():
    rng = np.random.default_rng(5)
    p = 1.0 / np.arange(1, 257) ** 1.1
    p /= p.sum()
    x = rng.choice(256, size=300000, p=p).astype(np.uint8)
    buf = hx.compress(x)
    f = np.bincount(x, minlength=256)
    q = f[f > 0] / f.sum()
    H = float(-(q * np.log2(q)).sum())
    coded_bits = 8 * (len(buf) - 64 - 48 - 3 * 256 - 8 * 300)
    assert H * len(x) <= coded_bits < (H + 1) * len(x)


def test_parameters_are_checked():
    with pytest.raises(ValueError):
        hx.compress(np.zeros(4, np.uint8), D=128)
    with pytest.raises(ValueError):
        hx.compress(np.zeros(4, np.int32), D=1)
    with pytest.raises(ValueError):
        hx.compress(np.zeros(4, np.int32), D=65537)
    with pytest.raises(ValueError):
        hx.compress(np.zeros(4, np.int32), b=2 ** 31)
    with pytest.raises(TypeError):
        hx.compress(np.zeros(4, np.float32))
    buf = bytearray(hx.compress(np.arange(10, dtype=np.int32), D=4, b=0))
    struct.pack_into("<Q", buf, 32, 5)   # escaped count no longer matches the keys
    with pytest.raises(ValueError):
        hx.decompress(bytes(buf))
