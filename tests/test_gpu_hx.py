"""GPU Huffman-X codec (the Huffman pipeline of Algorithm 2 as a standalone
lossless codec, Section IV-B): streams byte-identical to the oracle's, exact
round trips, decoding of oracle streams, and rejection of corrupt streams."""
import struct

import numpy as np
import pytest

from oracle import hx
from oracle.huffman import code_lengths, histogram
from tests.gpu_common import gpu, to_bytes

pytestmark = pytest.mark.gpu


def _values(dt, n, seed, scale=8.0, wild=1e-3):
    """Laplacian values around zero with a fraction of arbitrary ones (the
    shape of quantised multilevel coefficients with outliers); Zipf-like
    bytes; Laplacian 16-bit codes around 32768."""
    rng = np.random.default_rng(seed)
    if dt == np.uint8:
        p = 1.0 / np.arange(1, 257) ** 1.2
        return rng.choice(256, size=n, p=p / p.sum()).astype(np.uint8)
    if dt == np.uint16:
        k = np.round(rng.laplace(0, scale * 40, size=n)).astype(np.int64) + 32768
        return np.clip(k, 0, 65535).astype(np.uint16)
    info = np.iinfo(dt)
    v = np.round(rng.laplace(0, scale, size=n)).astype(dt)
    m = rng.random(n) < wild
    v[m] = rng.integers(info.min, info.max, size=int(m.sum()), dtype=dt, endpoint=True)
    return v


def _torch_of(torch, a):
    t = torch.from_numpy(np.ascontiguousarray(a))
    return t.cuda()


CASES = [  # (dtype, n, dict, base, C)
    (np.uint8, 1, None, None, 1024), (np.uint8, 1000, None, None, 64),
    (np.uint8, 1024, None, None, 1024), (np.uint8, 70001, None, None, 1024),
    (np.uint8, 3_000_017, None, None, 4096),
    (np.uint16, 1, None, None, 1024), (np.uint16, 65537, None, None, 1024),
    (np.uint16, 2_000_003, None, None, 1024),
    (np.int32, 1, None, None, 1024), (np.int32, 1023, None, None, 1024),
    (np.int32, 100_003, 4096, -2047, 1024), (np.int32, 100_003, 2, 0, 64),
    (np.int32, 5_000_011, None, None, 1024), (np.int32, 777_777, 64, -31, 2048),
    (np.int64, 1, None, None, 1024), (np.int64, 100_003, 1024, -511, 1024),
    (np.int64, 3_000_001, None, None, 1024),
]


@pytest.mark.parametrize("dt,n,D,b,C", CASES)
def test_stream_is_byte_identical_to_oracle(dt, n, D, b, C):
    torch, mgc = gpu()
    v = _values(dt, n, n + C)
    x = _torch_of(torch, v)
    got = mgc.hx_compress(x, D, b, C)
    ref = hx.compress(v, D, b, C)
    gb = to_bytes(got)
    assert len(gb) == len(ref)
    assert gb == ref
    back = mgc.hx_decompress(got)
    assert back.dtype == x.dtype and bool((back == x).all())


@pytest.mark.parametrize("dt", [np.uint8, np.uint16, np.int32, np.int64])
def test_decodes_oracle_streams(dt):
    torch, mgc = gpu()
    v = _values(dt, 300_007, 3)
    ref = hx.compress(v)
    s = torch.from_numpy(np.frombuffer(ref, dtype=np.uint8).copy()).cuda()
    back = mgc.hx_decompress(s).cpu().numpy()
    assert np.array_equal(back, v)


def test_empty_and_edge_streams():
    torch, mgc = gpu()
    for dt in (np.uint8, np.uint16, np.int32, np.int64):
        v = np.zeros(0, dtype=dt)
        got = mgc.hx_compress(_torch_of(torch, np.zeros(1, dtype=dt))[:0])
        assert to_bytes(got) == hx.compress(v)
        assert mgc.hx_decompress(got).numel() == 0
    # every value escaped, no value escaped, one value repeated, type extremes
    for v, D, b in [(np.arange(100000, 160000, dtype=np.int32), 16, 0),
                    (np.arange(100000, 160000, dtype=np.int32), 65536, 100000),
                    (np.full(50000, -7, dtype=np.int64), 4, -7),
                    (np.array([np.iinfo(np.int64).min, np.iinfo(np.int64).max, 0] * 3000,
                              dtype=np.int64), 8, np.iinfo(np.int64).max - 3),
                    (np.array([np.iinfo(np.int32).min, np.iinfo(np.int32).max] * 3000,
                              dtype=np.int32), 65536, np.iinfo(np.int32).min)]:
        got = mgc.hx_compress(_torch_of(torch, v), D, b)
        assert to_bytes(got) == hx.compress(v, D, b)
        assert np.array_equal(mgc.hx_decompress(got).cpu().numpy(), v)


def test_corrupt_streams_are_rejected():
    torch, mgc = gpu()
    v = _values(np.int32, 20000, 9, wild=0.01)
    ref = bytearray(hx.compress(v, 256, -127))
    n_esc = struct.unpack_from("<Q", ref, 32)[0]
    assert n_esc > 0

    def dec(buf):
        return mgc.hx_decompress(torch.from_numpy(np.frombuffer(bytes(buf), dtype=np.uint8).copy()).cuda())

    bad = bytearray(ref)
    struct.pack_into("<Q", bad, 32, n_esc - 1)   # escape count and lengths disagree
    with pytest.raises(mgc.MgcError) as e:
        dec(bad)
    assert e.value.name == "EFORMAT"
    bad = bytearray(ref)
    struct.pack_into("<I", bad, 0, 0)            # magic
    with pytest.raises(mgc.MgcError):
        dec(bad)
    with pytest.raises(mgc.MgcError) as e:
        dec(ref[: len(ref) - 8])                 # truncated
    assert e.value.name == "EFORMAT"
    # one escape key fewer in the coded keys than escaped values stored:
    # rebuild the coded section from keys with one escape turned into key 0
    k, esc = hx.keys(v, 2, 256, -127)
    k2 = k.copy()
    k2[np.nonzero(k2 == 255)[0][0]] = 0
    sec = hx.huffman_section(k2, 1024)
    forged = bytearray(ref[:64]) + sec + esc.astype("<i4").tobytes()
    forged += b"\0" * (-len(forged) % 8)
    struct.pack_into("<QQ", forged, 40, len(sec), len(forged))
    with pytest.raises(mgc.MgcError) as e:
        dec(forged)
    assert e.value.name == "EFORMAT"


def test_full_size_streams_round_trip_with_oracle_codebook():
    # 2^27 bytes and 2^25 int32 values: every value back exactly, the
    # codebook equal to the oracle's code lengths of the full histogram, and
    # the chunk offsets equal to the bits those lengths give each chunk
    torch, mgc = gpu()
    for dt, n in ((np.uint8, 1 << 27), (np.int32, 1 << 25)):
        v = _values(dt, n, 17)
        x = _torch_of(torch, v)
        s = mgc.hx_compress(x)
        back = mgc.hx_decompress(s)
        assert bool((back == x).all())
        buf = to_bytes(s)
        hd = hx.parse_header(buf)
        k, esc = hx.keys(v, hx.type_code(v.dtype), hd["D"], hd["base"])
        assert hd["n_escaped"] == len(esc)
        ln = code_lengths(histogram(k, 65536))
        sec = buf[64:64 + hd["section"]]
        nc, n_chunks = struct.unpack_from("<QQ", sec, 16)
        coded = np.nonzero(ln)[0]
        assert np.array_equal(np.frombuffer(sec, "<u2", nc, 48), coded)
        assert np.array_equal(np.frombuffer(sec, "u1", nc, 48 + 2 * nc), ln[coded])
        off = np.frombuffer(sec, "<u8", n_chunks + 1, (48 + 3 * nc + 7) // 8 * 8)
        bits = np.add.reduceat(ln[k], np.arange(0, n, 1024))
        assert np.array_equal(np.diff(off.astype(np.int64)), (bits + 31) // 32)
        if len(esc):
            tail = np.frombuffer(buf, v.dtype, len(esc), 64 + hd["section"])
            assert np.array_equal(tail, esc)
