"""GPU Huffman stage: bit-exact against the oracle on identical symbols."""
import struct

import numpy as np
import pytest

from oracle import huffman
from tests.gpu_common import gpu, oracle_huffman_stream, to_bytes

pytestmark = pytest.mark.gpu


def _laplace_symbols(n, scale, seed):
    rng = np.random.default_rng(seed)
    k = np.round(rng.laplace(0, scale, size=n)).astype(np.int64)
    return np.clip(k + 32768, 0, 65535).astype(np.int64)


CASES = [  # (n, scale, C)
    (1, 3.0, 1024), (1000, 3.0, 1024), (1024, 3.0, 1024), (5000, 0.2, 1024),
    (100003, 40.0, 1024), (300000, 3000.0, 1024), (70000, 5.0, 64), (4097, 2.0, 128),
    (2_000_000, 9000.0, 1024),
    (12_600_007, 3000.0, 1024),  # enough chunks for the persistent encoder
]


@pytest.mark.parametrize("n,scale,C", CASES)
def test_encode_bit_exact(n, scale, C):
    torch, mgc = gpu()
    sym = _laplace_symbols(n, scale, n)
    t = torch.from_numpy(sym.astype(np.uint16).view(np.int16)).cuda()
    got = to_bytes(mgc.huffman_encode(t, C))
    ref = oracle_huffman_stream(sym, C)
    assert len(got) == len(ref)
    assert got == ref
    back = mgc.huffman_decode(mgc.huffman_encode(t, C), n).cpu().numpy().view(np.uint16)
    assert np.array_equal(back.astype(np.int64), sym)


def test_single_symbol_and_all_symbols():
    torch, mgc = gpu()
    for sym in (np.full(5000, 7, dtype=np.int64), np.arange(65536, dtype=np.int64),
                np.repeat(np.arange(65536, dtype=np.int64), 3)):
        t = torch.from_numpy(sym.astype(np.uint16).view(np.int16)).cuda()
        got = to_bytes(mgc.huffman_encode(t, 1024))
        assert got == oracle_huffman_stream(sym, 1024)
        back = mgc.huffman_decode(mgc.huffman_encode(t, 1024), len(sym)).cpu().numpy().view(np.uint16)
        assert np.array_equal(back.astype(np.int64), sym)


def test_length_limit_flattening_matches_oracle():
    torch, mgc = gpu()
    fib = [1, 1]
    while len(fib) < 40:
        fib.append(fib[-1] + fib[-2])
    sym = np.repeat(np.arange(40, dtype=np.int64) * 7 + 100, fib)
    rng = np.random.default_rng(3)
    rng.shuffle(sym)
    ln = huffman.code_lengths(huffman.histogram(sym, 65536))
    assert ln.max() <= 32
    t = torch.from_numpy(sym.astype(np.uint16).view(np.int16)).cuda()
    enc = mgc.huffman_encode(t, 1024)
    assert to_bytes(enc) == oracle_huffman_stream(sym, 1024)
    # codes up to the 32-bit limit, prefixes holding several lengths
    back = mgc.huffman_decode(enc, len(sym))
    assert bool((back == t).all())


def test_gpu_decodes_oracle_stream_and_rejects_corruption():
    torch, mgc = gpu()
    sym = _laplace_symbols(50000, 30.0, 5)
    ref = oracle_huffman_stream(sym, 1024)
    dev = torch.from_numpy(np.frombuffer(ref, dtype=np.uint8).copy()).cuda()
    back = mgc.huffman_decode(dev, len(sym)).cpu().numpy().view(np.uint16)
    assert np.array_equal(back.astype(np.int64), sym)
    bad = bytearray(ref)
    n_codes = struct.unpack_from("<Q", ref, 16)[0]
    bad[48 + 2 * n_codes] = 0    # the first code length becomes 0
    with pytest.raises(mgc.MgcError) as e:
        mgc.huffman_decode(torch.from_numpy(np.frombuffer(bytes(bad), dtype=np.uint8).copy()).cuda(),
                           len(sym))
    assert e.value.name == "EFORMAT"
    # lengths beyond the 32-bit limit (one far beyond the per-length count
    # tables) are rejected too, and a good stream decodes again afterwards
    for bad_len in (33, 200, 255):
        bad = bytearray(ref)
        bad[48 + 2 * n_codes + 3] = bad_len
        with pytest.raises(mgc.MgcError) as e:
            mgc.huffman_decode(torch.from_numpy(np.frombuffer(bytes(bad), dtype=np.uint8).copy()).cuda(),
                               len(sym))
        assert e.value.name == "EFORMAT"
    back = mgc.huffman_decode(dev, len(sym)).cpu().numpy().view(np.uint16)
    assert np.array_equal(back.astype(np.int64), sym)
    with pytest.raises(mgc.MgcError) as e:
        mgc.huffman_decode(dev[: len(ref) - 64], len(sym))
    assert e.value.name == "EFORMAT"


def test_four_digit_frequencies_and_tile_edges():
    """Leaf sort over all four 8-bit digits (a count above 2^24) and symbols
    on the edges of the 2048-bin sort tiles; codebook and stream must equal
    the oracle's."""
    torch, mgc = gpu()
    rng = np.random.default_rng(11)
    edges = np.array([0, 1, 2047, 2048, 2049, 4095, 4096, 30719, 30720, 63487, 63488, 65534, 65535])
    parts = [np.full((1 << 24) + 5, 32768, dtype=np.int64)]
    for j, e in enumerate(edges):
        parts.append(np.full(1 + 37 * j, e, dtype=np.int64))
    parts.append(rng.integers(32000, 33500, size=40000))
    sym = np.concatenate(parts)
    rng.shuffle(sym)
    print("case: four-digit frequencies, n =", len(sym), flush=True)
    t = torch.from_numpy(sym.astype(np.uint16).view(np.int16)).cuda()
    enc = mgc.huffman_encode(t, 1024)
    assert to_bytes(enc) == oracle_huffman_stream(sym, 1024)
    back = mgc.huffman_decode(enc, len(sym))
    assert bool((back == t).all())


def test_decode_rejects_codebook_out_of_order():
    """The codebook section lists symbols strictly ascending; a swapped pair
    must be refused with EFORMAT."""
    torch, mgc = gpu()
    sym = _laplace_symbols(30000, 20.0, 8)
    ref = oracle_huffman_stream(sym, 1024)
    n_codes = struct.unpack_from("<Q", ref, 16)[0]
    assert n_codes > 10
    bad = bytearray(ref)
    a, b = 48 + 2 * 5, 48 + 2 * 6  # symbols 5 and 6 of the section
    bad[a:a + 2], bad[b:b + 2] = ref[b:b + 2], ref[a:a + 2]
    with pytest.raises(mgc.MgcError) as e:
        mgc.huffman_decode(torch.from_numpy(np.frombuffer(bytes(bad), dtype=np.uint8).copy()).cuda(),
                           len(sym))
    assert e.value.name == "EFORMAT"


@pytest.mark.parametrize("C", [1024, 100])
def test_decode_stream_at_any_word_offset(C):
    """The decoder reads the coded words in aligned 16- and 64-byte pieces:
    a stream starting 4..60 bytes past an aligned address decodes the same
    (C = 100 also takes the element-wise symbol stores); a stream that does
    not start on a 4-byte boundary is refused."""
    torch, mgc = gpu()
    sym = _laplace_symbols(100_003, 700.0, 12)
    t = torch.from_numpy(sym.astype(np.uint16).view(np.int16)).cuda()
    # (the encoder takes chunk sizes in multiples of 64; the oracle any)
    ref = oracle_huffman_stream(sym, C)
    enc = torch.from_numpy(np.frombuffer(ref, dtype=np.uint8).copy()).cuda()
    n = enc.numel()
    for off in (0, 4, 8, 12, 20, 36, 60):
        print("case: C", C, "offset", off, flush=True)
        buf = torch.zeros(n + 128, dtype=torch.uint8, device="cuda")
        buf[off:off + n] = enc
        back = mgc.huffman_decode(buf[off:off + n], len(sym))
        assert bool((back == t).all()), off
    buf = torch.zeros(n + 128, dtype=torch.uint8, device="cuda")
    buf[2:2 + n] = enc
    with pytest.raises(mgc.MgcError) as e:
        mgc.huffman_decode(buf[2:2 + n], len(sym))
    assert e.value.name == "EINVAL"


@pytest.fixture
def forced_decoder():
    """Forces decoder shapes inside a test and restores automatic choice."""
    torch, mgc = gpu()
    yield mgc.set_decoder
    mgc.set_decoder(0, 0)


@pytest.mark.parametrize("n,scale,C", [(300000, 3000.0, 1024), (70000, 5.0, 64),
                                       (2_000_000, 9000.0, 1024), (12_600_007, 3000.0, 1024)])
def test_every_decoder_ring_with_several_wavefronts(n, scale, C, forced_decoder):
    """The three ring shapes (64-, 32- and 16-byte pieces, refill points every
    16, 8 and 4 symbols) with 2, 4 and 16 wavefronts per block decode the
    oracle's stream to exactly the encoded symbols (Algorithm 2, decoding).
    The automatic choice of the full-size benchmark field is the 16-byte ring
    with several wavefronts; these cases cover every shape on identical
    streams."""
    torch, mgc = gpu()
    sym = _laplace_symbols(n, scale, n + 1)
    ref = oracle_huffman_stream(sym, C)
    enc = torch.from_numpy(np.frombuffer(ref, dtype=np.uint8).copy()).cuda()
    t = torch.from_numpy(sym.astype(np.uint16).view(np.int16)).cuda()
    multi = 0
    for ring in (1, 2, 3):
        decoded = []
        for waves in (1, 2, 4, 8, 16):
            print("case: n", n, "ring", ring, "waves", waves, flush=True)
            forced_decoder(ring, waves)
            try:
                back = mgc.huffman_decode(enc, n)
            except mgc.MgcError as err:
                # a wide ring with many wavefronts may not fit beside the
                # codebook's table: refused, never run out of bounds
                assert err.name == "EINVAL", (ring, waves)
                continue
            assert mgc.decoder_info() == (ring, waves)
            assert bool((back == t).all()), (ring, waves)
            decoded.append(waves)
        assert decoded, ring
        multi += sum(1 for w in decoded if w >= 2)
    assert multi >= 2


@pytest.mark.parametrize("ring", [1, 2, 3])
def test_decode_at_any_word_offset_every_ring(ring, forced_decoder):
    """Stream starts 4..60 bytes past an aligned address, for each ring shape
    with two wavefronts per block."""
    torch, mgc = gpu()
    sym = _laplace_symbols(100_003, 700.0, 12)
    t = torch.from_numpy(sym.astype(np.uint16).view(np.int16)).cuda()
    ref = oracle_huffman_stream(sym, 1024)
    enc = torch.from_numpy(np.frombuffer(ref, dtype=np.uint8).copy()).cuda()
    n = enc.numel()
    forced_decoder(ring, 2)
    for off in (0, 4, 8, 12, 20, 36, 60):
        buf = torch.zeros(n + 128, dtype=torch.uint8, device="cuda")
        buf[off:off + n] = enc
        back = mgc.huffman_decode(buf[off:off + n], len(sym))
        assert mgc.decoder_info() == (ring, 2)
        assert bool((back == t).all()), off


def test_decoder_choice_on_large_codebook_and_forced_shapes_that_do_not_fit(forced_decoder):
    """A codebook of 55,000 codes (the size class of the 513^3 benchmark
    field's) leaves room only for a narrower ring when a block holds nine
    wavefronts: the automatic choice falls back to one, a forced 64-byte ring
    with nine wavefronts is refused (EINVAL) instead of overrunning LDS, and
    every shape that fits decodes the same symbols."""
    torch, mgc = gpu()
    rng = np.random.default_rng(4)
    base = np.arange(1, 55001, dtype=np.int64)
    lap = np.clip(np.round(rng.laplace(0, 2000, 3_000_000)) + 27500, 1, 55000).astype(np.int64)
    sym = np.concatenate([base, lap])
    rng.shuffle(sym)
    n = len(sym)
    ref = oracle_huffman_stream(sym, 1024)
    assert struct.unpack_from("<Q", ref, 16)[0] == 55000
    enc = torch.from_numpy(np.frombuffer(ref, dtype=np.uint8).copy()).cuda()
    t = torch.from_numpy(sym.astype(np.uint16).view(np.int16)).cuda()
    forced_decoder(0, 9)
    back = mgc.huffman_decode(enc, n)
    ring_auto, waves_auto = mgc.decoder_info()
    assert waves_auto == 9 and ring_auto > 1
    assert bool((back == t).all())
    forced_decoder(1, 9)
    with pytest.raises(mgc.MgcError) as e:
        mgc.huffman_decode(enc, n)
    assert e.value.name == "EINVAL"
    for ring in (1, 2, 3):
        for waves in (1, 2, 4, 9):
            forced_decoder(ring, waves)
            try:
                back = mgc.huffman_decode(enc, n)
            except mgc.MgcError as err:
                assert err.name == "EINVAL"
                continue
            assert mgc.decoder_info() == (ring, waves)
            assert bool((back == t).all()), (ring, waves)
