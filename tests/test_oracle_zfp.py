"""Pins of the fixed-rate block coder's oracle (Algorithm "ZFP Fix-Rate
Compression", Section IV-C): hand-worked negabinary, lifting and bit-plane
fixtures, exact invertibility, the transform's energy compaction, the stream
size and the fixed-point bound when every plane fits."""
import json
import os

import numpy as np
import pytest

import synthetic
from oracle import zfp

G = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "zfp_coder.json")))


def test_negabinary_digits_by_hand():
    v = np.array(G["negabinary"]["values"])
    for P in (32, 64):
        assert list(zfp.to_negabinary(v, P)) == G["negabinary"]["codes"]
        assert np.array_equal(zfp.from_negabinary(zfp.to_negabinary(v, P), P), v)


def test_lifting_of_one_line_by_hand():
    line = np.array([G["lifting"]["line"]])
    c = zfp.forward(line, 1)
    assert list(c[0]) == G["lifting"]["coefficients"]
    assert np.array_equal(zfp.inverse(c, 1), line)


def test_bit_plane_coder_by_hand():
    g = G["planes"]
    assert zfp.encode_planes(g["coefficients"], g["P"], 100) == g["full_bits"]
    assert zfp.encode_planes(g["coefficients"], g["P"], 5) == g["budget5_bits"]
    for bits, budget, want in ((g["full_bits"], 100, g["coefficients"]),
                               (g["budget5_bits"], 5, g["budget5_decoded"])):
        it = iter(bits + [0] * 100)
        assert zfp.decode_planes(lambda: next(it), 4, g["P"], budget) == want


@pytest.mark.parametrize("d", [1, 2, 3])
def test_transform_is_exactly_invertible_and_bounded(d):
    rng = np.random.default_rng(d)
    for P in (32, 64):
        q = P - 2 - d
        x = rng.integers(-(2 ** q) + 1, 2 ** q, size=(200, 4 ** d), dtype=np.int64)
        c = zfp.forward(x, d)
        assert np.array_equal(zfp.inverse(c, d), x)
        assert np.max(np.abs(c)) < 2 ** (P - 2)


def test_transform_compacts_smooth_blocks():
    # a constant block has only the zero-frequency coefficient; a block that
    # varies along the last axis only has no coefficient with a nonzero
    # frequency along the other axes
    d = 3
    c = zfp.forward(np.full((1, 64), 12345, dtype=np.int64), d)[0]
    assert c[0] == 12345 and np.all(c[1:] == 0)
    ramp = np.tile(np.array([10, 20, 35, 90], dtype=np.int64), 16)[None, :]
    c = zfp.forward(ramp, d)[0].reshape(4, 4, 4)
    assert np.all(c[1:, :, :] == 0) and np.all(c[:, 1:, :] == 0)
    assert zfp.order(3)[:4].tolist() == [0, 1, 4, 16]


def test_partial_blocks_replicate_the_last_value():
    u = np.arange(6, dtype=np.float32).reshape(6)
    b = zfp.blocks_of(u)
    assert b.tolist() == [[0, 1, 2, 3], [4, 5, 5, 5]]
    u2 = np.arange(15, dtype=np.float64).reshape(3, 5)
    assert np.array_equal(zfp.unblock(zfp.blocks_of(u2), u2.shape), u2)


@pytest.mark.parametrize("dt", [np.float32, np.float64])
@pytest.mark.parametrize("shape", [(37,), (9, 13), (9, 9, 6)])
def test_all_planes_give_the_fixed_point_bound(dt, shape):
    # with a budget that holds every plane the integers round-trip exactly,
    # so the error is the alignment's truncation: below one quantum 2^(e - q)
    rng = np.random.default_rng(len(shape))
    u = (rng.standard_normal(shape) * np.exp(3 * rng.standard_normal(shape))).astype(dt)
    d = len(shape)
    P, q, _, _ = zfp.params(dt, d)
    v = zfp.decompress(zfp.compress(u, P + 8 if d == 1 else P))
    e = zfp.block_exponent(zfp.blocks_of(u))
    quantum = zfp.unblock(np.repeat(np.ldexp(1.0, e - q)[:, None], 4 ** d, axis=1), shape)
    assert np.all(np.abs(v.astype(np.float64) - u.astype(np.float64)) < quantum)


def test_error_falls_with_rate_and_stream_size_is_fixed():
    u = synthetic.grf((17, 9, 6), 3)
    prev = np.inf
    for rate in (2, 4, 8, 12, 16, 24):
        b = zfp.compress(u, rate)
        h = zfp.parse_header(b)
        nblk = 5 * 3 * 2
        assert h["blocks"] == nblk and h["maxbits"] == 64 * rate
        assert len(b) == 64 + 8 * ((nblk * 64 * rate + 63) // 64) == h["total"]
        err = float(np.max(np.abs(zfp.decompress(b).astype(np.float64) - u)))
        assert err < prev
        prev = err
    z = np.zeros((8, 8), dtype=np.float32)
    assert np.array_equal(zfp.decompress(zfp.compress(z, 4)), z)


def test_parameters_are_checked():
    with pytest.raises(ValueError):
        zfp.compress(np.ones(8, np.float32), 65)
    with pytest.raises(ValueError):
        zfp.compress(np.ones(8, np.float32), 2)      # 8 bits: no room past the exponent
    with pytest.raises(ValueError):
        zfp.compress(np.array([1.0, np.nan], np.float32), 8)
    with pytest.raises(TypeError):
        zfp.compress(np.ones(8, np.int32), 8)
