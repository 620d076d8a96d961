"""Oracle stream layout, edge cases and failure handling (CPU)."""
import numpy as np
import pytest

import oracle
import synthetic
from oracle.stream import HEADER_BYTES, section_offsets


def test_cfg1_roundtrip_and_header():
    u = synthetic.bumps((65, 65, 65), 1)
    b = oracle.compress(u, 1e-3)
    hd = oracle.parse_header(b)
    assert hd["total"] == len(b) and len(b) % 8 == 0
    assert hd["L"] == 6 and hd["N"] == 65 ** 3 and hd["shape"] == (65, 65, 65)
    assert hd["n_chunks"] == (65 ** 3 + 1023) // 1024
    cb, off, opos, oval, w, end = section_offsets(hd["L"], hd["n_codes"], hd["n_chunks"],
                                                 hd["n_outliers"], hd["n_words"])
    assert end == len(b) and all(x % 8 == 0 for x in (off, opos, oval, w))
    offs = np.frombuffer(b, "<u8", hd["n_chunks"] + 1, off)
    assert offs[0] == 0 and offs[-1] == hd["n_words"] and np.all(np.diff(offs.astype(np.int64)) >= 0)
    pos = np.frombuffer(b, "<u8", hd["n_outliers"], opos)
    assert np.all(np.diff(pos.astype(np.int64)) > 0)
    v = oracle.decompress(b)
    x = u.astype(np.float64)
    assert np.max(np.abs(v - x)) <= 1e-3 * (x.max() - x.min())
    assert u.nbytes / len(b) > 2.0


@pytest.mark.parametrize("shape", [(1,), (1, 1, 1), (7,), (2, 2, 2), (1, 5, 1), (3, 1, 9)])
def test_small_and_squeezed_shapes(shape):
    rng = np.random.default_rng(4)
    u = rng.standard_normal(shape)
    if u.size == 1:
        u[...] = 3.25
    b = oracle.compress(u, 1e-3)
    v = oracle.decompress(b)
    assert v.shape == u.shape
    rngu = u.max() - u.min()
    assert np.max(np.abs(v - u)) <= 1e-3 * rngu + (0 if rngu else 0)


def test_constant_and_empty():
    u = np.full((10, 3), -2.5, dtype=np.float32)
    b = oracle.compress(u, 1e-3)
    assert len(b) == HEADER_BYTES + 8
    assert np.array_equal(oracle.decompress(b), u)
    e = np.zeros((0, 4), dtype=np.float64)
    b = oracle.compress(e, 1e-3)
    assert oracle.decompress(b).shape == (0, 4)


def test_rejects_bad_input():
    u = np.ones((4, 4), dtype=np.float32)
    u[1, 1] = np.nan
    with pytest.raises(ValueError):
        oracle.compress(u, 1e-3)
    with pytest.raises(ValueError):
        oracle.compress(np.ones((4, 4), dtype=np.float32), 0.0)
    with pytest.raises(ValueError):
        oracle.compress(np.ones((2, 2, 2, 2), dtype=np.float32), 1e-3)
    with pytest.raises(TypeError):
        oracle.compress(np.ones((4, 4), dtype=np.int32), 1e-3)
    with pytest.raises(ValueError):
        # relative bound far below float32 resolution
        oracle.compress(np.linspace(1000, 1000.001, 64).astype(np.float32), 1e-9)


def test_rejects_corrupt_streams():
    u = synthetic.grf((17, 17), 2)
    b = bytearray(oracle.compress(u, 1e-2))
    with pytest.raises(ValueError):
        oracle.decompress(bytes(b[:len(b) - 8]))
    with pytest.raises(ValueError):
        oracle.decompress(bytes(b[:40]))
    bad = bytearray(b)
    bad[0] ^= 0xFF
    with pytest.raises(ValueError):
        oracle.decompress(bytes(bad))
