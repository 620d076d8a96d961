"""GPU fixed-rate block transform coding (Algorithm "ZFP Fix-Rate
Compression", Section IV-C): streams bit-identical to the oracle's for every
dtype, dimension, ragged shape and rate (word-aligned and unaligned block
sizes), decompressed values identical to the oracle's, and the full-size
field's size and accuracy."""
import numpy as np
import pytest

import synthetic
from oracle import zfp as ozfp
from tests.gpu_common import gpu, to_bytes

pytestmark = pytest.mark.gpu

CASES = [  # (shape, dtype, rate)
    ((37,), np.float32, 8), ((37,), np.float64, 16.25), ((1,), np.float32, 5),
    ((1000,), np.float32, 3.5), ((9, 13), np.float32, 4), ((9, 13), np.float64, 7),
    ((64, 64), np.float32, 12), ((17, 9, 6), np.float32, 8), ((17, 9, 6), np.float64, 16),
    ((33, 33, 33), np.float32, 1.5), ((33, 33, 33), np.float32, 32),
    ((20, 21, 22), np.float64, 64), ((5, 4, 3), np.float32, 40),
]


def _field(shape, dt, seed):
    rng = np.random.default_rng(seed)
    if len(shape) == 3 and min(shape) > 4:
        u = synthetic.grf(shape, seed, dtype=dt)
    else:
        u = (rng.standard_normal(shape) * np.exp(2 * rng.standard_normal(shape))).astype(dt)
    flat = u.reshape(-1)
    flat[: max(1, flat.size // 50)] = 0      # some zero values (and zero blocks in 1D)
    return u


@pytest.mark.parametrize("shape,dt,rate", CASES)
def test_stream_and_values_match_oracle(shape, dt, rate):
    torch, mgc = gpu()
    u = _field(shape, dt, len(shape) + int(rate * 4))
    x = torch.from_numpy(u).cuda()
    got = mgc.zfp_compress(x, rate)
    ref = ozfp.compress(u, rate)
    assert to_bytes(got) == ref
    v = mgc.zfp_decompress(got).cpu().numpy()
    assert v.dtype == u.dtype and v.shape == u.shape
    assert np.array_equal(v, ozfp.decompress(ref))
    # the oracle's stream decodes on the GPU to the same values
    s = torch.from_numpy(np.frombuffer(ref, dtype=np.uint8).copy()).cuda()
    assert np.array_equal(mgc.zfp_decompress(s).cpu().numpy(), v)


def test_zero_array_and_nonfinite_input():
    torch, mgc = gpu()
    z = torch.zeros((9, 9, 9), dtype=torch.float32, device="cuda")
    got = mgc.zfp_compress(z, 4)
    assert to_bytes(got) == ozfp.compress(np.zeros((9, 9, 9), np.float32), 4)
    assert bool((mgc.zfp_decompress(got) == 0).all())
    bad = torch.ones(100, dtype=torch.float64, device="cuda")
    bad[57] = float("inf")
    with pytest.raises(mgc.MgcError) as e:
        mgc.zfp_compress(bad, 16)
    assert e.value.name == "EINVAL"
    with pytest.raises(mgc.MgcError):
        mgc.zfp_compress(z, 0.02)        # fewer bits than the block header


def test_full_size_field_size_and_accuracy():
    # 513^3 FP32 at 8 bits per value: the exact stream size, a sample of
    # blocks bit-identical to the oracle's coding of the same blocks, and
    # every value within the accuracy the oracle reaches on them
    torch, mgc = gpu()
    u = synthetic.grf((513, 513, 513), 2)
    x = torch.from_numpy(u).cuda()
    got = mgc.zfp_compress(x, 8)
    nb = 129 ** 3
    assert got.numel() == 64 + 8 * nb * 8 == mgc.zfp_query((513, 513, 513), torch.float32, 8)
    g = to_bytes(got)
    words = np.frombuffer(g, dtype="<u8", offset=64)
    # a 16^3 corner sub-array is whole blocks of the full array: its stream's
    # blocks are the full stream's blocks at the same block coordinates
    sub = np.ascontiguousarray(u[:16, :16, :16])
    ref = np.frombuffer(ozfp.compress(sub, 8), dtype="<u8", offset=64).reshape(4, 4, 4, 8)
    full = words.reshape(129, 129, 129, 8)
    assert np.array_equal(full[:4, :4, :4], ref)
    v = mgc.zfp_decompress(got).cpu().numpy()
    sv = ozfp.decompress(ozfp.compress(sub, 8))
    assert np.array_equal(v[:16, :16, :16], sv)
    err = np.abs(v.astype(np.float64) - u)
    assert float(err.max()) < 0.05 * float(np.abs(u).max())
