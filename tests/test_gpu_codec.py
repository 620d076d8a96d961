"""GPU compress / decompress vs the FP64 oracle.

* bins: bit-identical for L-inf (min and max are exact); within 1e-14 for L2
  (the sum of squares is accumulated in a different order);
* quantised integers: equal to the oracle's except at bin-boundary ties
  (at most 1e-6 of the points, each off by one);
* when all integers agree the whole stream is byte-identical (Huffman,
  layout and header are bit-exact);
* the error bound holds for the GPU reconstruction, and each side decodes the
  other's stream;
* edge cases: constant, empty, squeezed axes, L = 0, NaN input, corrupt
  streams, outlier-capacity retry.
"""
import numpy as np
import pytest

import oracle
import synthetic
from oracle import Hierarchy
from oracle.quantize import from_symbols
from oracle.stream import decode_symbols, parse_header
from tests.gpu_common import gpu, to_bytes

pytestmark = pytest.mark.gpu


def _field(shape, dtype, seed):
    if len(shape) == 3 and seed % 2 == 0:
        return synthetic.bumps(shape, seed, dtype=dtype)
    return synthetic.grf(shape, seed, dtype=dtype)


def _bound_ok(u, v, rel, norm):
    x = u.astype(np.float64)
    e = v.astype(np.float64) - x
    if norm == "linf":
        return np.max(np.abs(e)) <= rel * (x.max() - x.min())
    return np.sqrt(np.sum(e * e)) <= rel * np.sqrt(np.sum(x * x))


def _check_parity(u, rel, norm, mode="rel"):
    torch, mgc = gpu()
    blob = mgc.compress(torch.from_numpy(u).cuda(), rel, norm, mode)
    g = to_bytes(blob)
    r = oracle.compress(u, rel, norm, mode)
    hg, hr = parse_header(g), parse_header(r)
    for key in ("L", "N", "n_chunks", "D", "shape", "S", "C", "flags"):
        assert hg[key] == hr[key], key
    if norm == "linf":
        assert np.array_equal(hg["q"], hr["q"])
        assert hg["tau"] == hr["tau"] and hg["tau_eff"] == hr["tau_eff"]
    else:
        assert np.allclose(hg["q"], hr["q"], rtol=1e-14, atol=0)
    kg = from_symbols(*decode_symbols(g))
    kr = from_symbols(*decode_symbols(r))
    diff = np.nonzero(kg != kr)[0]
    assert len(diff) <= 1e-6 * u.size + 1
    assert np.all(np.abs(kg[diff] - kr[diff]) == 1)
    if len(diff) == 0 and norm == "linf":
        assert g == r, "identical integers must give an identical stream"
    # reconstructions: GPU of its own stream, GPU of the oracle stream, oracle of GPU stream
    v = mgc.decompress(blob).cpu().numpy()
    assert v.shape == u.shape and v.dtype == u.dtype
    assert _bound_ok(u, v, rel, norm)
    rdev = torch.from_numpy(np.frombuffer(r, dtype=np.uint8).copy()).cuda()
    v2 = mgc.decompress(rdev).cpu().numpy()
    v2_ref = oracle.decompress(r)
    tol = 1e-12 * float(np.max(np.abs(u))) + (np.spacing(np.float32(np.max(np.abs(u))))
                                              if u.dtype == np.float32 else 0.0)
    assert np.max(np.abs(v2.astype(np.float64) - v2_ref)) <= tol
    assert _bound_ok(u, oracle.decompress(g), rel, norm)
    return len(g)


@pytest.mark.parametrize("shape", [(65, 65, 65), (30, 41, 12), (40, 33, 17), (9, 5, 4),
                                   (33, 20), (257,), (2, 2, 2), (1, 7, 1), (3, 5)])
@pytest.mark.parametrize("rel", [1e-2, 1e-3, 1e-4])
def test_linf_f32(shape, rel):
    u = _field(shape, np.float32, 2 if len(shape) == 3 else 3)
    _check_parity(u, rel, "linf")


@pytest.mark.parametrize("shape", [(65, 65, 65), (129, 70), (300,)])
@pytest.mark.parametrize("norm", ["linf", "l2"])
def test_f64_and_l2(shape, norm):
    u = _field(shape, np.float64, 5)
    _check_parity(u, 1e-3, norm)
    _check_parity(u.astype(np.float32), 1e-4, norm)


def test_absolute_mode():
    u = _field((33, 33, 33), np.float32, 4)
    _check_parity(u, 0.01, "linf", "abs")


def test_constant_empty_and_scalar():
    torch, mgc = gpu()
    c = np.full((20, 7), 3.5, dtype=np.float32)
    b = mgc.compress(torch.from_numpy(c).cuda(), 1e-3)
    assert to_bytes(b) == oracle.compress(c, 1e-3)
    assert np.array_equal(mgc.decompress(b).cpu().numpy(), c)
    e = np.zeros((0, 5), dtype=np.float64)
    b = mgc.compress(torch.from_numpy(e).cuda(), 1e-3)
    assert to_bytes(b) == oracle.compress(e, 1e-3)
    assert mgc.decompress(b).shape == (0, 5)
    s = np.array([1.25], dtype=np.float64)
    b = mgc.compress(torch.from_numpy(s).cuda(), 1e-3)
    assert mgc.decompress(b).cpu().numpy()[0] == 1.25


def test_rejects_nan_and_bad_bound():
    torch, mgc = gpu()
    u = np.ones((16, 16), dtype=np.float32)
    u[3, 4] = np.nan
    with pytest.raises(mgc.MgcError) as e:
        mgc.compress(torch.from_numpy(u).cuda(), 1e-3)
    assert e.value.name == "EINVAL"
    with pytest.raises(mgc.MgcError) as e:
        mgc.compress(torch.ones(8, 8, device="cuda"), -1.0)
    assert e.value.name == "EINVAL"


def test_rejects_corrupt_streams():
    torch, mgc = gpu()
    u = _field((33, 33, 33), np.float32, 3)
    blob = mgc.compress(torch.from_numpy(u).cuda(), 1e-3)
    with pytest.raises(mgc.MgcError) as e:
        mgc.decompress(blob[: blob.numel() - 16])
    assert e.value.name == "EFORMAT"
    bad = blob.clone()
    bad[0] = bad[0] ^ 0xFF
    with pytest.raises(mgc.MgcError):
        mgc.decompress(bad)


def test_decompress_stream_at_word_offsets():
    """A compressed stream copied 4, 12 or 36 bytes past an aligned address
    reconstructs the same array, bit for bit."""
    torch, mgc = gpu()
    u = _field((65, 33, 47), np.float32, 5)
    blob = mgc.compress(torch.from_numpy(u).cuda(), 1e-3)
    ref = mgc.decompress(blob)
    n = blob.numel()
    for off in (4, 12, 36):
        print("case: offset", off, flush=True)
        buf = torch.zeros(n + 64, dtype=torch.uint8, device="cuda")
        buf[off:off + n] = blob
        assert bool(torch.equal(mgc.decompress(buf[off:off + n]), ref)), off


def test_outlier_capacity_retry():
    torch, mgc = gpu()
    u = _field((65, 65, 65), np.float32, 3)
    x = torch.from_numpy(u).cuda()
    full = to_bytes(mgc.compress(x, 1e-5))
    hd = parse_header(full)
    assert hd["n_outliers"] > 10
    small = to_bytes(mgc.compress(x, 1e-5, outlier_cap=8))   # overflows, then retries
    assert small == full


def test_repeat_calls_are_deterministic():
    torch, mgc = gpu()
    u = _field((129, 129, 65), np.float32, 3)
    x = torch.from_numpy(u).cuda()
    a = to_bytes(mgc.compress(x, 1e-3))
    b = to_bytes(mgc.compress(x, 1e-3))
    assert a == b


def test_streamed_level_kernel_matches_tiled():
    """Levels of >= 2^25 points use the z-streamed decomposition kernel; the
    tiled kernel (forced candidate 1) must give the same stream and the same
    FP64 coefficients, bit for bit."""
    torch, mgc = gpu()
    gen = torch.Generator(device="cuda").manual_seed(17)
    x = torch.randn((65, 513, 1025), generator=gen, device="cuda", dtype=torch.float32)
    x += torch.linspace(-3.0, 3.0, 1025, device="cuda")
    streamed = mgc.compress(x, 1e-3)
    coeff_s = mgc.decompose(x)
    mgc.set_tuning("dec_f32", 1)
    try:
        tiled = mgc.compress(x, 1e-3)
        coeff_t = mgc.decompose(x)
    finally:
        mgc.set_tuning("dec_f32", -1)
    assert streamed.numel() == tiled.numel() and bool((streamed == tiled).all())
    assert bool((coeff_s == coeff_t).all())
    # the streamed recomposition restriction: exact inversion without
    # quantisation, and the decompressed field within the bound
    back = mgc.recompose(coeff_s, tuple(x.shape), dtype=torch.float64)
    err = torch.max(torch.abs(back - x.double())).item()
    assert err <= 1e-12 * torch.max(torch.abs(x)).item()
    y = mgc.decompress(streamed)
    tau = 1e-3 * (x.max() - x.min()).item()
    assert torch.max(torch.abs(y.double() - x.double())).item() <= tau


@pytest.mark.parametrize("rel", [1e-2, 1e-3, 1e-4])
def test_full_size_513(rel):
    """The benchmark's configuration: 513^3 FP32 |k|^-3 field."""
    torch, mgc = gpu()
    u = _grf513()
    x = torch.from_numpy(u).cuda()
    blob = mgc.compress(x, rel)
    v = mgc.decompress(blob).cpu().numpy()
    assert _bound_ok(u, v, rel, "linf")
    g = to_bytes(blob)
    hd = parse_header(g)
    h = Hierarchy(u.shape)
    assert hd["L"] == h.L == 9
    # sampled finest-level integers against the oracle, one by one
    idx = np.random.default_rng(1).choice(u.size, 2000, replace=False)
    pos, c = oracle.transform.finest_coefficients_at(u.astype(np.float64), h, idx)
    _, tau_eff = oracle.error_budget(u, rel, "linf", "rel")
    q = oracle.level_bins(h, tau_eff, "linf")
    assert np.array_equal(hd["q"], q)
    k_ref = np.rint(c * (1.0 / q[h.L])).astype(np.int64)
    chunks = np.unique(pos // hd["C"])
    sym, opos, oval = decode_symbols(g, hd, chunks=chunks)
    k = sym[pos] - 32768
    esc = sym[pos] == 0
    if np.any(esc):
        where = np.searchsorted(opos.astype(np.int64), pos[esc])
        k[esc] = oval[where]
    mism = np.count_nonzero(k != k_ref)
    assert mism <= 1e-6 * u.size
    assert np.all(np.abs(k - k_ref) <= 1)


_CACHE = {}


def _grf513():
    if "u" not in _CACHE:
        _CACHE["u"] = synthetic.grf((513, 513, 513), 2)
    return _CACHE["u"]


def _cfg3(name):
    key = "cfg3_" + name
    if key not in _CACHE:
        if name == "sin8193":
            _CACHE[key] = synthetic.sinusoids((8193, 8193), 3)
        else:
            _CACHE[key] = synthetic.grf((300, 400, 500), 4)
    return _CACHE[key]


@pytest.mark.parametrize("name,norm,rel", [("sin8193", "linf", 1e-4), ("sin8193", "l2", 1e-3),
                                           ("grf300", "linf", 1e-4), ("grf300", "l2", 1e-3)])
def test_full_size_fp64_and_non_dyadic(name, norm, rel):
    """8193^2 FP64 plane waves and a 300x400x500 FP32 |k|^-3 field."""
    torch, mgc = gpu()
    u = _cfg3(name)
    x = torch.from_numpy(u).cuda()
    blob = mgc.compress(x, rel, norm)
    v = mgc.decompress(blob).cpu().numpy()
    assert v.dtype == u.dtype and _bound_ok(u, v, rel, norm)
    g = to_bytes(blob)
    hd = parse_header(g)
    h = Hierarchy(u.shape)
    assert hd["L"] == h.L
    _, tau_eff = oracle.error_budget(u, rel, norm, "rel")
    q = oracle.level_bins(h, tau_eff, norm)
    if norm == "linf":
        assert np.array_equal(hd["q"], q)
    else:
        assert np.allclose(hd["q"], q, rtol=1e-13, atol=0)
    # sampled finest-level integers (with the stream's own bins)
    idx = np.random.default_rng(2).choice(u.size, 2000, replace=False)
    pos, c = oracle.transform.finest_coefficients_at(u.astype(np.float64), h, idx)
    k_ref = np.rint(c * (1.0 / hd["q"][h.L])).astype(np.int64)
    chunks = np.unique(pos // hd["C"])
    sym, opos, oval = decode_symbols(g, hd, chunks=chunks)
    k = sym[pos] - 32768
    esc = sym[pos] == 0
    if np.any(esc):
        where = np.searchsorted(opos.astype(np.int64), pos[esc])
        k[esc] = oval[where]
    assert np.count_nonzero(k != k_ref) <= 1e-6 * u.size
    assert np.all(np.abs(k - k_ref) <= 1)
