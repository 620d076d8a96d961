"""GPU host-device pipeline (Section V, Algorithm "Adaptive Pipeline"):
containers equal to the oracle's (chunk table, per-chunk bounds, chunk
streams), the whole array's bound after decompression, model-driven chunk
sizes, and a full-size field against plain per-chunk GPU calls."""
import struct

import numpy as np
import pytest

import synthetic
from oracle import pipe as opipe
from oracle import stream as ostream
from tests.gpu_common import assert_stream_matches_oracle, gpu

pytestmark = pytest.mark.gpu


def _pinned(torch, a):
    t = torch.from_numpy(np.ascontiguousarray(a))
    return t.pin_memory()


def _check_container(g: bytes, r: bytes, norm: str):
    hg, hr = opipe.parse(g), opipe.parse(r)
    for k in ("K", "dtype", "norm", "mode", "shape", "bound"):
        assert hg[k] == hr[k], k
    assert abs(hg["tau"] - hr["tau"]) <= 1e-13 * abs(hr["tau"])
    assert [e[:2] for e in hg["entries"]] == [e[:2] for e in hr["entries"]]
    for (_, _, og, ng), (_, _, orr, nr) in zip(hg["entries"], hr["entries"]):
        assert_stream_matches_oracle(g[og:og + ng], r[orr:orr + nr], norm)


CASES = [  # (field, shape, dtype, norm, mode, bound, init planes)
    ("grf", (37, 20, 24), np.float32, "linf", "rel", 1e-3, 5),
    ("grf", (37, 20, 24), np.float32, "l2", "rel", 1e-3, 4),
    ("grf", (29, 33, 17), np.float64, "linf", "abs", 0.02, 6),
    ("sin", (300, 257), np.float64, "l2", "abs", 0.5, 40),
    ("bumps", (65, 65, 65), np.float32, "linf", "rel", 1e-4, 16),
]


@pytest.mark.parametrize("field,shape,dt,norm,mode,bound,ip", CASES)
def test_container_matches_oracle(field, shape, dt, norm, mode, bound, ip):
    torch, mgc = gpu()
    if field == "grf":
        u = synthetic.grf(shape, 11, dtype=dt)
    elif field == "sin":
        u = synthetic.sinusoids(shape, 12).astype(dt)
    else:
        u = synthetic.bumps(shape, 13).astype(dt)
    pb = int(np.prod(shape[1:])) * np.dtype(dt).itemsize
    model = {"init_chunk_bytes": ip * pb}
    got, st = mgc.pipe_compress(_pinned(torch, u), bound, norm, mode, model)
    g = got.numpy().tobytes()
    r = opipe.compress(u, bound, norm, mode, model)
    _check_container(g, r, norm)
    assert st["chunks"] == opipe.parse(r)["K"]
    v, _ = mgc.pipe_decompress(got)
    v = v.numpy()
    assert v.shape == u.shape and v.dtype == u.dtype
    tau = opipe.parse(g)["tau"]
    e = v.astype(np.float64) - u.astype(np.float64)
    if norm == "linf":
        assert np.max(np.abs(e)) <= tau
    else:
        assert np.linalg.norm(e.ravel()) <= tau
    ref = opipe.decompress(r)
    assert np.max(np.abs(v.astype(np.float64) - ref)) <= 1e-12 * max(1.0, float(np.max(np.abs(u))))


def test_model_driven_chunk_sizes_follow_the_oracle_rule():
    torch, mgc = gpu()
    u = synthetic.grf((120, 16, 16), 14)
    pb = 16 * 16 * 4
    model = {"init_chunk_bytes": 3 * pb, "limit_chunk_bytes": 40 * pb, "phi_alpha": 2.0,
             "phi_beta": 1.0e4, "phi_gamma": 5.0e5, "phi_threshold": 30 * pb,
             "h2d_bytes_per_s": 9.0e4}
    got, st = mgc.pipe_compress(_pinned(torch, u), 1e-3, "linf", "rel", model)
    g = got.numpy().tobytes()
    want = opipe.chunk_planes(u.shape, 4, model)
    assert len(want) > 4 and len({n for _, n in want}) > 2   # the sizes really change
    assert [e[:2] for e in opipe.parse(g)["entries"]] == want
    _check_container(g, opipe.compress(u, 1e-3, "linf", "rel", model), "linf")


def test_profiled_model_and_full_size_field():
    # 513^3 FP32 (540 MB): the profiled model, then every chunk stream equal
    # to the plain GPU compression of its planes at the chunk bound, the
    # whole array's bound after the pipeline's decompression, and copies
    # that overlap the kernels
    torch, mgc = gpu()
    u = synthetic.grf((513, 513, 513), 2)
    x = _pinned(torch, u)
    m = mgc.pipe_profile(x, 1e-3, "linf", "rel", {"init_chunk_bytes": 32 << 20,
                                                   "limit_chunk_bytes": 256 << 20})
    assert m["phi_gamma"] > 0 and m["h2d_bytes_per_s"] > 0 and m["phi_threshold"] > 0
    got, st = mgc.pipe_compress(x, 1e-3, "linf", "rel", m)
    g = got.numpy().tobytes()
    h = opipe.parse(g)
    assert h["K"] == st["chunks"] >= 2
    assert [e[:2] for e in h["entries"]] == opipe.chunk_planes(u.shape, 4, m)
    assert h["tau"] == 1e-3 * (float(u.max()) - float(u.min()))
    for p0, n, off, nb in h["entries"][:3]:
        part = torch.from_numpy(np.ascontiguousarray(u[p0:p0 + n])).cuda()
        ref = mgc.compress(part, h["tau"], "linf", "abs")
        assert g[off:off + nb] == ref.cpu().numpy().tobytes()
    v, st2 = mgc.pipe_decompress(got)
    err = np.max(np.abs(v.numpy().astype(np.float64) - u.astype(np.float64)))
    assert err <= h["tau"]
    assert st["overlap"] > 0.0 and st2["overlap"] > 0.0


def test_corrupt_containers_are_rejected():
    torch, mgc = gpu()
    u = synthetic.grf((20, 16, 16), 15)
    got, _ = mgc.pipe_compress(_pinned(torch, u), 1e-3, "linf", "rel",
                               {"init_chunk_bytes": 4 * 16 * 16 * 4})
    bad = got.clone()
    bad[0] = 0
    with pytest.raises(mgc.MgcError):
        mgc.pipe_decompress(bad)
    b = bytearray(got.numpy().tobytes())
    struct.pack_into("<Q", b, 64 + 32 + 8, 3)        # chunk 1 claims 3 planes, not 4
    with pytest.raises(mgc.MgcError) as e:
        mgc.pipe_decompress(torch.from_numpy(np.frombuffer(bytes(b), dtype=np.uint8).copy()))
    assert e.value.name == "EFORMAT"
