"""Asynchronous compression (mgc_compress): no host round trip, graph capture.

* the stream, the status and the length land in device memory; the blocking
  wrapper (mgc_compress_blocking, through ctypes) gives the same bytes;
* constant, NaN and too-small-bound inputs report their outcome in the
  device result words (MGC_OK with the trivial stream, MGC_EINVAL,
  MGC_ERANGE), and an outlier overflow reports MGC_ENOSPC with the count;
* mgc_compress captured once into a graph and replayed on new data (new
  bins: the relative bound is turned into bins on the device) gives, on
  every replay, the same bytes as an eager call; eager work and
  synchronisations run between the replays.
"""
import ctypes

import numpy as np
import pytest

import oracle
import synthetic
from tests.gpu_common import assert_stream_matches_oracle, gpu, to_bytes

pytestmark = pytest.mark.gpu


def _buffers(torch, mgc, shape, dtype, cap=0):
    ws_n, out_n = mgc.compress_query(shape, dtype, cap)
    ws = torch.empty(ws_n, dtype=torch.uint8, device="cuda")
    out = torch.zeros(out_n, dtype=torch.uint8, device="cuda")
    res = torch.full((2,), -1, dtype=torch.int64, device="cuda")
    return ws, out, res


@pytest.mark.parametrize("shape,dtype,norm", [((65, 65, 65), np.float32, "linf"),
                                              ((300, 41), np.float64, "l2"),
                                              ((1000,), np.float32, "linf")])
def test_async_result_words_and_blocking_wrapper(shape, dtype, norm):
    torch, mgc = gpu()
    u = synthetic.grf(shape, 3, dtype=dtype)
    x = torch.from_numpy(u).cuda()
    ws, out, res = _buffers(torch, mgc, shape, x.dtype)
    mgc.compress_async(x, 1e-3, norm, "rel", 0, ws, out, res)
    st, size = res.cpu().tolist()
    assert st == 0
    g = to_bytes(out[:size])
    assert_stream_matches_oracle(g, oracle.compress(u, 1e-3, norm), norm)
    # the blocking entry point through the C ABI writes the same stream
    lib = ctypes.CDLL(mgc.library_path())
    out2 = torch.zeros_like(out)
    n = ctypes.c_uint64()
    shp = (ctypes.c_uint64 * len(shape))(*shape)
    torch.cuda.synchronize()
    rc = lib.mgc_compress_blocking(
        mgc._ctx(0), ctypes.c_void_p(x.data_ptr()), len(shape), shp,
        0 if dtype == np.float32 else 1, ctypes.c_double(1e-3), {"linf": 0, "l2": 1}[norm], 0,
        ctypes.c_uint64(0), ctypes.c_void_p(out2.data_ptr()), ctypes.c_size_t(out2.numel()),
        ctypes.c_void_p(ws.data_ptr()), ctypes.c_size_t(ws.numel()),
        ctypes.c_void_p(torch.cuda.current_stream().cuda_stream), ctypes.byref(n))
    assert rc == 0 and n.value == size
    assert to_bytes(out2[:size]) == g


def test_async_outcomes_in_result_words():
    torch, mgc = gpu()
    shape = (33, 33, 33)
    const = torch.full(shape, 2.5, dtype=torch.float32, device="cuda")
    ws, out, res = _buffers(torch, mgc, shape, torch.float32)
    mgc.compress_async(const, 1e-3, "linf", "rel", 0, ws, out, res)
    st, size = res.cpu().tolist()
    assert st == 0 and size == 136
    assert to_bytes(out[:size]) == oracle.compress(const.cpu().numpy(), 1e-3)
    bad = torch.from_numpy(synthetic.grf(shape, 4)).cuda()
    bad[5, 6, 7] = float("inf")
    mgc.compress_async(bad, 1e-3, "linf", "rel", 0, ws, out, res)
    assert res.cpu().tolist()[0] == 1                      # EINVAL
    tiny = torch.from_numpy(synthetic.grf(shape, 5)).cuda()
    mgc.compress_async(tiny, 1e-9, "linf", "rel", 0, ws, out, res)
    assert res.cpu().tolist()[0] == 6                      # ERANGE: no budget left
    ws2, out2, res2 = _buffers(torch, mgc, shape, torch.float32, cap=4)
    mgc.compress_async(tiny, 1e-6, "linf", "rel", 4, ws2, out2, res2)
    st, need = res2.cpu().tolist()
    assert st == 3 and need > 4                           # ENOSPC + escaped count
    # after the failures a good input compresses normally on the same buffers
    mgc.compress_async(tiny, 1e-3, "linf", "rel", 0, ws, out, res)
    st, size = res.cpu().tolist()
    assert st == 0 and to_bytes(out[:size]) == to_bytes(mgc.compress(tiny, 1e-3))


@pytest.mark.parametrize("shape", [(129, 129, 129), (257, 200), (65, 65, 65)])
def test_compress_captured_in_a_graph_replays_identically(shape):
    torch, mgc = gpu()
    seeds = [21, 22, 23, 24]
    fields = [synthetic.grf(shape, sd) for sd in seeds]
    x = torch.from_numpy(fields[0]).cuda()
    ws, out, res = _buffers(torch, mgc, shape, x.dtype)
    mgc.compress_async(x, 1e-3, "linf", "rel", 0, ws, out, res)   # builds the plan
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        mgc.compress_async(x, 1e-3, "linf", "rel", 0, ws, out, res)
    torch.cuda.synchronize()
    for rep, u in enumerate(fields[1:] + fields[:1]):
        x.copy_(torch.from_numpy(u))
        out.zero_()
        res.fill_(-1)
        g.replay()
        torch.cuda.synchronize()
        st, size = res.cpu().tolist()
        assert st == 0, rep
        got = to_bytes(out[:size])
        # eager work between replays: a plain compression of the same data
        ref = to_bytes(mgc.compress(torch.from_numpy(u).cuda(), 1e-3))
        torch.cuda.synchronize()
        assert got == ref, "replay %d differs from the eager stream" % rep
    hd = oracle.parse_header(got)
    assert hd["N"] == int(np.prod(shape))
