"""Allocation-free compression (mgc_compress_noalloc) against mgc_compress.

The allocation-free call keeps its plan tables and work buffers in the
library's per-device scratch array; its streams and result words must equal
those of the ordinary asynchronous call, byte for byte, on consecutive calls
whose shapes differ (the scratch keeps the previous call's contents, and a
new shape re-uploads the tables).
"""
import numpy as np
import pytest

import synthetic
from tests.gpu_common import gpu

pytestmark = pytest.mark.gpu


def _both(torch, mgc, x, rel, norm):
    print("case: %s %s %s %g" % (tuple(x.shape), x.dtype, norm, rel), flush=True)
    ws_n, out_n = mgc.compress_query(tuple(x.shape), x.dtype)
    ws = torch.empty(ws_n, dtype=torch.uint8, device="cuda")
    out_a = torch.zeros(out_n, dtype=torch.uint8, device="cuda")
    out_b = torch.full((out_n,), 0xA5, dtype=torch.uint8, device="cuda")
    ra = torch.zeros(2, dtype=torch.int64, device="cuda")
    rb = torch.full((2,), -7, dtype=torch.int64, device="cuda")
    mgc.compress_async(x, rel, norm, workspace=ws, out=out_a, result=ra)
    mgc.compress_noalloc(x, rel, out_b, rb, norm)
    torch.cuda.synchronize()
    a, b = ra.tolist(), rb.tolist()
    assert a[0] == 0 and a == b, (a, b)
    n = a[1]
    assert torch.equal(out_a[:n], out_b[:n])
    return n


def test_noalloc_equals_compress_on_consecutive_calls():
    torch, mgc = gpu()
    big = torch.from_numpy(synthetic.grf((129, 129, 129), 21)).cuda()
    small = torch.from_numpy(synthetic.bumps((33, 20, 17), 22)).cuda()
    plane = torch.from_numpy(synthetic.sinusoids((257, 300), 23)).cuda()
    n_big = _both(torch, mgc, big, 1e-3, "linf")
    n_small = _both(torch, mgc, small, 1e-4, "linf")     # second call, smaller input
    assert n_small < n_big
    _both(torch, mgc, plane, 1e-3, "l2")
    _both(torch, mgc, small, 1e-2, "linf")
    _both(torch, mgc, big, 1e-4, "linf")                  # tables of the first shape again
    # the decompressed stream stays within the bound
    out = torch.empty(mgc.compress_query(tuple(small.shape), small.dtype)[1],
                      dtype=torch.uint8, device="cuda")
    res = torch.zeros(2, dtype=torch.int64, device="cuda")
    mgc.compress_noalloc(small, 1e-3, out, res)
    st, n = res.tolist()
    assert st == 0
    y = mgc.decompress(out[:n])
    tau = 1e-3 * (small.max() - small.min()).item()
    assert torch.max(torch.abs(y.double() - small.double())).item() <= tau


def test_noalloc_rejects_arrays_beyond_its_scratch():
    torch, mgc = gpu()
    x = torch.zeros((257, 257, 257), dtype=torch.float32, device="cuda")
    out = torch.empty(16, dtype=torch.uint8, device="cuda")
    res = torch.zeros(2, dtype=torch.int64, device="cuda")
    with pytest.raises(mgc.MgcError) as e:
        mgc.compress_noalloc(x, 1e-3, out, res)
    assert e.value.name == "ENOSPC"
    assert "scratch" in str(e.value)
    # nothing was enqueued: the result words are untouched
    torch.cuda.synchronize()
    assert res.tolist() == [0, 0]
