"""The C-ABI library loads and exports every function include/mgc.h declares.

No compute call is made (no GPU here); size queries are host-only.
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mgc.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(mgc_[a-z_0-9]+)\s*\(", txt)))


def _lib():
    import paper_2503_06322_amd as mgc
    path = mgc.library_path()
    if not os.path.exists(path):
        pytest.skip("libmgc.so not built")
    return ctypes.CDLL(path)


def test_header_declares_entry_points():
    names = _declared()
    for n in ("mgc_compress", "mgc_decompress", "mgc_decompose", "mgc_recompose",
              "mgc_huffman_encode", "mgc_huffman_decode", "mgc_header_info"):
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = _lib()
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_host_only_queries():
    import paper_2503_06322_amd as mgc
    import torch
    _lib()
    ws, mx = mgc.compress_query((513, 513, 513), torch.float32)
    N = 513 ** 3
    assert ws > 2 * N and mx > 4 * N
    assert mgc.transform_query((65, 65, 65)) >= 2 * 8 * 33 ** 3
    with pytest.raises(mgc.MgcError) as e:
        mgc.compress_query((2, 2, 2, 2), torch.float32)
    assert e.value.name == "EUNSUPPORTED"


def test_header_info_parses_oracle_stream():
    import numpy as np
    import torch
    import oracle
    import synthetic
    import paper_2503_06322_amd as mgc
    _lib()
    u = synthetic.grf((17, 9, 5), 3)
    b = oracle.compress(u, 1e-2)
    info = mgc.header_info(torch.from_numpy(np.frombuffer(b, dtype=np.uint8).copy()))
    assert info["shape"] == (17, 9, 5) and info["dtype"] == torch.float32
    assert info["stream_bytes"] == len(b)
    bad = bytearray(b)
    bad[0] ^= 1
    with pytest.raises(mgc.MgcError) as e:
        mgc.header_info(torch.from_numpy(np.frombuffer(bytes(bad), dtype=np.uint8).copy()))
    assert e.value.name == "EFORMAT"


def test_gpu_entry_points_refuse_cpu_tensors():
    import torch
    import paper_2503_06322_amd as mgc
    _lib()
    with pytest.raises(ValueError):
        mgc.compress(torch.zeros(8, 8), 1e-3)


def test_batch_query_lays_out_plain_slots():
    """Batched output slots are the plain worst-case sizes, 256-byte aligned."""
    import torch
    import paper_2503_06322_amd as mgc
    _lib()
    shapes = [(33, 65, 17), (257,), (0, 5), (9, 9), (65, 65, 65)]
    dtypes = [torch.float32, torch.float64, torch.float32, torch.float64, torch.float32]
    ws, total, offs = mgc.batch_query(shapes, dtypes)
    pos = 0
    wsum = 0
    for shp, dt, off in zip(shapes, dtypes, offs):
        w1, m1 = mgc.compress_query(shp, dt)
        assert off == pos
        pos += (m1 + 255) // 256 * 256
        wsum += (w1 + 255) // 256 * 256
    assert total == pos and ws == wsum
    with pytest.raises(ValueError):
        mgc.batch_query([(4, 4, 4, 4)], [torch.float32])
    with pytest.raises(mgc.MgcError) as e:
        mgc.batch_query([], [])
    assert e.value.name == "EINVAL"


def test_hx_host_calls():
    """Huffman-X size query and header parsing run on the host."""
    import numpy as np
    from oracle import hx
    lib = _lib()
    ws, mx = ctypes.c_size_t(), ctypes.c_size_t()
    assert lib.mgc_hx_query(ctypes.c_uint64(100000), 2, ctypes.c_uint32(1024), ctypes.byref(ws),
                            ctypes.byref(mx)) == 0
    # header, the largest coded section, and every value escaped (4 bytes each)
    assert mx.value >= 64 + 48 + 4 * 100000 + 4 * 100000
    assert lib.mgc_hx_query(ctypes.c_uint64(10), 7, ctypes.c_uint32(1024), None, None) == 1
    assert lib.mgc_hx_query(ctypes.c_uint64(10), 0, ctypes.c_uint32(100), None, None) == 1
    buf = hx.compress(np.array([5, -70000, 3], dtype=np.int64), D=1024, b=-7)
    t, n, d, C, tot = ctypes.c_int(), ctypes.c_uint64(), ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint64()
    b = ctypes.c_int64()
    assert lib.mgc_hx_parse_header(buf, ctypes.c_size_t(len(buf)), ctypes.byref(t), ctypes.byref(n),
                                   ctypes.byref(d), ctypes.byref(b), ctypes.byref(C),
                                   ctypes.byref(tot)) == 0
    assert (t.value, n.value, d.value, b.value, C.value, tot.value) == (3, 3, 1024, -7, 1024, len(buf))
    assert lib.mgc_hx_parse_header(b"\0" * 64, ctypes.c_size_t(64), None, None, None, None, None,
                                   None) == 4
