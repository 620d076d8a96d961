"""Pins of the chunked host-resident pipeline's oracle (Section V, Algorithm
"Adaptive Pipeline"): the chunk-size rule worked by hand, the container, and
the whole array's error bound after chunk-wise compression."""
import struct

import numpy as np
import pytest

import synthetic
from oracle import pipe


def test_chunk_rule_without_a_model_keeps_the_initial_size():
    # 100 planes of 1 KiB, C_init = 7 KiB: 7 planes a chunk, 2 left over
    ch = pipe.chunk_planes((100, 16, 16), 4, {"init_chunk_bytes": 7 * 1024})
    assert ch == [(7 * k, 7) for k in range(14)] + [(98, 2)]


def test_chunk_rule_follows_the_throughput_models_by_hand():
    # Phi(C) = 0.5 C + 1000 B/s below 8000 B, 5000 B/s above; Theta(t) = 2000 t.
    # C0 = 1000: Phi = 1500, t = 2/3 s, Theta = 1333.3 -> 1333
    # C1 = 1333: Phi = 1666.5, t = 0.79988, Theta = 1599.76 -> 1599
    # C2 = 1599: Phi = 1799.5, t = 0.88858, Theta = 1777.16 -> 1777
    m = {"init_chunk_bytes": 1000, "limit_chunk_bytes": 100000, "phi_alpha": 0.5,
         "phi_beta": 1000.0, "phi_gamma": 5000.0, "phi_threshold": 8000,
         "h2d_bytes_per_s": 2000.0}
    seq = [1000]
    for _ in range(3):
        seq.append(pipe.next_chunk_bytes(m, seq[-1]))
    assert seq == [1000, 1333, 1599, 1777]
    # a fast compressor (Phi above the copy rate) never shrinks the chunks
    m2 = dict(m, phi_alpha=0.0, phi_beta=1e9, phi_gamma=1e9)
    assert pipe.next_chunk_bytes(m2, 1000) == 1000
    # the limit caps the growth
    m3 = dict(m, limit_chunk_bytes=1200)
    assert pipe.next_chunk_bytes(m3, 1000) == 1200
    # planes from the sizes: 100-byte planes
    ch = pipe.chunk_planes((40, 25), 4, m)
    assert ch[:4] == [(0, 10), (10, 13), (23, 15), (38, 2)]


@pytest.mark.parametrize("norm,mode,bound", [("linf", "rel", 1e-3), ("l2", "rel", 1e-3),
                                              ("linf", "abs", 0.01), ("l2", "abs", 0.5)])
def test_container_holds_the_whole_arrays_bound(norm, mode, bound):
    u = synthetic.grf((37, 20, 24), 6)
    buf = pipe.compress(u, bound, norm, mode, {"init_chunk_bytes": 5 * 20 * 24 * 4})
    h = pipe.parse(buf)
    assert h["K"] == 8 and len(buf) == h["total"]
    assert [e[:2] for e in h["entries"]] == [(5 * k, 5) for k in range(7)] + [(35, 2)]
    v = pipe.decompress(buf)
    e = v.astype(np.float64) - u.astype(np.float64)
    tau = pipe.absolute_bound(u, bound, norm, mode)
    if norm == "linf":
        assert np.max(np.abs(e)) <= tau
    else:
        assert np.linalg.norm(e.ravel()) <= tau
    # every chunk is the stream of its planes alone, at its share of the bound
    from oracle import stream
    for p0, n, off, nb in h["entries"]:
        s = stream.compress(u[p0:p0 + n], pipe.chunk_bound(tau, norm, n * 480, u.size), norm, "abs")
        assert buf[off:off + nb] == s
    assert struct.unpack_from("<I", buf, 0)[0] == 0x5043474D


def test_constant_array_and_single_chunk():
    u = np.full((9, 5), 3.25, dtype=np.float32)
    buf = pipe.compress(u, 1e-3, "linf", "rel", {"init_chunk_bytes": 4 * 5 * 4})
    assert np.array_equal(pipe.decompress(buf), u)
    u = synthetic.grf((12, 8, 8), 7)
    buf = pipe.compress(u, 1e-2, "linf", "rel")
    assert pipe.parse(buf)["K"] == 1
