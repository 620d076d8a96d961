"""Helpers shared by the GPU parity tests (test-side only)."""
import struct

import numpy as np
import pytest

from oracle import huffman


def gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2503_06322_amd as mgc
    import os
    if not os.path.exists(mgc.library_path()):
        pytest.fail("libmgc.so is not built")
    return torch, mgc


def to_bytes(t) -> bytes:
    return t.cpu().numpy().tobytes()


def oracle_huffman_stream(sym: np.ndarray, C: int) -> bytes:
    """The Huffman-only stream layout assembled from the oracle's stages."""
    N = len(sym)
    ln = huffman.code_lengths(huffman.histogram(sym, 65536))
    codes = huffman.canonical_codes(ln)
    off, words = huffman.encode_chunks(sym, ln, codes, C)
    coded = np.nonzero(ln)[0]
    nc = len(coded)
    n_chunks = len(off) - 1
    pad8 = lambda n: (n + 7) // 8 * 8
    o_off = pad8(48 + 3 * nc)
    w_off = o_off + 8 * (n_chunks + 1)
    end = pad8(w_off + 4 * len(words))
    out = bytearray(end)
    out[0:48] = struct.pack("<II5Q", 0x3148474D, C, N, nc, n_chunks, len(words), end)
    out[48:48 + 2 * nc] = coded.astype("<u2").tobytes()
    out[48 + 2 * nc:48 + 3 * nc] = ln[coded].astype("u1").tobytes()
    out[o_off:w_off] = off.astype("<u8").tobytes()
    out[w_off:w_off + 4 * len(words)] = words.astype("<u4").tobytes()
    return bytes(out)
