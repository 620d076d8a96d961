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
    from oracle import hx
    return hx.huffman_section(np.asarray(sym, dtype=np.int64), C)


def rebuild_stream_from_integers(gpu_stream: bytes, k: np.ndarray) -> bytes:
    """The oracle's stream for the integers ``k``, with ``gpu_stream``'s own
    header and bins: symbols, outliers, codebook, chunk offsets and coded
    words all come from the oracle's Huffman stage (Algorithm 2).  Used when
    a full-size GPU stream differs from the oracle's only because some
    integers sit on bin-boundary ties, to show the Huffman stage is still
    bit-exact on the GPU's own integers."""
    from oracle import stream as ostream
    from oracle.quantize import to_symbols
    hd = ostream.parse_header(gpu_stream)
    S, C, L = hd["S"], hd["C"], hd["L"]
    sym, opos, oval = to_symbols(np.asarray(k, dtype=np.int64), S)
    ln = huffman.code_lengths(huffman.histogram(sym, S))
    codes = huffman.canonical_codes(ln)
    offsets, words = huffman.encode_chunks(sym, ln, codes, C)
    coded = np.nonzero(ln)[0]
    cb, off, o_pos, o_val, w_off, end = ostream.section_offsets(L, len(coded), len(offsets) - 1,
                                                                 len(opos), len(words))
    out = bytearray(end)
    out[0:cb] = gpu_stream[0:cb]
    out[cb:cb + 2 * len(coded)] = coded.astype("<u2").tobytes()
    out[cb + 2 * len(coded):cb + 3 * len(coded)] = ln[coded].astype("u1").tobytes()
    out[off:o_pos] = offsets.astype("<u8").tobytes()
    out[o_pos:o_val] = opos.astype("<u8").tobytes()
    out[o_val:w_off] = oval.astype("<i8").tobytes()
    out[w_off:w_off + 4 * len(words)] = words.astype("<u4").tobytes()
    return bytes(out)


def assert_stream_matches_oracle(g: bytes, r: bytes, norm: str, tie_frac: float = 1e-6):
    """A GPU stream against the oracle's stream of the same array and request.

    Every header field must agree; the bins, tau and tau' exactly for L-inf
    and to 1e-13 relative for L2 (their sum of squares is reduced in a
    different order).  Then the rest of the stream must be byte-identical,
    which makes every quantised integer of every level, the codebook, the
    chunk offsets, the outliers and the coded words equal.  Otherwise the
    integers may differ only at bin-boundary ties (at most ``tie_frac`` of
    the points, each by one), and the oracle's Huffman stage applied to the
    GPU's own integers must then reproduce the GPU stream exactly.
    Returns the number of integers that differ.
    """
    from oracle import stream as ostream
    from oracle.quantize import from_symbols
    hg, hr = ostream.parse_header(g), ostream.parse_header(r)
    for key in ("dtype", "norm", "mode", "shape", "flags", "D", "L", "bound", "const", "S",
                "C", "N", "n_chunks"):
        assert hg[key] == hr[key], "header field %s: %r vs %r" % (key, hg[key], hr[key])
    if hg["flags"]:
        assert g == r
        return 0
    L = hg["L"]
    qa, qb = hg["q"], hr["q"]
    if norm == "linf":
        assert np.array_equal(qa, qb) and hg["tau"] == hr["tau"] and hg["tau_eff"] == hr["tau_eff"]
    else:
        assert np.allclose(qa, qb, rtol=1e-13, atol=0)
        assert abs(hg["tau"] - hr["tau"]) <= 1e-13 * abs(hr["tau"])
        assert abs(hg["tau_eff"] - hr["tau_eff"]) <= 1e-13 * abs(hr["tau_eff"])

    def masked(b):
        b = bytearray(b)
        b[48:64] = bytes(16)                       # tau, tau'
        b[128:128 + 8 * (L + 1)] = bytes(8 * (L + 1))  # bins
        return bytes(b)

    if len(g) == len(r) and masked(g) == masked(r):
        return 0
    kg = from_symbols(*ostream.decode_symbols(g, hg))
    kr = from_symbols(*ostream.decode_symbols(r, hr))
    diff = np.nonzero(kg != kr)[0]
    assert len(diff) <= tie_frac * hg["N"], "%d integers differ" % len(diff)
    assert np.all(np.abs(kg[diff] - kr[diff]) <= 1)
    assert rebuild_stream_from_integers(g, kg) == g, \
        "the GPU's Huffman stage differs from the oracle's on the GPU's integers"
    return len(diff)
