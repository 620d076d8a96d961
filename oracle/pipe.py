"""Chunked compression of host-resident arrays (oracle; test infrastructure).

TEST INFRASTRUCTURE ONLY.

Section V of the paper moves large arrays through the GPU in chunks along
their largest dimension, each chunk reduced on its own, with the chunk size
adapted as the pipeline runs (Algorithm "Adaptive Pipeline"):
C_next = min(Theta(C_curr / Phi(C_curr)), C_limit), capped by the data left,
Phi(C) = alpha C + beta below a threshold and gamma above (the compression
throughput model), Theta(t) = t / beta_h2d (the bytes the host can copy in
during t).  The readings used (the printed algorithm is garbled: its queue
and buffer indices are swapped against the prose and its remaining-size
update subtracts the wrong chunk):

* chunks are whole planes of the slowest axis (contiguous in host memory;
  the paper's largest dimension for its NYX and E3SM fields);
* a chunk of C bytes holds max(1, floor(C / plane bytes)) planes;
* the chunk size never shrinks (the prose: the size grows as the reduction
  makes progress) and starts at C_init; with no throughput model every chunk
  has C_init bytes;
* each chunk is compressed as an array of its own with the whole array's
  absolute bound: tau for L-inf, tau * sqrt(chunk values / values) for L2,
  so the errors of the chunks add up to at most tau in that norm; a relative
  bound is turned into tau from the whole array's range (or norm) first.

Container (little-endian): u32 magic 0x5043474D, u32 chunk count, u8 dtype,
norm, mode, ndim, u32 0, u64 shape[3], f64 bound, f64 tau, u64 total bytes
(64-byte header); per chunk {u64 first plane, u64 planes, u64 stream
offset, u64 stream bytes}; then the chunk streams (``stream.compress``'s
format), each at a multiple of 8 bytes, zero padding between them.
"""
from __future__ import annotations

import math
import struct

import numpy as np

from . import stream as _stream

MAGIC = 0x5043474D
HEADER_BYTES = 64
ENTRY_BYTES = 32
DEFAULT_INIT = 64 << 20
DEFAULT_LIMIT = 1 << 30
_DT = {np.dtype(np.float32): 0, np.dtype(np.float64): 1}
_NORMS = {"linf": 0, "l2": 1}
_MODES = {"rel": 0, "abs": 1}


def _pad8(n: int) -> int:
    return (n + 7) // 8 * 8


def resolve_model(model: dict | None) -> dict:
    m = dict(init_chunk_bytes=0, limit_chunk_bytes=0, phi_alpha=0.0, phi_beta=0.0,
             phi_gamma=0.0, phi_threshold=0, h2d_bytes_per_s=0.0)
    if model:
        m.update(model)
    if not m["init_chunk_bytes"]:
        m["init_chunk_bytes"] = DEFAULT_INIT
    if not m["limit_chunk_bytes"]:
        m["limit_chunk_bytes"] = DEFAULT_LIMIT
    m["limit_chunk_bytes"] = max(m["limit_chunk_bytes"], m["init_chunk_bytes"])
    return m


def phi(m: dict, C: float) -> float:
    """Compression throughput model (bytes/s) at a chunk of C bytes."""
    if C >= float(m["phi_threshold"]):
        return float(m["phi_gamma"])
    return max(float(m["phi_alpha"]) * C + float(m["phi_beta"]), 1.0)


def next_chunk_bytes(m: dict, cur: int) -> int:
    """C_next = min(max(Theta(C / Phi(C)), C), C_limit) in bytes."""
    if not (m["phi_gamma"] > 0.0) or not (m["h2d_bytes_per_s"] > 0.0):
        return cur
    t = float(cur) / phi(m, float(cur))
    c = t * float(m["h2d_bytes_per_s"])
    return int(min(max(c, float(cur)), float(m["limit_chunk_bytes"])))


def chunk_planes(shape, itemsize: int, model: dict | None):
    """[(first plane, planes)] of the chunks of an array of ``shape``."""
    m = resolve_model(model)
    pb = int(np.prod(shape[1:], dtype=np.int64)) * itemsize
    out, p0, cur = [], 0, int(m["init_chunk_bytes"])
    while p0 < shape[0]:
        n = min(max(1, cur // pb), shape[0] - p0)
        out.append((p0, n))
        p0 += n
        cur = next_chunk_bytes(m, cur)
    return out


def absolute_bound(u: np.ndarray, bound: float, norm: str, mode: str) -> float:
    if mode == "abs":
        return float(bound)
    ud = np.asarray(u, dtype=np.float64)
    mn, mx = float(ud.min()), float(ud.max())
    if mn == mx:
        return 1.0          # a constant array: every chunk stores its value
    if norm == "linf":
        return float(bound) * (mx - mn)
    return float(bound) * math.sqrt(float(np.sum(ud * ud)))


def chunk_bound(tau: float, norm: str, n_chunk: int, n: int) -> float:
    return tau if norm == "linf" else tau * math.sqrt(float(n_chunk) / float(n))


def compress(u: np.ndarray, bound: float, norm: str = "linf", mode: str = "rel",
             model: dict | None = None) -> bytes:
    u = np.asarray(u)
    tau = absolute_bound(u, bound, norm, mode)
    chunks = chunk_planes(u.shape, u.dtype.itemsize, model)
    K = len(chunks)
    table = HEADER_BYTES + ENTRY_BYTES * K
    off = _pad8(table)
    body, entries = [], []
    for p0, n in chunks:
        part = u[p0:p0 + n]
        s = _stream.compress(part, chunk_bound(tau, norm, part.size, u.size), norm, "abs")
        entries.append((p0, n, off, len(s)))
        body.append((off, s))
        off = _pad8(off + len(s))
    out = bytearray(off)
    shp = list(u.shape) + [0] * (3 - u.ndim)
    out[0:HEADER_BYTES] = struct.pack("<IIBBBBI3QddQ", MAGIC, K, _DT[np.dtype(u.dtype)],
                                      _NORMS[norm], _MODES[mode], u.ndim, 0, *shp,
                                      float(bound), tau, off)
    for i, e in enumerate(entries):
        struct.pack_into("<4Q", out, HEADER_BYTES + ENTRY_BYTES * i, *e)
    for o, s in body:
        out[o:o + len(s)] = s
    return bytes(out)


def parse(buf: bytes) -> dict:
    f = struct.unpack_from("<IIBBBBI3QddQ", buf, 0)
    magic, K, dt, nm, md, ndim, _, s0, s1, s2, bound, tau, total = f
    if magic != MAGIC:
        raise ValueError("not a chunked container")
    ent = [struct.unpack_from("<4Q", buf, HEADER_BYTES + ENTRY_BYTES * i) for i in range(K)]
    return dict(K=K, dtype=np.float32 if dt == 0 else np.float64, norm=["linf", "l2"][nm],
                mode=["rel", "abs"][md], shape=(s0, s1, s2)[:ndim], bound=bound, tau=tau,
                total=total, entries=ent)


def decompress(buf: bytes) -> np.ndarray:
    h = parse(buf)
    parts = [_stream.decompress(buf[o:o + nb]) for (_, _, o, nb) in h["entries"]]
    return np.concatenate(parts, axis=0).reshape(h["shape"])
