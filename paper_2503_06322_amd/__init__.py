"""MI355X multigrid error-bounded lossy compressor: Python binding of libmgc.

Thin ctypes layer over the C ABI declared in ``include/mgc.h``.  It only
marshals arguments: every stage runs in the HIP kernels of ``libmgc.so``;
PyTorch provides device memory and the current stream.  There is no CPU
fallback: calling any entry point without the built library or with tensors
that are not on a GPU raises.

Entry points (same names as the C functions, without the ``mgc_`` prefix):

``compress(x, error_bound, norm="linf", mode="rel")``  -> uint8 device tensor
``decompress(stream)``                                   -> device tensor
``decompose(x)`` / ``recompose(coeffs, shape, dtype)``   (FP64 coefficients)
``compress_batched(tensors, bounds)`` / ``Batch`` (one graph launch for many arrays)
``huffman_encode(symbols, C=1024)`` / ``huffman_decode(stream, n)``
``hx_compress(x, dict, base, C)`` / ``hx_decompress(stream)`` (Huffman-X lossless codec)
``pipe_compress(host_x, bound)`` / ``pipe_decompress(container)`` / ``pipe_profile`` (host-resident arrays)
``zfp_compress(x, rate)`` / ``zfp_decompress(stream)`` (fixed-rate block transform coding)
``header_info(stream)``, ``profile_enable / profile_reset / profile_read``
"""
from __future__ import annotations

import ctypes
import os
import threading

__all__ = ["MgcError", "library_path", "compress", "compress_async", "decompress", "decompose", "recompose",
           "recompose_adjoint", "recompose_levels", "Recompose", "huffman_encode",
           "huffman_decode", "header_info", "profile_enable", "profile_reset", "profile_read",
           "compress_query", "transform_query", "batch_query", "Batch", "compress_batched",
           "set_tuning", "tuning_info", "set_decoder", "decoder_info", "compress_noalloc",
           "NOALLOC_SCRATCH_BYTES", "hx_query", "hx_compress", "hx_decompress", "hx_header",
           "pipe_max_bytes", "pipe_compress", "pipe_decompress", "pipe_profile", "zfp_query",
           "zfp_compress", "zfp_decompress"]

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libmgc.so")
_lib = None
_lock = threading.Lock()
_ctxs = {}

_STATUS = {0: "OK", 1: "EINVAL", 2: "EUNSUPPORTED", 3: "ENOSPC", 4: "EFORMAT",
           5: "EDEVICE", 6: "ERANGE"}
_NORM = {"linf": 0, "l2": 1}
_MODE = {"rel": 0, "abs": 1}
HEADER_PREFIX = 128 + 8 * 63


class PipeModel(ctypes.Structure):
    """mgc_pipe_model: chunk sizes and the throughput models of the pipeline."""
    _fields_ = [("init_chunk_bytes", ctypes.c_uint64), ("limit_chunk_bytes", ctypes.c_uint64),
                ("phi_alpha", ctypes.c_double), ("phi_beta", ctypes.c_double),
                ("phi_gamma", ctypes.c_double), ("phi_threshold", ctypes.c_uint64),
                ("h2d_bytes_per_s", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class PipeStats(ctypes.Structure):
    """mgc_pipe_stats: seconds per kind of task, overlap ratio, chunk count."""
    _fields_ = [("total_s", ctypes.c_double), ("h2d_s", ctypes.c_double),
                ("kernel_s", ctypes.c_double), ("d2h_s", ctypes.c_double),
                ("prepass_s", ctypes.c_double), ("overlap", ctypes.c_double),
                ("chunks", ctypes.c_uint64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class MgcError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__("%s: %s" % (_STATUS.get(status, status), message))
        self.status = status
        self.name = _STATUS.get(status, str(status))


def library_path() -> str:
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(_LIB_PATH):
            raise ImportError("libmgc.so is not built; run `python -m paper_2503_06322_amd.build`")
        lib = ctypes.CDLL(_LIB_PATH)
        c_u64p = ctypes.POINTER(ctypes.c_uint64)
        c_szp = ctypes.POINTER(ctypes.c_size_t)
        vp = ctypes.c_void_p
        sig = {
            "mgc_create": [ctypes.c_int, ctypes.POINTER(vp)],
            "mgc_destroy": [vp],
            "mgc_compress_query": [ctypes.c_int, c_u64p, ctypes.c_int, ctypes.c_uint64, c_szp, c_szp],
            "mgc_compress": [vp, vp, ctypes.c_int, c_u64p, ctypes.c_int, ctypes.c_double,
                             ctypes.c_int, ctypes.c_int, ctypes.c_uint64, vp, ctypes.c_size_t,
                             vp, ctypes.c_size_t, vp, vp],
            "mgc_compress_blocking": [vp, vp, ctypes.c_int, c_u64p, ctypes.c_int,
                                      ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                      ctypes.c_uint64, vp, ctypes.c_size_t, vp, ctypes.c_size_t,
                                      vp, c_u64p],
            "mgc_compress_noalloc": [vp, vp, ctypes.c_int, c_u64p, ctypes.c_int,
                                     ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                     ctypes.c_uint64, vp, ctypes.c_size_t, vp, vp],
            "mgc_header_info": [vp, ctypes.c_size_t, ctypes.POINTER(ctypes.c_int), c_u64p,
                                ctypes.POINTER(ctypes.c_int), c_u64p, c_szp],
            "mgc_decompress": [vp, vp, ctypes.c_size_t, vp, ctypes.c_size_t, vp, ctypes.c_size_t, vp],
            "mgc_transform_query": [ctypes.c_int, c_u64p, c_szp],
            "mgc_decompose": [vp, vp, ctypes.c_int, c_u64p, ctypes.c_int, vp, vp, ctypes.c_size_t, vp],
            "mgc_recompose": [vp, vp, ctypes.c_int, c_u64p, ctypes.c_int, vp, vp, ctypes.c_size_t, vp],
            "mgc_adjoint_query": [ctypes.c_int, c_u64p, c_szp],
            "mgc_recompose_adjoint": [vp, vp, ctypes.c_int, c_u64p, vp, vp, ctypes.c_size_t, vp],
            "mgc_levels_query": [ctypes.c_int, c_u64p, c_szp],
            "mgc_recompose_levels": [vp, vp, ctypes.c_int, c_u64p, ctypes.c_int, vp, vp,
                                     ctypes.c_size_t, vp, ctypes.c_size_t, vp],
            "mgc_huffman_query": [ctypes.c_uint64, ctypes.c_uint32, c_szp, c_szp],
            "mgc_huffman_encode": [vp, vp, ctypes.c_uint64, ctypes.c_uint32, vp, ctypes.c_size_t,
                                   vp, ctypes.c_size_t, vp, c_u64p],
            "mgc_huffman_decode": [vp, vp, ctypes.c_size_t, vp, ctypes.c_uint64, vp,
                                   ctypes.c_size_t, vp],
            "mgc_pipe_max_bytes": [ctypes.c_int, c_u64p, ctypes.c_int,
                                   ctypes.POINTER(PipeModel), c_szp],
            "mgc_pipe_compress": [vp, vp, ctypes.c_int, c_u64p, ctypes.c_int, ctypes.c_double,
                                  ctypes.c_int, ctypes.c_int, ctypes.POINTER(PipeModel), vp,
                                  ctypes.c_size_t, c_u64p, ctypes.POINTER(PipeStats)],
            "mgc_pipe_decompress": [vp, vp, ctypes.c_size_t, vp, ctypes.c_size_t,
                                    ctypes.POINTER(PipeStats)],
            "mgc_pipe_info": [vp, ctypes.c_size_t, ctypes.POINTER(ctypes.c_int), c_u64p,
                              ctypes.POINTER(ctypes.c_int), c_u64p, c_u64p],
            "mgc_pipe_profile": [vp, vp, ctypes.c_int, c_u64p, ctypes.c_int, ctypes.c_double,
                                 ctypes.c_int, ctypes.c_int, ctypes.POINTER(PipeModel)],
            "mgc_zfp_query": [ctypes.c_int, c_u64p, ctypes.c_int, ctypes.c_double, c_szp],
            "mgc_zfp_compress": [vp, vp, ctypes.c_int, c_u64p, ctypes.c_int, ctypes.c_double, vp,
                                 ctypes.c_size_t, vp, vp],
            "mgc_zfp_parse_header": [vp, ctypes.c_size_t, ctypes.POINTER(ctypes.c_int), c_u64p,
                                     ctypes.POINTER(ctypes.c_int),
                                     ctypes.POINTER(ctypes.c_double), c_u64p],
            "mgc_zfp_decompress": [vp, vp, ctypes.c_size_t, vp, ctypes.c_size_t, vp],
            "mgc_hx_query": [ctypes.c_uint64, ctypes.c_int, ctypes.c_uint32, c_szp, c_szp],
            "mgc_hx_compress": [vp, vp, ctypes.c_uint64, ctypes.c_int, ctypes.c_uint32,
                                ctypes.c_int64, ctypes.c_uint32, vp, ctypes.c_size_t, vp,
                                ctypes.c_size_t, vp, vp],
            "mgc_hx_parse_header": [vp, ctypes.c_size_t, ctypes.POINTER(ctypes.c_int), c_u64p,
                                    ctypes.POINTER(ctypes.c_uint32),
                                    ctypes.POINTER(ctypes.c_int64),
                                    ctypes.POINTER(ctypes.c_uint32), c_u64p],
            "mgc_hx_decompress": [vp, vp, ctypes.c_size_t, vp, ctypes.c_uint64, ctypes.c_int, vp,
                                  ctypes.c_size_t, vp],
            "mgc_batch_query": [ctypes.c_int, ctypes.POINTER(ctypes.c_int), c_u64p,
                                ctypes.POINTER(ctypes.c_int), ctypes.c_uint64, c_szp, c_szp,
                                c_u64p],
            "mgc_compress_batched": [vp, ctypes.c_int, ctypes.POINTER(vp),
                                     ctypes.POINTER(ctypes.c_int), c_u64p,
                                     ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double),
                                     ctypes.c_int, ctypes.c_int, ctypes.c_uint64, vp,
                                     ctypes.c_size_t, vp, ctypes.c_size_t, vp, vp, ctypes.c_int,
                                     vp],
            "mgc_set_tuning": [vp, ctypes.c_int, ctypes.c_int],
            "mgc_tuning_info": [vp, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                ctypes.POINTER(ctypes.c_int)],
            "mgc_set_decoder": [vp, ctypes.c_int, ctypes.c_int],
            "mgc_decoder_info": [vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)],
            "mgc_profile_enable": [vp, ctypes.c_int],
            "mgc_profile_reset": [vp],
            "mgc_profile_read": [vp, ctypes.c_char_p, ctypes.c_size_t, c_u64p,
                                 ctypes.POINTER(ctypes.c_double), ctypes.c_int,
                                 ctypes.POINTER(ctypes.c_int)],
        }
        for name, args in sig.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int
        lib.mgc_last_error.restype = ctypes.c_char_p
        lib.mgc_last_error.argtypes = []
        lib.mgc_version.restype = ctypes.c_int
        _lib = lib
        return lib


def _check(st: int):
    if st != 0:
        msg = _load().mgc_last_error()
        raise MgcError(st, msg.decode() if msg else "")


def _ctx(device: int):
    lib = _load()
    with _lock:
        h = _ctxs.get(device)
        if h is None:
            h = ctypes.c_void_p()
            _check(lib.mgc_create(device, ctypes.byref(h)))
            _ctxs[device] = h
        return h


def _torch():
    import torch
    return torch


def _stream_ptr(device):
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _shape_arg(shape):
    arr = (ctypes.c_uint64 * max(len(shape), 1))(*[int(s) for s in shape])
    return arr


def _dtype_code(dt) -> int:
    torch = _torch()
    if dt == torch.float32:
        return 0
    if dt == torch.float64:
        return 1
    raise TypeError("only float32 and float64 tensors are supported")


def _require_gpu(t, what):
    if not t.is_cuda:
        raise ValueError("%s must be a GPU tensor (no CPU path exists)" % what)


def _empty(nbytes: int, device):
    torch = _torch()
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


def compress_query(shape, dtype, outlier_cap: int = 0):
    """(workspace bytes, output capacity) of compress for this shape and dtype.

    The library builds the level plan to answer (≈0.1 ms at 513^3), so the
    answers are kept per (shape, dtype, capacity)."""
    key = (tuple(int(s) for s in shape), _dtype_code(dtype), int(outlier_cap))
    hit = _query_cache.get(key)
    if hit is None:
        ws = ctypes.c_size_t()
        mx = ctypes.c_size_t()
        _check(_load().mgc_compress_query(len(key[0]), _shape_arg(key[0]), key[1], key[2],
                                          ctypes.byref(ws), ctypes.byref(mx)))
        hit = _query_cache[key] = (ws.value, mx.value)
    return hit


_query_cache = {}


_DEVICE_MESSAGES = {1: "input holds NaN or Inf",
                    3: "more escaped values than the outlier capacity",
                    5: "device-side consistency check failed",
                    6: "error bound below the resolution of the data or the output type"}


def compress_async(x, error_bound: float, norm: str = "linf", mode: str = "rel",
                   outlier_cap: int = 0, workspace=None, out=None, result=None):
    """Enqueue a compression on the current stream without waiting for it.

    ``workspace`` and ``out`` are uint8 GPU tensors of at least the queried
    sizes (compress_query) and ``result`` an int64 GPU tensor of 2 entries;
    when the stream work is done, result[0] holds the status (0 = OK, else an
    MgcError code) and result[1] the stream length in bytes (or, for status
    3, the escaped values needed).  No host synchronisation takes place, so
    the call can be captured into a CUDA/HIP graph (after one call outside
    the capture has built the shape's plan).
    """
    _require_gpu(x, "input")
    if not x.is_contiguous():
        raise ValueError("input must be contiguous")
    dev = x.device.index if x.device.index is not None else _torch().cuda.current_device()
    shape = tuple(x.shape)
    ws_n, out_n = compress_query(shape, x.dtype, outlier_cap)
    torch = _torch()
    if workspace is None or out is None or result is None:
        raise ValueError("workspace, out and result tensors are required")
    if workspace.numel() < ws_n or out.numel() < out_n or result.numel() < 2 \
            or result.dtype != torch.int64:
        raise ValueError("buffers smaller than the queried sizes")
    _check(_load().mgc_compress(_ctx(dev), ctypes.c_void_p(x.data_ptr()), len(shape),
                                _shape_arg(shape), _dtype_code(x.dtype), float(error_bound),
                                _NORM[norm], _MODE[mode], outlier_cap,
                                ctypes.c_void_p(out.data_ptr()), out.numel(),
                                ctypes.c_void_p(workspace.data_ptr()), workspace.numel(),
                                ctypes.c_void_p(result.data_ptr()), _stream_ptr(dev)))


NOALLOC_SCRATCH_BYTES = 64 << 20


def compress_noalloc(x, error_bound: float, out, result, norm: str = "linf",
                     mode: str = "rel", outlier_cap: int = 0):
    """Enqueue a compression that allocates no device memory.

    The library keeps the work buffers and plan tables in a device array of
    NOALLOC_SCRATCH_BYTES per device; ``out`` (uint8, at least the queried
    output capacity) and ``result`` (int64, 2 entries: status and stream
    length, as in compress_async) are the caller's.  Larger arrays raise
    MgcError (code 3).  Calls that overlap on one device share the scratch
    and must be ordered by the caller.
    """
    _require_gpu(x, "input")
    if not x.is_contiguous():
        raise ValueError("input must be contiguous")
    torch = _torch()
    dev = x.device.index if x.device.index is not None else torch.cuda.current_device()
    shape = tuple(x.shape)
    if result.numel() < 2 or result.dtype != torch.int64 or not result.is_cuda:
        raise ValueError("result must be an int64 GPU tensor of 2 entries")
    _check(_load().mgc_compress_noalloc(_ctx(dev), ctypes.c_void_p(x.data_ptr()), len(shape),
                                        _shape_arg(shape), _dtype_code(x.dtype),
                                        float(error_bound), _NORM[norm], _MODE[mode],
                                        outlier_cap, ctypes.c_void_p(out.data_ptr()),
                                        out.numel(), ctypes.c_void_p(result.data_ptr()),
                                        _stream_ptr(dev)))


def compress(x, error_bound: float, norm: str = "linf", mode: str = "rel",
             outlier_cap: int = 0, workspace=None, out=None):
    """Compress a 1-3D float32/float64 GPU tensor; returns a uint8 GPU tensor.

    The reconstruction error is at most ``error_bound`` in the chosen norm
    (relative to max-min for L-inf or to ||x||_2 for L2 when mode="rel").
    ``workspace``/``out`` may be preallocated uint8 tensors of the queried
    sizes; the returned tensor is a view into ``out``.  Waits for the
    stream length (one read of two device words).
    """
    _require_gpu(x, "input")
    x = x.contiguous()
    torch = _torch()
    shape = tuple(x.shape)
    result = torch.empty(2, dtype=torch.int64, device=x.device)
    for _ in range(2):
        ws_n, out_n = compress_query(shape, x.dtype, outlier_cap)
        ws = workspace if workspace is not None and workspace.numel() >= ws_n else _empty(ws_n, x.device)
        ob = out if out is not None and out.numel() >= out_n else _empty(out_n, x.device)
        compress_async(x, error_bound, norm, mode, outlier_cap, ws, ob, result)
        st, size = (int(v) for v in result.cpu().tolist())
        if st == 3 and size > outlier_cap:
            outlier_cap = size   # more escaped values than room: retry once
            continue
        if st != 0:
            raise MgcError(st, _DEVICE_MESSAGES.get(st, "device status %d" % st))
        return ob[:size]
    raise MgcError(st, _DEVICE_MESSAGES.get(st, "device status %d" % st))


BATCH_EAGER = 1
BATCH_NO_TUNE = 2
TUNE_KINDS = {"dec_f32": 0, "dec_f64": 1, "thomas_strided": 2, "thomas_rows": 3}


def _batch_desc(shapes, dtypes):
    n = len(shapes)
    ndims = (ctypes.c_int * n)(*[len(s) for s in shapes])
    flat = []
    for s in shapes:
        if not 1 <= len(s) <= 3:
            raise ValueError("arrays of 1 to 3 axes")
        flat += [int(v) for v in s] + [0] * (3 - len(s))
    shp = (ctypes.c_uint64 * (3 * n))(*flat)
    dts = (ctypes.c_int * n)(*[_dtype_code(d) for d in dtypes])
    return n, ndims, shp, dts


def batch_query(shapes, dtypes, outlier_cap: int = 0):
    """(workspace bytes, output bytes, per-array output offsets) of a batch."""
    n, ndims, shp, dts = _batch_desc(shapes, dtypes)
    ws = ctypes.c_size_t()
    ob = ctypes.c_size_t()
    offs = (ctypes.c_uint64 * n)()
    _check(_load().mgc_batch_query(n, ndims, shp, dts, outlier_cap, ctypes.byref(ws),
                                   ctypes.byref(ob), offs))
    return ws.value, ob.value, [int(v) for v in offs]


class Batch:
    """Buffers of a batched compression of fixed shapes and dtypes.

    ``run`` enqueues the compression of one list of tensors (asynchronous);
    ``streams`` waits for it and returns one uint8 GPU tensor per array (views
    into the shared output buffer; an array whose escaped values overflowed
    the capacity is compressed again alone with the capacity it needs).
    """

    def __init__(self, shapes, dtypes, outlier_cap: int = 0, device=None):
        torch = _torch()
        self.shapes = [tuple(int(v) for v in s) for s in shapes]
        self.dtypes = list(dtypes)
        self.outlier_cap = int(outlier_cap)
        self.device = torch.device("cuda", device if device is not None else torch.cuda.current_device())
        self.ws_bytes, self.out_bytes, self.offsets = batch_query(self.shapes, self.dtypes,
                                                                  self.outlier_cap)
        n = len(self.shapes)
        self.workspace = _empty(self.ws_bytes, self.device)
        self.out = _empty(self.out_bytes, self.device)
        self.sizes = torch.zeros(n, dtype=torch.int64, device=self.device)
        self.status = torch.zeros(n, dtype=torch.int32, device=self.device)
        self._desc = _batch_desc(self.shapes, self.dtypes)
        self._last = None

    def run(self, tensors, bounds, norm: str = "linf", mode: str = "rel", flags: int = 0):
        n, ndims, shp, dts = self._desc
        if len(tensors) != n or len(bounds) != n:
            raise ValueError("one tensor and one bound per array")
        for j, t in enumerate(tensors):
            _require_gpu(t, "input %d" % j)
            if tuple(t.shape) != self.shapes[j] or t.dtype != self.dtypes[j] or not t.is_contiguous():
                raise ValueError("input %d does not match the batch description" % j)
        ptrs = (ctypes.c_void_p * n)(*[t.data_ptr() for t in tensors])
        bnd = (ctypes.c_double * n)(*[float(b) for b in bounds])
        dev = self.device.index
        _check(_load().mgc_compress_batched(
            _ctx(dev), n, ptrs, ndims, shp, dts, bnd, _NORM[norm], _MODE[mode], self.outlier_cap,
            ctypes.c_void_p(self.out.data_ptr()), self.out.numel(),
            ctypes.c_void_p(self.workspace.data_ptr()), self.workspace.numel(),
            ctypes.c_void_p(self.sizes.data_ptr()), ctypes.c_void_p(self.status.data_ptr()),
            int(flags), _stream_ptr(dev)))
        self._last = (list(tensors), list(bounds), norm, mode)

    def streams(self):
        if self._last is None:
            raise RuntimeError("run() has not been called")
        sizes = self.sizes.cpu().tolist()
        status = self.status.cpu().tolist()
        tensors, bounds, norm, mode = self._last
        res = []
        for j, (st, sz) in enumerate(zip(status, sizes)):
            if st == 3:   # escaped values overflowed: this array alone, with the room it needs
                res.append(compress(tensors[j], bounds[j], norm, mode, outlier_cap=int(sz)))
            elif st != 0:
                raise MgcError(st, "array %d of the batch" % j)
            else:
                res.append(self.out[self.offsets[j]: self.offsets[j] + sz])
        return res


def compress_batched(tensors, bounds, norm: str = "linf", mode: str = "rel",
                     outlier_cap: int = 0, flags: int = 0):
    """Compress a list of GPU tensors (uneven shapes, per-array bounds) in one
    batched call; returns one uint8 GPU tensor per array."""
    tensors = [t.contiguous() for t in tensors]
    b = Batch([t.shape for t in tensors], [t.dtype for t in tensors], outlier_cap,
              device=tensors[0].device.index)
    b.run(tensors, bounds, norm, mode, flags)
    return b.streams()


def set_tuning(kind: str, candidate: int, device=None):
    """Force candidate ``candidate`` of a tuning kind for later batched calls
    (-1: autotune)."""
    torch = _torch()
    dev = device if device is not None else torch.cuda.current_device()
    _check(_load().mgc_set_tuning(_ctx(dev), TUNE_KINDS[kind], int(candidate)))


def tuning_info(kind: str, device=None):
    """(number of candidates, candidate used by the latest batched call)."""
    torch = _torch()
    dev = device if device is not None else torch.cuda.current_device()
    n = ctypes.c_int()
    last = ctypes.c_int()
    _check(_load().mgc_tuning_info(_ctx(dev), TUNE_KINDS[kind], ctypes.byref(n),
                                   ctypes.byref(last)))
    return n.value, last.value


def set_decoder(ring: int = 0, waves: int = 0, device=None):
    """Force the decoder's ring (1: 64-byte pieces, 2: 32-byte, 3: 16-byte;
    0 = automatic) and wavefronts per block (1..16, 0 = automatic)."""
    torch = _torch()
    dev = device if device is not None else torch.cuda.current_device()
    _check(_load().mgc_set_decoder(_ctx(dev), int(ring), int(waves)))


def decoder_info(device=None):
    """(ring, wavefronts per block) used by the latest decode."""
    torch = _torch()
    dev = device if device is not None else torch.cuda.current_device()
    ring = ctypes.c_int()
    waves = ctypes.c_int()
    _check(_load().mgc_decoder_info(_ctx(dev), ctypes.byref(ring), ctypes.byref(waves)))
    return ring.value, waves.value


def header_info(stream):
    """Shape, dtype and sizes of a compressed stream (reads its header)."""
    import numpy as np
    n = min(int(stream.numel()), HEADER_PREFIX)
    host = stream[:n].cpu().numpy() if stream.is_cuda else np.asarray(stream[:n])
    buf = np.ascontiguousarray(host, dtype=np.uint8)
    ndim = ctypes.c_int()
    shp = (ctypes.c_uint64 * 3)()
    dt = ctypes.c_int()
    total = ctypes.c_uint64()
    ws = ctypes.c_size_t()
    _check(_load().mgc_header_info(buf.ctypes.data_as(ctypes.c_void_p), n, ctypes.byref(ndim), shp,
                                   ctypes.byref(dt), ctypes.byref(total), ctypes.byref(ws)))
    torch = _torch()
    return {"shape": tuple(int(shp[i]) for i in range(ndim.value)),
            "dtype": torch.float32 if dt.value == 0 else torch.float64,
            "stream_bytes": int(total.value), "workspace_bytes": int(ws.value)}


def decompress(stream, workspace=None, out=None, info=None):
    """Reconstruct the array held in a compressed GPU stream.

    ``info`` may pass a header_info() result for this stream's shape to skip
    reading the header from the device here (the library reads it anyway).
    """
    _require_gpu(stream, "stream")
    torch = _torch()
    dev = stream.device.index if stream.device.index is not None else torch.cuda.current_device()
    info = info or header_info(stream)
    res = out if out is not None else torch.empty(info["shape"], dtype=info["dtype"], device=stream.device)
    ws = workspace if workspace is not None and workspace.numel() >= info["workspace_bytes"] \
        else _empty(info["workspace_bytes"], stream.device)
    stream = stream.contiguous()
    _check(_load().mgc_decompress(_ctx(dev), ctypes.c_void_p(stream.data_ptr()), stream.numel(),
                                  ctypes.c_void_p(res.data_ptr()), res.numel() * res.element_size(),
                                  ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream_ptr(dev)))
    return res


def transform_query(shape) -> int:
    ws = ctypes.c_size_t()
    _check(_load().mgc_transform_query(len(shape), _shape_arg(shape), ctypes.byref(ws)))
    return ws.value


def decompose(x, workspace=None):
    """Multilevel coefficients (FP64, stream order) of a 1-3D GPU tensor."""
    _require_gpu(x, "input")
    torch = _torch()
    x = x.contiguous()
    dev = x.device.index if x.device.index is not None else torch.cuda.current_device()
    shape = tuple(x.shape)
    ws_n = transform_query(shape)
    ws = workspace if workspace is not None and workspace.numel() >= ws_n else _empty(ws_n, x.device)
    out = torch.empty(x.numel(), dtype=torch.float64, device=x.device)
    _check(_load().mgc_decompose(_ctx(dev), ctypes.c_void_p(x.data_ptr()), len(shape),
                                 _shape_arg(shape), _dtype_code(x.dtype),
                                 ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(ws.data_ptr()),
                                 ws.numel(), _stream_ptr(dev)))
    return out


def recompose(coeffs, shape, dtype=None, workspace=None):
    """Inverse of decompose: nodal values of ``shape`` from FP64 coefficients."""
    _require_gpu(coeffs, "coefficients")
    torch = _torch()
    dtype = dtype or torch.float64
    coeffs = coeffs.contiguous()
    if coeffs.dtype != torch.float64:
        raise TypeError("coefficients must be float64")
    dev = coeffs.device.index if coeffs.device.index is not None else torch.cuda.current_device()
    shape = tuple(int(s) for s in shape)
    ws_n = transform_query(shape)
    ws = workspace if workspace is not None and workspace.numel() >= ws_n else _empty(ws_n, coeffs.device)
    out = torch.empty(shape, dtype=dtype, device=coeffs.device)
    _check(_load().mgc_recompose(_ctx(dev), ctypes.c_void_p(coeffs.data_ptr()), len(shape),
                                 _shape_arg(shape), _dtype_code(dtype),
                                 ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(ws.data_ptr()),
                                 ws.numel(), _stream_ptr(dev)))
    return out


def recompose_adjoint(grad_u, workspace=None):
    """R^T grad_u: gradient with respect to the multilevel coefficients (FP64,
    stream order) of a quantity whose gradient on the grid is ``grad_u``."""
    _require_gpu(grad_u, "gradient")
    torch = _torch()
    g = grad_u.contiguous().to(torch.float64)
    dev = g.device.index if g.device.index is not None else torch.cuda.current_device()
    shape = tuple(g.shape)
    ws_n = ctypes.c_size_t()
    _check(_load().mgc_adjoint_query(len(shape), _shape_arg(shape), ctypes.byref(ws_n)))
    ws = workspace if workspace is not None and workspace.numel() >= ws_n.value \
        else _empty(ws_n.value, g.device)
    out = torch.empty(g.numel(), dtype=torch.float64, device=g.device)
    _check(_load().mgc_recompose_adjoint(_ctx(dev), ctypes.c_void_p(g.data_ptr()), len(shape),
                                         _shape_arg(shape), ctypes.c_void_p(out.data_ptr()),
                                         ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                         _stream_ptr(dev)))
    return out


def recompose_levels(coeffs, shape, dtype=None):
    """recompose() that also returns every coarse level's grid G_0..G_{L-1}
    (FP64) as one flat tensor, level after level (per-level checkpoints)."""
    _require_gpu(coeffs, "coefficients")
    torch = _torch()
    dtype = dtype or torch.float64
    coeffs = coeffs.contiguous()
    dev = coeffs.device.index if coeffs.device.index is not None else torch.cuda.current_device()
    shape = tuple(int(x) for x in shape)
    lv = ctypes.c_size_t()
    _check(_load().mgc_levels_query(len(shape), _shape_arg(shape), ctypes.byref(lv)))
    levels = torch.empty(lv.value // 8, dtype=torch.float64, device=coeffs.device)
    ws = _empty(transform_query(shape), coeffs.device)
    out = torch.empty(shape, dtype=dtype, device=coeffs.device)
    _check(_load().mgc_recompose_levels(_ctx(dev), ctypes.c_void_p(coeffs.data_ptr()), len(shape),
                                        _shape_arg(shape), _dtype_code(dtype),
                                        ctypes.c_void_p(out.data_ptr()),
                                        ctypes.c_void_p(levels.data_ptr()), levels.numel() * 8,
                                        ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                        _stream_ptr(dev)))
    return out, levels


def _autograd_function():
    torch = _torch()

    class Recompose(torch.autograd.Function):
        """u = R c with the GPU recomposition; backward applies the GPU adjoint.

        ``Recompose.apply(coeffs, shape, keep_levels)``: coeffs is the FP64
        coefficient vector in stream order.  With keep_levels the forward pass
        also stores the coarse levels' grids (checkpoints), available as
        ``ctx.levels`` during backward; recomposition being linear, the
        gradient does not need them.  Quantisation, if the coefficients came
        from a compressed stream, is treated as the identity (straight-through).
        """

        @staticmethod
        def forward(ctx, coeffs, shape, keep_levels=False):
            shape = tuple(int(x) for x in shape)
            ctx.shape = shape
            if keep_levels:
                u, levels = recompose_levels(coeffs.detach(), shape, torch.float64)
                ctx.save_for_backward(levels)
            else:
                u = recompose(coeffs.detach(), shape, torch.float64)
            return u

        @staticmethod
        def backward(ctx, grad_u):
            return recompose_adjoint(grad_u), None, None

    return Recompose


class _LazyRecompose:
    _cls = None

    def apply(self, *args):
        if _LazyRecompose._cls is None:
            _LazyRecompose._cls = _autograd_function()
        return _LazyRecompose._cls.apply(*args)


Recompose = _LazyRecompose()


def huffman_encode(symbols, C: int = 1024):
    """Huffman-code 16-bit symbols (an int16/uint16/int32 GPU tensor of values 0..65535)."""
    _require_gpu(symbols, "symbols")
    torch = _torch()
    if symbols.dtype == torch.int32 or symbols.dtype == torch.int64:
        symbols = symbols.to(torch.int32).to(torch.int16)
    symbols = symbols.contiguous()
    if symbols.element_size() != 2:
        raise TypeError("symbols must be 16-bit")
    dev = symbols.device.index if symbols.device.index is not None else torch.cuda.current_device()
    n = symbols.numel()
    ws_n = ctypes.c_size_t()
    out_n = ctypes.c_size_t()
    _check(_load().mgc_huffman_query(n, C, ctypes.byref(ws_n), ctypes.byref(out_n)))
    ws = _empty(ws_n.value, symbols.device)
    out = _empty(out_n.value, symbols.device)
    size = ctypes.c_uint64()
    _check(_load().mgc_huffman_encode(_ctx(dev), ctypes.c_void_p(symbols.data_ptr()), n, C,
                                      ctypes.c_void_p(out.data_ptr()), out.numel(),
                                      ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream_ptr(dev),
                                      ctypes.byref(size)))
    return out[: size.value]


def huffman_decode(stream, n: int):
    """Decode n symbols; returns an int16 GPU tensor holding the 16-bit patterns."""
    _require_gpu(stream, "stream")
    torch = _torch()
    dev = stream.device.index if stream.device.index is not None else torch.cuda.current_device()
    stream = stream.contiguous()
    ws_n = ctypes.c_size_t()
    _check(_load().mgc_huffman_query(n, 64, ctypes.byref(ws_n), None))
    ws = _empty(ws_n.value, stream.device)
    out = torch.empty(max(n, 1), dtype=torch.int16, device=stream.device)
    _check(_load().mgc_huffman_decode(_ctx(dev), ctypes.c_void_p(stream.data_ptr()), stream.numel(),
                                      ctypes.c_void_p(out.data_ptr()), n,
                                      ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream_ptr(dev)))
    return out[:n]


def _hx_types():
    torch = _torch()
    return {torch.uint8: 0, torch.uint16: 1, torch.int32: 2, torch.int64: 3}


def hx_query(n: int, dtype, C: int = 1024):
    """(workspace bytes, largest stream bytes) of the Huffman-X codec."""
    t = _hx_types().get(dtype)
    if t is None:
        raise TypeError("Huffman-X streams hold uint8, uint16, int32 or int64 values")
    ws = ctypes.c_size_t()
    mx = ctypes.c_size_t()
    _check(_load().mgc_hx_query(n, t, C, ctypes.byref(ws), ctypes.byref(mx)))
    return ws.value, mx.value


def hx_compress(x, dict: int | None = None, base: int | None = None, C: int = 1024,
                workspace=None, out=None, result=None, sync: bool = True):
    """Lossless Huffman-X stream of a uint8/uint16/int32/int64 GPU tensor.

    Defaults: the full range for uint8 and uint16; 65536 keys with base
    -32767 for int32 and int64.  Returns the stream as a uint8 GPU tensor;
    with ``sync=False`` returns (output buffer, result) at once, result being
    the device words {status, stream bytes}.
    """
    _require_gpu(x, "x")
    torch = _torch()
    t = _hx_types().get(x.dtype)
    if t is None:
        raise TypeError("Huffman-X streams hold uint8, uint16, int32 or int64 values")
    x = x.contiguous().reshape(-1)
    if dict is None:
        dict = 256 if t == 0 else 65536
    if base is None:
        base = 0 if t < 2 else -(65536 // 2 - 1)
    dev = x.device.index if x.device.index is not None else torch.cuda.current_device()
    ws_n, out_n = hx_query(x.numel(), x.dtype, C)
    ws = workspace if workspace is not None else _empty(ws_n, x.device)
    o = out if out is not None else _empty(out_n, x.device)
    res = result if result is not None else torch.zeros(2, dtype=torch.int64, device=x.device)
    _check(_load().mgc_hx_compress(_ctx(dev), ctypes.c_void_p(x.data_ptr()), x.numel(), t, dict,
                                   base, C, ctypes.c_void_p(o.data_ptr()), o.numel(),
                                   ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                   ctypes.c_void_p(res.data_ptr()), _stream_ptr(dev)))
    if not sync:
        return o, res
    st, size = (int(v) for v in res.cpu())
    if st:
        raise MgcError(st, "Huffman-X compression failed on the device")
    return o[:size]


def hx_header(stream):
    """(dtype, n, dict, base, C, total) of a Huffman-X stream."""
    head = stream[:64].cpu().numpy().tobytes()
    t = ctypes.c_int()
    n = ctypes.c_uint64()
    d = ctypes.c_uint32()
    b = ctypes.c_int64()
    C = ctypes.c_uint32()
    tot = ctypes.c_uint64()
    _check(_load().mgc_hx_parse_header(head, len(head), ctypes.byref(t), ctypes.byref(n),
                                       ctypes.byref(d), ctypes.byref(b), ctypes.byref(C),
                                       ctypes.byref(tot)))
    dtype = {v: k for k, v in _hx_types().items()}[t.value]
    return dtype, n.value, d.value, b.value, C.value, tot.value


def hx_decompress(stream, workspace=None, out=None):
    """Values of a Huffman-X stream (uint8 GPU tensor) as a GPU tensor."""
    _require_gpu(stream, "stream")
    torch = _torch()
    stream = stream.contiguous()
    dev = stream.device.index if stream.device.index is not None else torch.cuda.current_device()
    dtype, n, _, _, C, _ = hx_header(stream)
    ws_n, _ = hx_query(n, dtype, C)
    ws = workspace if workspace is not None else _empty(ws_n, stream.device)
    y = out if out is not None else torch.empty(max(n, 1), dtype=dtype, device=stream.device)
    _check(_load().mgc_hx_decompress(_ctx(dev), ctypes.c_void_p(stream.data_ptr()),
                                     stream.numel(), ctypes.c_void_p(y.data_ptr()), n,
                                     _hx_types()[dtype], ctypes.c_void_p(ws.data_ptr()),
                                     ws.numel(), _stream_ptr(dev)))
    return y[:n]


def zfp_query(shape, dtype, rate: float) -> int:
    """Exact stream bytes of a fixed-rate block-coded array."""
    shp = _shape_arg(shape)
    out = ctypes.c_size_t()
    _check(_load().mgc_zfp_query(len(shape), shp, _dtype_code(dtype), rate, ctypes.byref(out)))
    return out.value


def zfp_compress(x, rate: float, out=None, result=None, sync: bool = True):
    """Fixed-rate block transform coding of an FP32/FP64 GPU tensor (1 to 3
    axes) at ``rate`` bits per value; returns the stream (uint8 GPU tensor),
    or (buffer, result words) with ``sync=False``."""
    _require_gpu(x, "x")
    torch = _torch()
    x = x.contiguous()
    dev = x.device.index if x.device.index is not None else torch.cuda.current_device()
    shp = _shape_arg(tuple(x.shape))
    n = zfp_query(tuple(x.shape), x.dtype, rate)
    o = out if out is not None else _empty(n, x.device)
    res = result if result is not None else torch.zeros(2, dtype=torch.int64, device=x.device)
    _check(_load().mgc_zfp_compress(_ctx(dev), ctypes.c_void_p(x.data_ptr()), x.dim(), shp,
                                    _dtype_code(x.dtype), rate, ctypes.c_void_p(o.data_ptr()),
                                    o.numel(), ctypes.c_void_p(res.data_ptr()), _stream_ptr(dev)))
    if not sync:
        return o, res
    st, size = (int(v) for v in res.cpu())
    if st:
        raise MgcError(st, "fixed-rate coding failed: the data holds NaN or Inf")
    return o[:size]


def zfp_decompress(stream, out=None):
    """Array of a fixed-rate block-coded stream (uint8 GPU tensor)."""
    _require_gpu(stream, "stream")
    torch = _torch()
    stream = stream.contiguous()
    dev = stream.device.index if stream.device.index is not None else torch.cuda.current_device()
    head = stream[:64].cpu().numpy().tobytes()
    nd = ctypes.c_int()
    shp = (ctypes.c_uint64 * 3)()
    dt = ctypes.c_int()
    rate = ctypes.c_double()
    _check(_load().mgc_zfp_parse_header(head, len(head), ctypes.byref(nd), shp, ctypes.byref(dt),
                                        ctypes.byref(rate), None))
    shape = tuple(int(shp[d]) for d in range(nd.value))
    dtype = torch.float32 if dt.value == 0 else torch.float64
    y = out if out is not None else torch.empty(shape, dtype=dtype, device=stream.device)
    _check(_load().mgc_zfp_decompress(_ctx(dev), ctypes.c_void_p(stream.data_ptr()),
                                      stream.numel(), ctypes.c_void_p(y.data_ptr()),
                                      y.numel() * y.element_size(), _stream_ptr(dev)))
    return y


def _pipe_model(model):
    m = PipeModel()
    if model:
        for k, v in dict(model).items():
            setattr(m, k, v)
    return m


def _require_host(t, what):
    if t.device.type != "cpu":
        raise ValueError("%s must be a host (CPU) tensor" % what)


def pipe_max_bytes(shape, dtype, model=None) -> int:
    shp = _shape_arg(shape)
    out = ctypes.c_size_t()
    m = _pipe_model(model)
    _check(_load().mgc_pipe_max_bytes(len(shape), shp, _dtype_code(dtype), ctypes.byref(m),
                                      ctypes.byref(out)))
    return out.value


def pipe_compress(x, error_bound: float, norm: str = "linf", mode: str = "rel", model=None,
                  out=None, device: int = 0):
    """Compress a host (CPU, preferably pinned) FP32/FP64 tensor through the
    chunked host-device pipeline.  Returns (container as a uint8 CPU tensor,
    stats dict)."""
    torch = _torch()
    _require_host(x, "x")
    x = x.contiguous()
    shp = _shape_arg(tuple(x.shape))
    m = _pipe_model(model)
    if out is None:
        out = torch.empty(pipe_max_bytes(tuple(x.shape), x.dtype, model), dtype=torch.uint8,
                          pin_memory=True)
    size = ctypes.c_uint64()
    st = PipeStats()
    _check(_load().mgc_pipe_compress(_ctx(device), ctypes.c_void_p(x.data_ptr()), x.dim(), shp,
                                     _dtype_code(x.dtype), error_bound, _NORM[norm], _MODE[mode],
                                     ctypes.byref(m), ctypes.c_void_p(out.data_ptr()), out.numel(),
                                     ctypes.byref(size), ctypes.byref(st)))
    return out[: size.value], st.as_dict()


def pipe_decompress(container, out=None, device: int = 0):
    """Array of a pipeline container (uint8 CPU tensor) as a CPU tensor.
    Returns (array, stats dict)."""
    torch = _torch()
    _require_host(container, "container")
    container = container.contiguous()
    nd = ctypes.c_int()
    shp = (ctypes.c_uint64 * 3)()
    dt = ctypes.c_int()
    _check(_load().mgc_pipe_info(ctypes.c_void_p(container.data_ptr()), container.numel(),
                                 ctypes.byref(nd), shp, ctypes.byref(dt), None, None))
    shape = tuple(int(shp[d]) for d in range(nd.value))
    dtype = torch.float32 if dt.value == 0 else torch.float64
    if out is None:
        out = torch.empty(shape, dtype=dtype, pin_memory=True)
    st = PipeStats()
    _check(_load().mgc_pipe_decompress(_ctx(device), ctypes.c_void_p(container.data_ptr()),
                                       container.numel(), ctypes.c_void_p(out.data_ptr()),
                                       out.numel() * out.element_size(), ctypes.byref(st)))
    return out, st.as_dict()


def pipe_profile(x, error_bound: float, norm: str = "linf", mode: str = "rel", model=None,
                 device: int = 0):
    """Fit the pipeline's throughput models on a host tensor; returns the
    model dict for pipe_compress."""
    _require_host(x, "x")
    x = x.contiguous()
    shp = _shape_arg(tuple(x.shape))
    m = _pipe_model(model)
    _check(_load().mgc_pipe_profile(_ctx(device), ctypes.c_void_p(x.data_ptr()), x.dim(), shp,
                                    _dtype_code(x.dtype), error_bound, _NORM[norm], _MODE[mode],
                                    ctypes.byref(m)))
    return m.as_dict()


def profile_enable(flag: bool = True, device: int = 0):
    _check(_load().mgc_profile_enable(_ctx(device), 1 if flag else 0))


def profile_reset(device: int = 0):
    _check(_load().mgc_profile_reset(_ctx(device)))


def profile_read(device: int = 0):
    """{stage: (launches, total GPU ms)} accumulated since the last reset."""
    lib = _load()
    cap = 64
    names = ctypes.create_string_buffer(8192)
    counts = (ctypes.c_uint64 * cap)()
    ms = (ctypes.c_double * cap)()
    n = ctypes.c_int()
    _check(lib.mgc_profile_read(_ctx(device), names, 8192, counts, ms, cap, ctypes.byref(n)))
    keys = names.value.decode().split("\n") if n.value else []
    return {k: (int(counts[i]), float(ms[i])) for i, k in enumerate(keys[:cap])}
