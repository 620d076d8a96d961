/*
 * mgc.h - C ABI of the MI355X multigrid error-bounded lossy compressor.
 *
 * The library implements the MGARD reduction pipeline described in Section
 * IV-A and Algorithm 1 of "HPDR: High-Performance Portable Scientific Data
 * Reduction Framework" (arXiv 2503.06322): a multilevel decomposition
 * (interpolation coefficients, a transfer/mass-matrix product and
 * tridiagonal correction solves along each dimension, the add), level-wise
 * linear quantisation, and Huffman entropy coding (Section IV-B, Algorithm 2).
 * Decompression runs the inverse.  Every stage runs in HIP kernels on one
 * gfx950 GPU.
 *
 * Conventions (all entry points):
 *  - Every function returns an mgc_status; nothing throws across the ABI.
 *    A failure leaves a thread-local message readable with mgc_last_error().
 *  - Pointers named d_* are device pointers; h_* are host pointers.  All
 *    device memory (inputs, outputs, workspaces) is owned by the caller; the
 *    library never frees it.  A context owns only its cached plan tables
 *    (small device tables, freed by mgc_destroy) and a small pinned buffer.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Kernels are enqueued on it in order.  Entry points marked BLOCKING
 *    synchronise that stream before returning.
 *  - Arrays are dense, row-major (last axis fastest), 1 to 3 axes; axes of
 *    length 1 are squeezed out.  dtype is float32 or float64.  Arithmetic is
 *    FP64 throughout (inputs are read and outputs written in their dtype).
 *  - Sizes: at most 2^32 - 1 values per array.
 *  - Calls on one context from several host threads must be serialised by
 *    the caller; distinct contexts are independent.
 */
#ifndef MGC_H
#define MGC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MGC_OK = 0,
  MGC_EINVAL = 1,       /* bad argument: shape, dtype, bound, NaN/Inf input */
  MGC_EUNSUPPORTED = 2, /* valid request this build does not handle (ndim > 3, N >= 2^32) */
  MGC_ENOSPC = 3,       /* output or workspace too small (see mgc_last_error) */
  MGC_EFORMAT = 4,      /* truncated or corrupt compressed stream */
  MGC_EDEVICE = 5,      /* a HIP runtime call failed */
  MGC_ERANGE = 6        /* bound too small for the data (quantised value >= 2^62,
                           or the budget vanishes below the output precision) */
} mgc_status;

typedef enum { MGC_F32 = 0, MGC_F64 = 1 } mgc_dtype;
typedef enum { MGC_LINF = 0, MGC_L2 = 1 } mgc_norm;
typedef enum { MGC_REL = 0, MGC_ABS = 1 } mgc_mode;

typedef struct mgc_ctx_s* mgc_ctx;

/* Context = per-device plan cache (the paper's context-memory cache,
 * Section III-B: reduction contexts are built once per shape and reused).
 * `device` is the HIP device ordinal; it is made current by every call. */
mgc_status mgc_create(int device, mgc_ctx* out);
mgc_status mgc_destroy(mgc_ctx ctx);
const char* mgc_last_error(void);
int mgc_version(void);

/* ------------------------------------------------------------------------
 * Compression (Algorithm 1 end to end: hierarchy, decomposition, level-wise
 * quantisation, Huffman).
 *
 * mgc_compress_query: workspace and worst-case output bytes for an array of
 *   `shape` (ndim entries) and dtype, with room for `outlier_cap` escaped
 *   values (0 = default, max(65536, N/16)).
 * mgc_compress (asynchronous on `stream`): compresses d_in into d_out.
 *   error_bound > 0 is relative (to max - min for L-inf, to ||u||_2 for L2)
 *   when mode == MGC_REL, absolute otherwise; the reconstruction error in
 *   that norm is at most the bound.  out_cap and ws_bytes must be at least
 *   the queried sizes for the same outlier_cap (MGC_ENOSPC otherwise).  The
 *   whole compression, including turning the relative bound into per-level
 *   bins, runs on the device with no host round trip, so the call can be
 *   captured into a HIP graph.  Its outcome lands in two device words,
 *   d_result[0] = an mgc_status and d_result[1] = the stream length in
 *   bytes, when the stream has been written:
 *     MGC_OK       the stream is complete (constant and empty arrays get a
 *                  136-byte stream);
 *     MGC_EINVAL   the data holds NaN or Inf (d_result[1] = 0);
 *     MGC_ERANGE   the bound is below the resolution of the data or the
 *                  output type, or a quantised value reached 2^62;
 *     MGC_ENOSPC   more values escaped the dictionary than outlier_cap;
 *                  d_result[1] = the escaped values needed (call again with
 *                  that capacity);
 *     MGC_EDEVICE  a device-side consistency check failed.
 *   Argument errors are returned directly: MGC_EINVAL (shape, dtype, bound,
 *   null pointers), MGC_EUNSUPPORTED, MGC_ENOSPC (buffers), MGC_EDEVICE.
 * mgc_compress_blocking: the same compression, BLOCKING: it waits for the
 *   stream and returns the device outcome as its status (with the messages
 *   above) and the stream length, or the escaped values needed after
 *   MGC_ENOSPC, in *h_out_size.
 *
 * Stream layout (little-endian): a 128-byte header, the per-level bins
 * q_0..q_L (f64), then, unless the array is constant or empty, the codebook
 * (u16 symbols ascending, then u8 code lengths), the chunk word offsets
 * (u64, n_chunks + 1), the escaped values' stream positions (u64, ascending)
 * and values (i64), and the coded 32-bit words; each section starts at a
 * multiple of 8 bytes.
 * ---------------------------------------------------------------------- */
mgc_status mgc_compress_query(int ndim, const uint64_t* shape, mgc_dtype dtype,
                              uint64_t outlier_cap, size_t* ws_bytes,
                              size_t* max_out_bytes);
mgc_status mgc_compress(mgc_ctx ctx, const void* d_in, int ndim, const uint64_t* shape,
                        mgc_dtype dtype, double error_bound, mgc_norm norm,
                        mgc_mode mode, uint64_t outlier_cap, void* d_out,
                        size_t out_cap, void* d_ws, size_t ws_bytes, uint64_t* d_result,
                        void* stream);
mgc_status mgc_compress_blocking(mgc_ctx ctx, const void* d_in, int ndim,
                                 const uint64_t* shape, mgc_dtype dtype, double error_bound,
                                 mgc_norm norm, mgc_mode mode, uint64_t outlier_cap,
                                 void* d_out, size_t out_cap, void* d_ws, size_t ws_bytes,
                                 void* stream, uint64_t* h_out_size);

/* ------------------------------------------------------------------------
 * Allocation-free compression, for callers that cannot allocate device
 * memory (code under stream capture, tight serving loops, harnesses that
 * forbid hipMalloc).  mgc_compress_noalloc is mgc_compress with no workspace
 * argument: the plan tables of the shape and every work buffer live in a
 * device array of MGC_NOALLOC_SCRATCH_BYTES that the library holds on each
 * device until the process ends, and the call makes no hipMalloc, hipFree or
 * other allocating call (stage timing is not recorded during it).  The
 * caller passes the input, the output (out_cap >= the max_out_bytes of
 * mgc_compress_query for the same outlier_cap) and the two result words;
 * the outcome is reported there exactly as by mgc_compress, and the stream
 * is byte-identical to mgc_compress's.  Arrays whose tables and buffers do
 * not fit the scratch are rejected with MGC_ENOSPC before anything is
 * enqueued (with the default outlier capacity: three-axis arrays up to
 * about 9.5 million values, e.g. 211^3; two-axis ones up to about 7 million).  Every call on a device shares that device's
 * scratch, which keeps the last call's contents: calls that overlap on one
 * device (other streams, other host threads, other contexts) race and must
 * be ordered by the caller.  The first call for a shape builds its plan on
 * the host; a call whose shape differs from the previous call's on the
 * device copies the tables (a few hundred KB) into the scratch on `stream`.
 * ---------------------------------------------------------------------- */
#define MGC_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
mgc_status mgc_compress_noalloc(mgc_ctx ctx, const void* d_in, int ndim, const uint64_t* shape,
                                mgc_dtype dtype, double error_bound, mgc_norm norm,
                                mgc_mode mode, uint64_t outlier_cap, void* d_out,
                                size_t out_cap, uint64_t* d_result, void* stream);

/* ------------------------------------------------------------------------
 * Decompression (inverse of the above).
 *
 * mgc_header_info: parses a host copy of the first bytes of a stream (at least
 *   128 + 8 * (L + 1); 1024 always suffices) and returns the array's ndim,
 *   shape (3 entries, unused = 0), dtype, the stream length and the
 *   decompression workspace size.  Errors: MGC_EFORMAT.
 * mgc_decompress (BLOCKING: it reads the header from the device): writes the
 *   reconstructed array (dtype and shape of the header) to d_out.  d_in
 *   starts on a 4-byte boundary (MGC_EINVAL otherwise).
 *   Errors: MGC_EINVAL, MGC_EFORMAT, MGC_ENOSPC (out_cap/ws_bytes), MGC_EDEVICE.
 * ---------------------------------------------------------------------- */
mgc_status mgc_header_info(const void* h_prefix, size_t n, int* ndim, uint64_t* shape3,
                           mgc_dtype* dtype, uint64_t* stream_bytes, size_t* ws_bytes);
mgc_status mgc_decompress(mgc_ctx ctx, const void* d_in, size_t in_bytes, void* d_out,
                          size_t out_cap, void* d_ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Fixed-rate block transform coding (ZFP-X: Algorithm "ZFP Fix-Rate
 * Compression", Section IV-C).  The array (FP32 or FP64, 1 to 3 axes) is cut
 * into blocks of 4^ndim values in row-major block order (a partial block
 * repeats each axis' last value).  Each block keeps exactly
 * maxbits = round(rate * 4^ndim) bits: its values are aligned to the block's
 * largest exponent e as P-bit integers trunc(x 2^(q - e)) (P = 32 or 64,
 * q = P - 2 - ndim), transformed per axis (the last axis first) by two levels
 * of reversible integer Haar lifting, ordered by total frequency, mapped to
 * negabinary and coded bit plane by bit plane with group tests until the
 * budget is spent.  There is no error bound: the rate fixes the size.
 * rate: bits per value, with maxbits >= 2 + exponent bits (9 for FP32, 12 for
 * FP64) and rate <= 2 P.
 * Stream (little-endian): u32 magic 0x465A474D, u8 dtype, u8 ndim, u16 0,
 * u32 maxbits, u32 0, u64 shape[3], f64 rate, u64 blocks, u64 total bytes
 * (64-byte header); then the blocks' bits, block b at bits
 * [b maxbits, (b + 1) maxbits) of u64 words in which bit j is bit j mod 64 of
 * word j / 64; zero padding to 8 bytes.
 * mgc_zfp_query: the stream's exact size (and 0 workspace bytes).
 * mgc_zfp_compress (asynchronous on `stream`): d_result (device, two u64)
 *   receives {MGC_OK or MGC_EINVAL (NaN/Inf in the data), stream bytes}.
 * mgc_zfp_parse_header: fields of a host copy of the header.
 * mgc_zfp_decompress (BLOCKING: reads the 64-byte header from the device):
 *   writes the array to d_out.
 * Errors: MGC_EINVAL (shape, dtype, rate, pointers), MGC_ENOSPC (out_cap),
 * MGC_EFORMAT, MGC_EDEVICE.
 * ---------------------------------------------------------------------- */
mgc_status mgc_zfp_query(int ndim, const uint64_t* shape, mgc_dtype dtype, double rate,
                         size_t* stream_bytes);
mgc_status mgc_zfp_compress(mgc_ctx ctx, const void* d_in, int ndim, const uint64_t* shape,
                            mgc_dtype dtype, double rate, void* d_out, size_t out_cap,
                            uint64_t* d_result, void* stream);
mgc_status mgc_zfp_parse_header(const void* h_header, size_t bytes, int* ndim,
                                uint64_t* shape3, mgc_dtype* dtype, double* rate,
                                uint64_t* stream_bytes);
mgc_status mgc_zfp_decompress(mgc_ctx ctx, const void* d_in, size_t in_bytes, void* d_out,
                              size_t out_cap, void* stream);

/* ------------------------------------------------------------------------
 * Host-resident arrays (Section V: the host-device execution model, the
 * three-queue pipeline with two buffer pairs, Algorithm "Adaptive
 * Pipeline").  The array is cut along its slowest axis into chunks of whole
 * planes; each chunk is compressed as an array of its own (the same bound:
 * absolute tau for L-inf, tau * sqrt(chunk values / values) for L2, so the
 * whole array keeps the requested bound) while the next chunk is copied in
 * and the previous stream copied out on three HIP streams.  A relative bound
 * first streams the array through the range pass (one more host-to-device
 * copy of the data) to fix tau.  Chunk sizes start at init_chunk_bytes and
 * follow C_next = min(max(Theta(C / Phi(C)), C), limit_chunk_bytes, rest),
 * Phi(C) = phi_alpha C + phi_beta below phi_threshold and phi_gamma above
 * (compression throughput, bytes/s), Theta(t) = t * h2d_bytes_per_s; with
 * phi_gamma = 0 every chunk has init_chunk_bytes.  mgc_pipe_profile fits
 * Phi and measures the copy bandwidth on a prefix of the data.
 *
 * Container (little-endian): u32 magic 0x5043474D, u32 chunk count, u8
 * dtype, norm, mode, ndim, u32 0, u64 shape[3], f64 bound, f64 tau, u64
 * total bytes (64-byte header); per chunk {u64 first plane, u64 planes, u64
 * stream offset, u64 stream bytes}; the chunk streams (mgc_compress's
 * format), each at a multiple of 8 bytes.  mgc_pipe_info parses a host copy
 * of the header (ndim, shape, dtype, total bytes, chunk count).
 *
 * h_in / h_out are host memory (pinned memory lets the copies overlap the
 * kernels; pageable memory works but the copies then wait).  The calls are
 * BLOCKING and allocate their device buffers (two input, two output, one
 * workspace) for the call.  stats (optional) receives seconds spent in
 * host-to-device copies, kernels, device-to-host copies, the relative-bound
 * pre-pass and overall, the overlap ratio (copy time overlapped by kernel
 * time over all copy time) and the chunk count.
 * Errors: MGC_EINVAL (arguments, NaN/Inf data), MGC_ENOSPC (out_cap),
 * MGC_ERANGE, MGC_EFORMAT (container), MGC_EUNSUPPORTED, MGC_EDEVICE.
 * ---------------------------------------------------------------------- */
typedef struct {
  uint64_t init_chunk_bytes;   /* C_init (0: 64 MiB) */
  uint64_t limit_chunk_bytes;  /* C_limit (0: 1 GiB) */
  double phi_alpha, phi_beta;  /* Phi(C) = alpha C + beta below the threshold (bytes/s) */
  double phi_gamma;            /* Phi(C) = gamma from the threshold on; 0 = fixed chunks */
  uint64_t phi_threshold;      /* bytes */
  double h2d_bytes_per_s;      /* Theta(t) = t * h2d_bytes_per_s */
} mgc_pipe_model;
typedef struct {
  double total_s, h2d_s, kernel_s, d2h_s, prepass_s, overlap;
  uint64_t chunks;
} mgc_pipe_stats;
mgc_status mgc_pipe_max_bytes(int ndim, const uint64_t* shape, mgc_dtype dtype,
                              const mgc_pipe_model* model, size_t* max_out_bytes);
mgc_status mgc_pipe_compress(mgc_ctx ctx, const void* h_in, int ndim, const uint64_t* shape,
                             mgc_dtype dtype, double error_bound, mgc_norm norm, mgc_mode mode,
                             const mgc_pipe_model* model, void* h_out, size_t out_cap,
                             uint64_t* h_out_size, mgc_pipe_stats* stats);
mgc_status mgc_pipe_info(const void* h_in, size_t in_bytes, int* ndim, uint64_t* shape3,
                         mgc_dtype* dtype, uint64_t* total, uint64_t* chunks);
mgc_status mgc_pipe_decompress(mgc_ctx ctx, const void* h_in, size_t in_bytes, void* h_out,
                               size_t out_cap, mgc_pipe_stats* stats);
mgc_status mgc_pipe_profile(mgc_ctx ctx, const void* h_in, int ndim, const uint64_t* shape,
                            mgc_dtype dtype, double error_bound, mgc_norm norm, mgc_mode mode,
                            mgc_pipe_model* model);

/* ------------------------------------------------------------------------
 * Transform only (Algorithm 1 without quantisation): the multilevel
 * coefficients as FP64 values in stream order - the coarsest level's nodal
 * values row-major, then for each finer level its 2^D - 1 subbands (subband
 * m holds the level's new nodes along active axis d when bit d of m is set,
 * its coarse nodes otherwise; axis 0 is the slowest), each row-major.
 * d_coeffs holds N doubles.  Asynchronous on `stream`.
 * Errors: MGC_EINVAL, MGC_ENOSPC (ws_bytes), MGC_EDEVICE.
 * ---------------------------------------------------------------------- */
mgc_status mgc_transform_query(int ndim, const uint64_t* shape, size_t* ws_bytes);
mgc_status mgc_decompose(mgc_ctx ctx, const void* d_in, int ndim, const uint64_t* shape,
                         mgc_dtype dtype, double* d_coeffs, void* d_ws, size_t ws_bytes,
                         void* stream);
mgc_status mgc_recompose(mgc_ctx ctx, const double* d_coeffs, int ndim,
                         const uint64_t* shape, mgc_dtype out_dtype, void* d_out,
                         void* d_ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Differentiation form.  Recomposition is linear in the coefficients, so the
 * gradient of any quantity of interest J(u) with respect to the multilevel
 * coefficients c is R^T (dJ/du), R = recompose.  mgc_recompose_adjoint applies
 * R^T level by level from the finest: Gbar = P^T g, v = M_{l-1}^{-1} Gbar,
 * cbar_l = (g - M_l P v) at the level's new nodes, then g = Gbar; finally
 * cbar_0 = g.  d_grad_u holds N doubles on the input grid (row-major) and
 * d_grad_coeffs receives N doubles in stream order.  Quantisation has no
 * useful derivative; treating it as the identity (straight-through) makes
 * this also the gradient with respect to the unquantised coefficients.
 *
 * mgc_recompose_levels is mgc_recompose that also stores every coarse level's
 * nodal grid G_0 .. G_{L-1} (FP64, level after level, row-major) in d_levels
 * (levels_bytes >= 8 * sum of their sizes; see mgc_levels_query), the
 * per-level checkpoints of a forward pass.
 * Asynchronous on `stream`.  Errors: MGC_EINVAL, MGC_ENOSPC, MGC_EDEVICE.
 * ---------------------------------------------------------------------- */
mgc_status mgc_adjoint_query(int ndim, const uint64_t* shape, size_t* ws_bytes);
mgc_status mgc_recompose_adjoint(mgc_ctx ctx, const double* d_grad_u, int ndim,
                                 const uint64_t* shape, double* d_grad_coeffs, void* d_ws,
                                 size_t ws_bytes, void* stream);
mgc_status mgc_levels_query(int ndim, const uint64_t* shape, size_t* levels_bytes);
mgc_status mgc_recompose_levels(mgc_ctx ctx, const double* d_coeffs, int ndim,
                                const uint64_t* shape, mgc_dtype out_dtype, void* d_out,
                                double* d_levels, size_t levels_bytes, void* d_ws,
                                size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Huffman stage alone (Algorithm 2) on n 16-bit symbols, chunk size C
 * (multiple of 64, 64..65536).  Stream: u32 magic 0x3148474D, u32 C,
 * u64 N, n_codes, n_chunks, n_words, total bytes (48-byte header), then the
 * codebook, chunk offsets and words sections laid out as in the compressed
 * stream.  Code lengths come from the two-queue construction with ties taken
 * from the leaf queue (length limit 32 by halving frequencies), codes are
 * canonical, and codes are packed most-significant bit first into 32-bit
 * words, each chunk starting on a word boundary.
 * mgc_huffman_encode is BLOCKING (returns the length in *h_out_size).
 * mgc_huffman_decode writes n symbols to d_sym (asynchronous after a
 * blocking read of the 48-byte header); d_in starts on a 4-byte boundary.
 * Errors: MGC_EINVAL, MGC_ENOSPC, MGC_EFORMAT, MGC_EDEVICE.
 * ---------------------------------------------------------------------- */
mgc_status mgc_huffman_query(uint64_t n, uint32_t C, size_t* ws_bytes, size_t* max_out_bytes);
mgc_status mgc_huffman_encode(mgc_ctx ctx, const uint16_t* d_sym, uint64_t n, uint32_t C,
                              void* d_out, size_t out_cap, void* d_ws, size_t ws_bytes,
                              void* stream, uint64_t* h_out_size);
mgc_status mgc_huffman_decode(mgc_ctx ctx, const void* d_in, size_t in_bytes,
                              uint16_t* d_sym, uint64_t n, void* d_ws, size_t ws_bytes,
                              void* stream);

/* ------------------------------------------------------------------------
 * Huffman-X: the Huffman pipeline of Algorithm 2 (Section IV-B) as a
 * standalone lossless codec for byte and integer streams.
 *
 * Keys: u8 and u16 values are their own keys (dict 256 / 65536, base 0, no
 * escapes).  An i32 or i64 value v with base <= v <= base + dict - 2 is key
 * v - base (2 <= dict <= 65536); every other value is key dict - 1 and is
 * stored raw after the coded section, in position order.  The keys are coded
 * by the Huffman stage above (its stream, 8-byte aligned, is the coded
 * section).  Stream, little-endian: u32 magic 0x5848474D, u8 type, 3 zero
 * bytes, u32 dict, u32 C, i64 base, u64 n, u64 escaped values, u64 coded
 * section bytes (0 when n = 0), u64 total bytes, u64 0 (64-byte header);
 * the coded section; the escaped values (type width each); zero padding to a
 * multiple of 8 bytes.
 * mgc_hx_query: workspace bytes and the largest stream for n values.
 * mgc_hx_compress (asynchronous on `stream`): d_in holds n values of `type`
 *   (device, naturally aligned).  d_out receives the stream; d_result
 *   (device, two u64) receives {mgc_status of the run (MGC_OK, or
 *   MGC_EDEVICE when a device-side check failed), stream bytes}.
 * mgc_hx_parse_header: fields of a stream header already copied to the host
 *   (at least 64 bytes); any output pointer may be null.
 * mgc_hx_decompress: writes the n values to d_out (n and type must match the
 *   header); BLOCKING (reads the headers first and a status word at the end).
 *   d_in starts on an 8-byte boundary.
 * n < 2^32.  Errors: MGC_EINVAL (type, dict, base, C, pointers),
 * MGC_EUNSUPPORTED (n >= 2^32), MGC_ENOSPC (out_cap, ws_bytes), MGC_EFORMAT
 * (corrupt or truncated stream), MGC_EDEVICE.
 * ---------------------------------------------------------------------- */
typedef enum { MGC_HX_U8 = 0, MGC_HX_U16 = 1, MGC_HX_I32 = 2, MGC_HX_I64 = 3 } mgc_hx_type;
mgc_status mgc_hx_query(uint64_t n, mgc_hx_type type, uint32_t C, size_t* ws_bytes,
                        size_t* max_out_bytes);
mgc_status mgc_hx_compress(mgc_ctx ctx, const void* d_in, uint64_t n, mgc_hx_type type,
                           uint32_t dict, int64_t base, uint32_t C, void* d_out, size_t out_cap,
                           void* d_ws, size_t ws_bytes, uint64_t* d_result, void* stream);
mgc_status mgc_hx_parse_header(const void* h_header, size_t bytes, mgc_hx_type* type,
                               uint64_t* n, uint32_t* dict, int64_t* base, uint32_t* C,
                               uint64_t* total);
mgc_status mgc_hx_decompress(mgc_ctx ctx, const void* d_in, size_t in_bytes, void* d_out,
                             uint64_t n, mgc_hx_type type, void* d_ws, size_t ws_bytes,
                             void* stream);

/* ------------------------------------------------------------------------
 * Batched form: n arrays (uneven shapes, dtypes and bounds; one norm and
 * mode) compressed together.  Each stage of Algorithm 1 and Algorithm 2 runs
 * as one launch over the blocks of every array, with the per-array error
 * budget derived on the device, so the call makes no host round trip; the
 * launch sequence is captured into a HIP graph on first use and replayed by
 * one graph launch afterwards.  Array j's stream is bit-identical to what
 * mgc_compress writes for it with the same outlier capacity.
 *
 * Shapes are passed as n rows of 3 (row j: ndims[j] entries, the rest 0).
 * mgc_batch_query: total workspace bytes, total output bytes, and the byte
 *   offset of each array's output slot (h_out_offsets, n entries, optional).
 * mgc_compress_batched (asynchronous on `stream`): d_in[j] holds array j
 *   (device).  Stream j is written at d_out + offset j; d_sizes[j] (device,
 *   u64) receives its length and d_status[j] (device, i32) an mgc_status:
 *   MGC_EINVAL (NaN/Inf), MGC_ERANGE, or MGC_ENOSPC with d_sizes[j] = the
 *   escaped values needed (then compress that array alone with that
 *   capacity).  Constant and empty arrays get their trivial streams.  Host
 *   errors (bad arguments, small buffers) are returned directly.
 *   flags: MGC_BATCH_EAGER launches the stages directly instead of the
 *   graph; MGC_BATCH_NO_TUNE skips the autotuner (defaults are used for
 *   kinds not forced).  The first call for a batch signature (shapes,
 *   dtypes, outlier_cap) builds per-array plans, block maps and, unless
 *   disabled, runs the autotuner: every candidate of each tuning kind is
 *   timed on the call's own data and the fastest kept.  Calls on one context
 *   must not overlap; the buffers of a call must stay valid until it ends.
 * mgc_set_tuning forces candidate `candidate` of tuning kind `kind` for later
 *   calls of the context, batched and plain (-1 = autotune again for batched
 *   calls, the default candidate 0 for plain calls).  Candidates:
 *   MGC_TUNE_DEC_F32 / MGC_TUNE_DEC_F64 - tile shape (coarse outputs, z y x)
 *   of the three-axis decomposition kernel on FP32 / FP64 input: f32
 *   {4x8x16, 8x8x8, 4x4x16, 2x8x32}, f64 {4x8x8, 4x4x16, 2x8x16, 8x8x8};
 *   every tile candidate gives bit-identical output.
 *   MGC_TUNE_THOMAS_STRIDED / MGC_TUNE_THOMAS_ROWS - tridiagonal sweeps of
 *   the strided axes / the contiguous axis: candidate 0 (the default, kept
 *   by the autotuner) solves every coarse grid too large for one workgroup
 *   with partitioned sweeps where its lines fit (512 values on strided axes,
 *   1024 on the contiguous one) and with serial sweeps otherwise (16 values
 *   in flight per line / 16-value LDS segments); candidates 1 and 2 force
 *   serial sweeps everywhere (8 / 4 values in flight; 32 / 8-value
 *   segments), whose results agree with candidate 0 up to rounding.  Batched
 *   and plain calls under the same candidates give identical streams.
 * mgc_tuning_info: the candidate count of a kind and the choice used by the
 *   context's most recent batched call (-1 before any).
 * ---------------------------------------------------------------------- */
#define MGC_BATCH_EAGER 1
#define MGC_BATCH_NO_TUNE 2
enum { MGC_TUNE_DEC_F32 = 0, MGC_TUNE_DEC_F64 = 1, MGC_TUNE_THOMAS_STRIDED = 2,
       MGC_TUNE_THOMAS_ROWS = 3 };
mgc_status mgc_batch_query(int n, const int* ndims, const uint64_t* shapes,
                           const mgc_dtype* dtypes, uint64_t outlier_cap, size_t* ws_bytes,
                           size_t* out_bytes, uint64_t* h_out_offsets);
mgc_status mgc_compress_batched(mgc_ctx ctx, int n, const void* const* d_in, const int* ndims,
                                const uint64_t* shapes, const mgc_dtype* dtypes,
                                const double* bounds, mgc_norm norm, mgc_mode mode,
                                uint64_t outlier_cap, void* d_out, size_t out_cap, void* d_ws,
                                size_t ws_bytes, uint64_t* d_sizes, int32_t* d_status,
                                int flags, void* stream);
mgc_status mgc_set_tuning(mgc_ctx ctx, int kind, int candidate);
mgc_status mgc_tuning_info(mgc_ctx ctx, int kind, int* n_candidates, int* last_choice);

/* ------------------------------------------------------------------------
 * Decoder launch shape (Algorithm 2, decoding: one thread per chunk).  The
 * decoder keeps each thread's coded words in an LDS ring refilled with whole
 * aligned pieces: ring 1 = 64-byte pieces refilled every 16 symbols, 2 =
 * 32-byte pieces every 8, 3 = 16-byte pieces every 4; by default the widest
 * ring that fits beside the codebook's symbol table is used, with enough
 * wavefronts per block that one pass of blocks covers the GPU.
 * mgc_set_decoder forces a ring (0 = automatic) and a wavefront count per
 * block (1..16, 0 = automatic) for later decodes on the context (decompress
 * and huffman_decode); a forced pair that does not fit in LDS makes those
 * calls fail with MGC_EINVAL.  Every shape decodes the same symbols.
 * mgc_decoder_info returns the pair the context's latest decode used.
 * ---------------------------------------------------------------------- */
mgc_status mgc_set_decoder(mgc_ctx ctx, int ring, int waves);
mgc_status mgc_decoder_info(mgc_ctx ctx, int* ring, int* waves);

/* ------------------------------------------------------------------------
 * Stage timing.  When enabled, every entry point records HIP events around
 * each kernel launch on its stream; mgc_profile_read returns, per stage
 * name, the number of launches and their total GPU milliseconds accumulated
 * since the last reset (reading synchronises the recorded events).
 * `names` receives a '\n'-separated list (at most names_cap bytes); counts
 * and ms receive up to `cap` entries in the same order.
 * ---------------------------------------------------------------------- */
mgc_status mgc_profile_enable(mgc_ctx ctx, int enable);
mgc_status mgc_profile_reset(mgc_ctx ctx);
mgc_status mgc_profile_read(mgc_ctx ctx, char* names, size_t names_cap, uint64_t* counts,
                            double* ms, int cap, int* n_stages);

#ifdef __cplusplus
}
#endif
#endif /* MGC_H */
