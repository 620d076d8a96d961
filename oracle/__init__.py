"""FP64 CPU oracle for the multigrid error-bounded compressor.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously correct
NumPy implementation of what the GPU library computes.  Only the tests, the
smoke check and the benchmark's CPU-baseline leg may import it; the product
path never does, and this package imports nothing from the GPU library.

It follows the paper's MGARD pipeline (Algorithm 1 and Section IV-A: per level
interpolation coefficients, a transfer/mass-matrix product, tridiagonal
correction solves along each dimension, the add, then level-wise linear
quantisation) and its Huffman pipeline (Algorithm 2 and Section IV-B:
histogram, sort by frequency, drop zeros, code construction, encode,
serialise).  Where the paper is silent the reading used is stated in the
docstring of the function that implements it.

Modules
-------
hierarchy   grid hierarchy (which nodes survive each coarsening step)
operators   per-axis prolongation P and mass matrices M of hat functions
transform   decompose / recompose / adjoint of recompose, stream order
quantize    error bound -> per-level bins, quantiser, symbols and outliers
huffman     code lengths, canonical codes, chunked bit packing, decoding
stream      byte layout of a compressed stream; compress / decompress
hx          the Huffman pipeline as a standalone lossless codec for byte and
            integer streams (keys, escapes, stream layout)
pipe        chunked compression of host-resident arrays: the adaptive chunk
            rule, per-chunk bounds and the container layout
zfp         fixed-rate block transform coding (alignment, lifting, negabinary,
            bit planes with group tests)
"""
from .hierarchy import Hierarchy
from .transform import decompose, recompose, recompose_adjoint, level_slices
from .quantize import error_budget, level_bins, quantize, dequantize, to_symbols, from_symbols
from .huffman import (histogram, code_lengths, canonical_codes, encode_chunks,
                      decode_chunks)
from .stream import compress, decompress, parse_header
from . import hx, pipe, zfp

__all__ = [
    "Hierarchy", "decompose", "recompose", "recompose_adjoint", "level_slices",
    "error_budget", "level_bins", "quantize", "dequantize", "to_symbols",
    "from_symbols", "histogram", "code_lengths", "canonical_codes",
    "encode_chunks", "decode_chunks", "compress", "decompress", "parse_header", "hx", "pipe", "zfp",
]
