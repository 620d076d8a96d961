// Launch wrappers of the HIP kernels (defined in transform.hip and
// huffman.hip), called by the host orchestration in api.cpp.
#pragma once

#include "common.hpp"

namespace mgc {

// ---- tile shapes ---------------------------------------------------------
// Coarse outputs per tile of the decomposition kernel.  Three-axis levels
// have candidates (the batched form's autotuner picks one per input type;
// every candidate gives bit-identical results); entry 0 is the plain default.
struct TileShape {
  int z, y, x;
};
constexpr int kDecCands = 4;
constexpr TileShape kDecTiles3F32[kDecCands] = {{4, 8, 16}, {8, 8, 8}, {4, 4, 16}, {2, 8, 32}};
constexpr TileShape kDecTiles3F64[kDecCands] = {{4, 8, 8}, {4, 4, 16}, {2, 8, 16}, {8, 8, 8}};
constexpr TileShape kDecTile2F32 = {1, 16, 32}, kDecTile2F64 = {1, 8, 32};
constexpr TileShape kDecTile1 = {1, 1, 256};
inline TileShape dec_tile(int D, bool f32, int cand) {
  if (cand < 0 || cand >= kDecCands) cand = 0;
  if (D == 3) return f32 ? kDecTiles3F32[cand] : kDecTiles3F64[cand];
  if (D == 2) return f32 ? kDecTile2F32 : kDecTile2F64;
  return kDecTile1;
}
// Thomas sweeps: values in flight per thread on strided axes, and the LDS
// segment length on the contiguous axis (entry 0 is the plain default).
constexpr int kThomasCands = 3;
constexpr int kThomasU[kThomasCands] = {16, 8, 4};
constexpr int kThomasSeg[kThomasCands] = {16, 32, 8};

// ---- transform.hip -------------------------------------------------------
// Blocks of the range pre-pass: a function of N alone, so that the sum of
// squares is reduced in the same order by every entry point.
constexpr int kRangeBlocks = 1024;
__host__ __device__ inline unsigned range_blocks(int64_t N) {
  const int64_t b = (N + 16383) / 16384;
  return (unsigned)(b < 1 ? 1 : (b > kRangeBlocks ? kRangeBlocks : b));
}
// Range pre-pass and error budget: bud[0..3] <- min, max, sum of squares and
// a non-finite flag of u (dtype dt); then tau, tau' and the bins (see Bud).
// part holds 4 * kRangeBlocks doubles.
void launch_range(const void* u, mgc_dtype dt, int64_t N, double* part, const BudgetIn& b,
                  double* bud, unsigned* status, hipStream_t s);
// One decomposition level: coefficients of the level's new nodes (quantised
// to symbols with the reciprocal bin *rp when sym != nullptr, else FP64 into
// raw) and the restriction f = (P^T M_l) G_l onto the coarse grid (fout,
// FP64).  rp is a device pointer (the compression's error-budget block); the
// kernels return at once when the gate is closed (see gate_closed).
// cand: tile candidate for three-axis levels (kDecTiles3F32/F64), others fixed.
void launch_dec_level(const void* G, bool g_is_f32, const LevelGeom& g, double* fout,
                      uint16_t* sym, double* raw, const double* rp, const OutlierBuf& ob,
                      unsigned* status, const unsigned* gate, hipStream_t s, int cand = 0);
// Solve the coarse mass matrix along internal axis `axis` for every line of
// x (coarse grid nc).  When sub != nullptr, x <- sub - solution.
// cand: kThomasSeg (axis 2) or kThomasU (axes 0, 1) candidate; with cand 0,
// grids of at most kThomasTilePoints points and lines of at most 540 values
// use the LDS line tiles instead (all variants give identical results).
// With cand 0 an axis whose lines fit (thomas_part_class) is solved by the
// partitioned sweeps, whose results agree with the serial ones up to
// rounding; the caller decides which grids go this way (a grid small enough
// for launch_thomas_grid is solved serially in one launch instead).  The
// batched form makes the same choice per array, so both agree bit for bit.
constexpr int64_t kThomasTilePoints = int64_t(1) << 22;
void launch_thomas(int axis, double* x, const int64_t nc[3], const AxisTab& t,
                   const double* sub, hipStream_t s, int cand = 0);
// Partitioned-sweep class of a line of len values along internal axis `axis`
// (kPartNone: serial sweeps).  kPartScanLong marks rows of 257..1024 values
// for the batched form's launches.
enum { kPartNone = 0, kPart40 = 1, kPart64 = 2, kPartScan = 3, kPartScanLong = 4 };
int thomas_part_class(int axis, int64_t len);
// All active axes of a coarse grid small enough for LDS in one launch (the
// same results as the per-axis launches, axis 2 first; sub as there, applied
// after the last sweep).  Only for grids with thomas_grid_fits(g).
bool thomas_grid_fits(const LevelGeom& g);
void launch_thomas_grid(double* x, const LevelGeom& g, const double* sub, hipStream_t s);
// Level-0 block: values of G0 (m0 entries) quantised with *rp (sym) or
// copied (raw); gated like launch_dec_level.
void launch_level0(const void* G0, bool g_is_f32, int64_t m0, uint16_t* sym, double* raw,
                   const double* rp, const OutlierBuf& ob, unsigned* status,
                   const unsigned* gate, hipStream_t s);
// Recomposition: f = (P^T M_l) c_l on the coarse grid from the coefficients.
void launch_rec_restrict(const LevelGeom& g, const CoeffSrc& src, double q, double* fout,
                         hipStream_t s);
// Recomposition: G_l = P Gc + c_l (out in FP32 or FP64).
void launch_rec_interp(const double* Gc, const LevelGeom& g, const CoeffSrc& src, double q,
                       void* out, bool out_f32, hipStream_t s);
// Dequantised coefficients of stream positions [0, m) (levels 0 .. n-1 of lb,
// level l starting at off[l], bin q[l]) into raw, escaped values included.
struct LevelBins {
  int64_t off[kMaxLevels + 1];
  double q[kMaxLevels + 1];
  int n;
};
void launch_dequant_prefix(const CoeffSrc& src, int64_t m, const LevelBins& lb, double* raw,
                           hipStream_t s);
void launch_rec_level0(const CoeffSrc& src, int64_t m0, double q, void* out, bool out_f32,
                       hipStream_t s);
// The smallest levels in one workgroup with their grids in LDS.  Level l
// qualifies when its fine grid, coarse grid and coarse lines fit; the levels
// 1..top taken must all qualify, with top < kTailLevels and their tables (a
// prefix of the plan's table block) at most tail_max_table() doubles.
constexpr int kTailLevels = 16;
struct TailTabArgs {
  const double* src;            // device: level 1's first table (axis 0 wl)
  uint32_t n;                   // doubles up to the end of level top's tables
  uint32_t wl[kTailLevels][3];  // offset of level l's axis-k wl from src
};
bool tail_level_fits(const LevelGeom& g);
size_t tail_max_table();
// Decomposition of levels top..1 and level 0 (as the level loop with
// launch_dec_level, the solves and launch_level0): G is level top's grid;
// d_geo the plan's device geometry (d_geo[l]).
void launch_dec_tail(const void* G, bool g_is_f32, const LevelGeom* d_geo, int top,
                     const TailTabArgs& tt, uint16_t* sym, double* raw, const double* rdev,
                     const OutlierBuf& ob, unsigned* status, const unsigned* gate, hipStream_t s);
// Recomposition of level 0 and levels 1..top (as launch_rec_level0 and the
// level loop): out receives level top's grid; the coefficients of levels
// <= coarse_top come from `coarse`, the others from src; q[0..top] host.
void launch_rec_tail(const CoeffSrc& src, const CoeffSrc& coarse, int coarse_top,
                     const double* q, const LevelGeom* d_geo, int top, const TailTabArgs& tt,
                     void* out, bool out_f32, hipStream_t s);
// Adjoint of recomposition, one level: Gc = P^T g (also copied to Gc_copy,
// which the Thomas sweeps then turn into v = M_{l-1}^{-1} Gc); Pv on the fine
// grid; cbar (stream order) = g - M_l P v at the level's new nodes.
void launch_adj_restrict(const double* gl, const LevelGeom& g, double* Gc, double* Gc_copy,
                         hipStream_t s);
void launch_prolong(const double* v, const LevelGeom& g, double* out, hipStream_t s);
void launch_adj_mass(const double* Pv, const double* gl, const LevelGeom& g, double* cbar,
                     hipStream_t s);
void launch_fill(void* out, bool out_f32, int64_t N, double v, hipStream_t s);
// Zeroes n (1..4) ranges of whole 4-byte words in one launch.
void launch_zero_words(void* const* ptrs, const size_t* bytes, int n, hipStream_t s);
// Copies n (<= a few KiB) bytes with one block, e.g. into mapped host memory.
void launch_copy_bytes(void* dst, const void* src, size_t n, hipStream_t s);

// ---- batched form (one launch per stage over every array of a batch) ----
// Map-driven launches take nb = number of map entries (grid covers them).
void launch_b_zero(const Job* jobs, int n, hipStream_t s);
void launch_b_range(const Job* jobs, const JobBlock* map, uint32_t nb, bool f32, hipStream_t s);
void launch_b_budget(const Job* jobs, int n, hipStream_t s);
void launch_b_dec_level(const Job* jobs, const JobBlock* map, uint32_t nb, int step, int D,
                        bool f32, int cand, hipStream_t s);
void launch_b_thomas(int axis, const Job* jobs, const JobBlock* map, uint32_t nb, int step,
                     int cand, hipStream_t s);
// Partitioned sweeps (class c of thomas_part_class; kPartScan / kPartScanLong
// on axis 2) of every mapped array; waves = wavefronts per block, at least
// the largest segment count of the mapped arrays (axes 0 and 1).
void launch_b_thomas_part(int axis, int c, int waves, const Job* jobs, const JobBlock* map,
                          uint32_t nb, int step, hipStream_t s);
void launch_b_level0(const Job* jobs, const JobBlock* map, uint32_t nb, bool f32,
                     hipStream_t s);
void launch_b_histogram(const Job* jobs, const JobBlock* map, uint32_t nb, hipStream_t s);
void launch_b_codebook(const Job* jobs, int n, hipStream_t s);
void launch_b_chunk_words(const Job* jobs, const JobBlock* map, uint32_t nb, hipStream_t s);
void launch_b_layout_scan(const Job* jobs, int n, hipStream_t s);
void launch_b_outlier_sort(const Job* jobs, int n, hipStream_t s);
// escaped values in stream order from the chunk escape counts and lane masks
void launch_b_escape_order(const Job* jobs, int n, hipStream_t s);
void launch_b_encode(const Job* jobs, const JobBlock* map, uint32_t nb, hipStream_t s);
void launch_b_header(const Job* jobs, int n, hipStream_t s);
// Blocks per array of the map-driven Huffman launches.
uint32_t hist_blocks(int64_t N);
uint32_t chunk_words_blocks(int64_t N, int C);
constexpr uint32_t kChunkSyms = 1024;   // symbols per coded chunk (C)

// ---- huffman.hip ---------------------------------------------------------
size_t codebook_scratch_bytes();
CodebookScratch carve_codebook_scratch(void* base);

struct DecodeTables;
size_t decode_tables_bytes();

// The Huffman stage's kernels take an optional gate (a compression's status
// word; see gate_closed): a null gate runs them unconditionally.
// The histogram counts symbols win_lo .. win_lo + kHistWindow - 1 and the
// symbol `hot` in LDS (the rest with global atomics); the default window is
// centred on the compressor's zero symbol and hot is its escape symbol.
constexpr uint32_t kHistWindow = 32768;
constexpr uint32_t kHistWinLo = kHalf - kHistWindow / 2;
void launch_histogram(const uint16_t* sym, int64_t n, unsigned* hist, hipStream_t s,
                      const unsigned* gate = nullptr, uint32_t win_lo = kHistWinLo,
                      uint32_t hot = 0);
// Code lengths (clen, and lay->n_codes), then, when canon is set, the
// canonical codes (code, the packed words with the first codes behind them,
// the codebook section, lay->max_len); with canon false the caller runs
// launch_canon after the lengths (the chunk-size pass needs the lengths
// only).
void launch_codebook(const unsigned* hist, const CodebookScratch& sc, uint32_t* code,
                     uint8_t* clen, uint8_t* cb_out_base, uint64_t cb_off, Layout* lay,
                     hipStream_t s, const unsigned* gate = nullptr, bool canon = true);
void launch_canon(const CodebookScratch& sc, uint32_t* code, uint8_t* cb_out_base,
                  uint64_t cb_off, Layout* lay, hipStream_t s, const unsigned* gate = nullptr);
// zc / zl (optional, C = 1024): per-chunk escape counts and per-lane escape
// masks with in-chunk prefix counts, for launch_escape_order.
void launch_chunk_words(const uint16_t* sym, int64_t N, int C, const uint8_t* clen,
                        uint32_t* cw, Layout* lay, hipStream_t s, const unsigned* gate = nullptr,
                        uint32_t* zc = nullptr, uint32_t* zl = nullptr);
// Escaped values in stream order without a sort: the rank of each appended
// (position, value) record among the escapes, from the chunk counts zc
// (prefix-summed into zpre) and the lane masks zl of launch_chunk_words;
// writes the stream's outlier sections (after the layout scan).  sums holds
// kEscSumsMax entries.  An inconsistent record sets ST_INTERNAL in *status.
constexpr int64_t kEscSumsMax = 1024;
// Exclusive prefix sums zpre of the n_chunks counts zc (sums: kEscSumsMax
// words); skipped when lay->status is set.
void launch_chunk_prefix(const uint32_t* zc, uint32_t* zpre, uint32_t* sums, int64_t n_chunks,
                         const Layout* lay, hipStream_t s);
void launch_escape_order(const OutlierBuf& ob, const uint32_t* zc, const uint32_t* zl,
                         uint32_t* zpre, uint32_t* sums, int64_t n_chunks, uint8_t* out,
                         Layout* lay, unsigned* status, hipStream_t s, const unsigned* gate);
// Section layout + exclusive scan of the chunk word counts into the stream's
// offsets section.  huff_only selects the Huffman-only stream layout.  cw
// holds the n_chunks counts and has room for kScanSumWords more words at
// cw + scan_sums_at(n_chunks) (the per-block totals of large scans).
constexpr int kScanSumWords = 512;
inline int64_t scan_sums_at(int64_t n_chunks) { return (n_chunks + 1) & ~int64_t(1); }
inline int64_t chunk_words_len(int64_t n_chunks) {
  return scan_sums_at(n_chunks) + kScanSumWords;
}
void launch_layout_scan(const uint32_t* cw, int64_t n_chunks, uint8_t* out, uint64_t cb_off,
                        Layout* lay, const unsigned long long* n_out, uint64_t out_cap_n,
                        bool huff_only, hipStream_t s, const unsigned* gate = nullptr);
void launch_outlier_sort(const OutlierBuf& ob, uint32_t* keyA, uint32_t* valA, uint32_t* keyB,
                         uint32_t* valB, int key_bits, uint8_t* out, Layout* lay,
                         hipStream_t s, const unsigned* gate = nullptr);
// pk: the codebook's packed (rank << 6 | length) words and first-code table
// (see CodebookScratch::pk).
void launch_encode(const uint16_t* sym, int64_t N, int C, const uint32_t* code,
                   const uint8_t* clen, const uint32_t* pk, uint8_t* out, const Layout* lay,
                   hipStream_t s, const unsigned* gate = nullptr);
// Writes the header and bins (from the device error-budget block bud) once
// the layout is known, or the trivial stream of a constant or empty array
// (empty: no range pass ran), and the result words res[0] = mgc_status,
// res[1] = stream bytes (MGC_ENOSPC: escaped values needed).
void launch_header(uint8_t* out, const Header& h, const double* bud, const Layout* lay,
                   const unsigned* status, bool empty, unsigned long long* res, hipStream_t s);
void launch_huff_header(uint8_t* out, uint32_t C, uint64_t N, uint64_t n_chunks,
                        const Layout* lay, unsigned long long* info, hipStream_t s);

// Decode tables from a codebook section; first sets status[0..3] to zero (it
// is the first kernel of a decompression), then ORs ST_FORMAT into status[0]
// when the section is invalid.
void launch_decode_tables(const uint8_t* cb, uint64_t n_codes, DecodeTables* t,
                          unsigned* status, hipStream_t s);
// Decoder launch shape: ring (1: 64-byte pieces, ring of 32 words, refill
// every 16 symbols; 2: 32-byte pieces, 16 words, every 8; 3: 16-byte pieces,
// 8 words, every 4) and wavefronts per block; 0 = automatic.  Returns the
// shape used.
struct DecodeShape {
  int ring = 0, waves = 0;
};
DecodeShape launch_decode(const uint8_t* in, uint64_t off_sec, uint64_t words_sec,
                          uint64_t n_chunks, uint64_t n_words, int C, int64_t N,
                          uint64_t n_codes, const DecodeTables* t, uint16_t* sym,
                          unsigned* status, hipStream_t s, DecodeShape force = DecodeShape{});

// Fixed-rate block coding (zfp.hip): blocks of 4^ndim values, maxbits bits
// each, payload at out + kZfpHeaderBytes (cleared beforehand unless maxbits
// is a multiple of 64); h is written as the header and res = {mgc_status,
// stream bytes} (MGC_EINVAL when *status shows a non-finite value).
void launch_zfp_encode(const void* in, bool f64, int ndim, const uint64_t* shape,
                       uint64_t nblocks, uint32_t maxbits, uint8_t* out, unsigned* status,
                       const ZfpHead& h, unsigned long long* res, hipStream_t s);
void launch_zfp_decode(const uint8_t* in, bool f64, int ndim, const uint64_t* shape,
                       uint64_t nblocks, uint32_t maxbits, void* out, hipStream_t s);

// Huffman-X (hx.hip).  Keys of n values of a stream type (mgc_hx_type):
// u8/u16 values are their keys; i32/i64 values in [lo, hi] are key v - lo,
// others key esc with zc[chunk] = escapes per 1024 values (zc unused for
// u8/u16).
void launch_hx_keys(const void* in, uint64_t n, int type, int64_t lo, int64_t hi, uint32_t esc,
                    uint16_t* key, uint32_t* zc, hipStream_t s);
// Escaped i32/i64 values, in position order, at sec + lay->end (after the
// coded section) from the exclusive chunk prefix zpre.
void launch_hx_place(const void* in, uint64_t n, int type, int64_t lo, int64_t hi,
                     const uint32_t* zc, const uint32_t* zpre, uint8_t* sec, const Layout* lay,
                     hipStream_t s);
// 64-byte stream header and res = {mgc_status, stream bytes}; zc/zpre null
// for types without escapes, lay unused when n = 0.
void launch_hx_header(uint8_t* out, int type, uint32_t D, uint32_t C, int64_t base, uint64_t n,
                      const uint32_t* zc, const uint32_t* zpre, const Layout* lay,
                      unsigned long long* res, hipStream_t s);
// Escape keys per 1024 decoded keys.
void launch_hx_count(const uint16_t* key, uint64_t n, uint32_t esc, uint32_t* zc, hipStream_t s);
// Values from decoded keys (u8, i32, i64); ST_FORMAT into *status for keys
// no value maps to or escape counts that disagree with n_esc.
void launch_hx_values(const uint16_t* key, uint64_t n, int type, int64_t lo, uint32_t kmax,
                      uint32_t esc_key, const void* esc, uint64_t n_esc, const uint32_t* zc,
                      const uint32_t* zpre, void* out, unsigned* status, hipStream_t s);

}  // namespace mgc
