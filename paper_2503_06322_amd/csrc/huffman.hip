// Huffman stage for gfx950 (Algorithm 2 and Section IV-B of the paper):
// histogram -> sort by frequency -> drop zero keys -> code construction ->
// encode -> serialise, plus the inverse decode.
//
//  * histogram: LDS-privatised counts for a central window of symbols (the
//    quantised coefficients cluster around the dictionary centre), global
//    atomics for the rest.
//  * codebook: the non-zero keys are sorted by (frequency, symbol) with a
//    stable LSD radix sort over many blocks (k_cbs_count / k_cbs_pass; the
//    batched form sorts in the one workgroup below).  Code lengths follow the
//    two-queue construction (leaves in that order, internal nodes in creation
//    order, ties to the leaf), computed by one workgroup of 1024 threads in
//    rounds: with m nodes already taken, no node created later can weigh less
//    than t = (the next node to be paired) + (the smallest remaining), so
//    every available node of weight <= t is taken in this round by a parallel
//    merge of the two sorted queues.  The threshold at least doubles every
//    two rounds, so the round count is logarithmic in the total weight.
//    Depths come from walking the rounds backwards; lengths above 32 halve
//    the frequencies and rebuild.  Codes are canonical (RFC 1951
//    construction), assigned on many blocks (k_canon_count / k_canon_rank:
//    each wavefront a run of the symbols with its count of each length in
//    one lane; the batched form assigns them in its one workgroup).
//  * chunk lengths and layout: one wavefront per chunk sums the code lengths
//    (and, in a compression, counts the escape symbols per chunk and lane);
//    an exclusive scan of the chunk word counts over many blocks gives the
//    offsets; escaped values are placed in stream order by their rank.
//  * encode: arrays of at least 8,192 chunks use persistent blocks of 16
//    wavefronts that keep the packed (rank, length) words of a central symbol
//    window in LDS (k_encode_win); smaller ones one wavefront per chunk
//    (k_encode).  A wave prefix scan of code lengths gives each lane its bit
//    offset; codes are OR-ed MSB-first into the chunk's 32-bit words in LDS,
//    then stored coalesced.
//  * decoding tables: the same runs on many blocks (k_dt_count / k_dt_rank)
//    validate the codebook section and build the per-length tables, the
//    (length, symbol)-ordered symbols and the prefix table.
//  * decode: one thread per chunk; a 12-bit prefix table in LDS gives the
//    code length shared by all codes under a prefix (or the lengths to test
//    against the canonical limits when several share it), and the code's
//    index in the (length, symbol)-ordered symbol table, also in LDS.  Coded
//    words reach each lane's LDS ring as whole aligned pieces; decoded
//    symbols leave as whole 128-byte rows.
#include "kernels.hpp"

#include <algorithm>

namespace mgc {

constexpr int kLutBits = 12;
// Prefix-table entry flag: the prefix holds codes of several lengths
// (lengths lo and hi in bits 16..21 and 22..27), or none (lo = 0).
constexpr uint32_t kLutMixed = 1u << 31;

struct DecodeTables {
  uint32_t first[34];
  uint32_t count[34];
  uint32_t base[34];
  uint64_t limit[34];   // left-justified exclusive upper bound of each length
  uint32_t maxlen;
  uint32_t valid;               // 1 only after a codebook passed validation
  // Entry of each kLutBits-bit prefix of the window.  When every window
  // with that prefix starts with a code of one length d: d << 16 |
  // ((base[d] - first[d]) mod 2^16), so that the code's index in sorted is
  // (top d bits of the window + entry) mod 2^16.  Otherwise kLutMixed with
  // the shortest and longest length under the prefix.
  uint32_t lut[1 << kLutBits];
  uint16_t sorted[kDict];       // symbols in (length, symbol) order
  // construction scratch: per run of the section, its counts per length and
  // (at 34) whether it holds an invalid length or symbol
  uint32_t runs[256 * 36];
};

size_t decode_tables_bytes() { return sizeof(DecodeTables); }

size_t codebook_scratch_bytes() { return (size_t)kDict * 4 * 16 + kPkFirstWords * 4; }

CodebookScratch carve_codebook_scratch(void* base) {
  uint32_t* p = static_cast<uint32_t*>(base);
  CodebookScratch s;
  s.keyA = p; p += kDict;
  s.valA = p; p += kDict;
  s.keyB = p; p += kDict;
  s.valB = p; p += kDict;
  s.symAsc = p; p += kDict;
  s.freqAsc = p; p += kDict;
  s.Iw = p; p += kDict;
  s.Sw = p; p += 2 * kDict;
  s.leafPar = p; p += kDict;
  s.parA = p; p += kDict;
  s.parB = p; p += kDict;
  s.dstA = p; p += kDict;
  s.dstB = p; p += kDict;
  s.pk = p; p += kDict + kPkFirstWords;
  s.hcnt = p; p += kDict / 2;
  s.fmaxT = p; p += kDict / 2;
  return s;
}

namespace {

__device__ __forceinline__ uint64_t lanemask_lt() {
  const int lane = threadIdx.x & 63;
  return (lane == 0) ? 0ull : (~0ull >> (64 - lane));
}

// Orders the wavefront's LDS accesses before the fence against those after.
__device__ __forceinline__ void wave_lds_fence() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Lanes of the wave whose `digit` (nbits bits) equals this lane's, among the
// lanes with valid set.
__device__ __forceinline__ uint64_t match_digit(unsigned digit, int nbits, bool valid) {
  uint64_t peers = __ballot(valid);
  for (int b = 0; b < nbits; ++b) {
    const bool bit = (digit >> b) & 1u;
    const uint64_t m = __ballot(bit);
    peers &= bit ? m : ~m;
  }
  return peers;
}

// ---------------------------------------------------------------- histogram
// One 1024-thread block per CU.  A window of 32768 bins around the
// dictionary centre (|k| < 16384) is counted in LDS; symbols outside it and
// the escape symbol go to global atomics.  Symbols are read 8 at a time.
constexpr int kHistWin = kHistWindow;

// Symbols lo .. lo + kHistWin - 1 are counted in LDS; h[kHistWin] counts the
// symbol `hot` when it lies outside (the escape symbol: frequent when many
// values escape the dictionary, and then too contended for one global
// counter); other symbols go to global atomics.
__device__ __forceinline__ void hist_add(unsigned s, unsigned* h, unsigned* hist, unsigned lo,
                                         unsigned hot, unsigned cnt = 1u) {
  const unsigned d = s - lo;
  if (d < (unsigned)kHistWin) atomicAdd(&h[d], cnt);
  else if (s == hot) atomicAdd(&h[kHistWin], cnt);
  else atomicAdd(&hist[s], cnt);
}

// The eight symbols of a 16-byte word, equal neighbours counted together:
// narrow distributions (most symbols equal) would otherwise send every lane
// of a wavefront to the same LDS counter at once.
__device__ __forceinline__ void hist_add8(const uint4& w, unsigned* h, unsigned* hist,
                                          unsigned lo, unsigned hot) {
  const unsigned a[4] = {w.x, w.y, w.z, w.w};
  unsigned cur = a[0] & 0xFFFFu, cnt = 0u;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const unsigned s = (k & 1) ? (a[k >> 1] >> 16) : (a[k >> 1] & 0xFFFFu);
    if (s != cur) {
      hist_add(cur, h, hist, lo, hot, cnt);
      cur = s;
      cnt = 0u;
    }
    ++cnt;
  }
  hist_add(cur, h, hist, lo, hot, cnt);
}

__device__ __forceinline__ void histogram_body(const uint16_t* __restrict__ sym, int64_t n,
                                               unsigned* __restrict__ hist, uint32_t blk,
                                               uint32_t nblk, unsigned lo, unsigned hot) {
  __shared__ unsigned h[kHistWin + 1];
  for (int i = threadIdx.x; i <= kHistWin; i += 1024) h[i] = 0;
  __syncthreads();
  const int64_t stride = (int64_t)nblk * 1024;
  const bool vec = (reinterpret_cast<uintptr_t>(sym) & 15) == 0;
  const int64_t nvec = vec ? n / 8 : 0;
  const uint4* sv = reinterpret_cast<const uint4*>(sym);
  int64_t i = (int64_t)blk * 1024 + threadIdx.x;
  for (; i + 3 * stride < nvec; i += 4 * stride) {
    uint4 w[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) w[u] = sv[i + u * stride];
#pragma unroll
    for (int u = 0; u < 4; ++u) hist_add8(w[u], h, hist, lo, hot);
  }
  for (; i < nvec; i += stride) hist_add8(sv[i], h, hist, lo, hot);
  for (int64_t i = nvec * 8 + (int64_t)blk * 1024 + threadIdx.x; i < n; i += stride)
    hist_add(sym[i], h, hist, lo, hot);
  __syncthreads();
  for (int i = threadIdx.x; i < kHistWin; i += 1024)
    if (h[i]) atomicAdd(&hist[lo + i], h[i]);
  if (threadIdx.x == 0 && h[kHistWin]) atomicAdd(&hist[hot], h[kHistWin]);
}

__global__ __launch_bounds__(1024) void k_histogram(const uint16_t* __restrict__ sym, int64_t n,
                                                     unsigned* __restrict__ hist,
                                                     const unsigned* __restrict__ gate,
                                                     unsigned lo, unsigned hot) {
  if (gate_closed(gate)) return;
  histogram_body(sym, n, hist, blockIdx.x, gridDim.x, lo, hot);
}

// ---------------------------------------------------- single-block helpers
struct SortSmem {
  unsigned hist[256];
  unsigned base[256];
  unsigned total[256];
  unsigned wcnt[16][256];
};

// Stable LSD radix sort by the low `bits` bits of the keys, 8 bits a pass,
// one 1024-thread block.  Returns true when the result is in (k1, v1).
// Wavefront w owns a contiguous run of the items (tiles of 64; eight tiles'
// loads in flight at once): per pass it counts its digits, one block scan
// turns the per-wavefront counts into output offsets, and it scatters its
// run in order (peers with the same digit found by ballots, ranked by lane),
// so the sort is stable with three block barriers per pass.
__device__ bool block_radix_sort(uint32_t* k0, uint32_t* v0, uint32_t* k1, uint32_t* v1,
                                 uint32_t n, int bits, SortSmem& sm) {
  constexpr int B = 8;  // tiles per batch of loads
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int passes = (bits + 7) / 8;
  const uint32_t run = ((n + 1023) / 1024) * 64;
  const uint32_t i0 = min(n, (uint32_t)wave * run), i1 = min(n, i0 + run);
  for (int pass = 0; pass < passes; ++pass) {
    const int shift = 8 * pass;
    for (int d = lane; d < 256; d += 64) sm.wcnt[wave][d] = 0;
    wave_lds_fence();
    for (uint32_t t = i0; t < i1; t += 64 * B) {
      uint32_t key[B];
#pragma unroll
      for (int b = 0; b < B; ++b) key[b] = k0[min(t + b * 64 + lane, i1 - 1)];
#pragma unroll
      for (int b = 0; b < B; ++b) {
        const bool valid = t + b * 64 + lane < i1;
        const unsigned d = (key[b] >> shift) & 255u;
        const uint64_t peers = match_digit(d, 8, valid);
        if (valid && __popcll(peers & lanemask_lt()) == 0) sm.wcnt[wave][d] += __popcll(peers);
        wave_lds_fence();
      }
    }
    __syncthreads();
    // offsets: digit d's output starts after all smaller digits, and wave
    // w's items of digit d after those of the earlier wavefronts
    unsigned tot = 0, incl = 0;
    if (tid < 256) {
      for (int w = 0; w < 16; ++w) tot += sm.wcnt[w][tid];
      incl = tot;
      for (int o = 1; o < 64; o <<= 1) {
        const unsigned y = (unsigned)__shfl_up((int)incl, o, 64);
        if (lane >= o) incl += y;
      }
      if (lane == 63) sm.total[wave] = incl;
    }
    __syncthreads();
    if (tid < 256) {
      unsigned acc = incl - tot;
      for (int w = 0; w < wave; ++w) acc += sm.total[w];
      for (int w = 0; w < 16; ++w) {
        const unsigned c = sm.wcnt[w][tid];
        sm.wcnt[w][tid] = acc;
        acc += c;
      }
    }
    __syncthreads();
    for (uint32_t t = i0; t < i1; t += 64 * B) {
      uint32_t key[B], val[B];
#pragma unroll
      for (int b = 0; b < B; ++b) {
        const uint32_t i = min(t + b * 64 + lane, i1 - 1);
        key[b] = k0[i];
        val[b] = v0[i];
      }
#pragma unroll
      for (int b = 0; b < B; ++b) {
        const bool valid = t + b * 64 + lane < i1;
        const unsigned d = (key[b] >> shift) & 255u;
        const uint64_t peers = match_digit(d, 8, valid);
        const unsigned r = __popcll(peers & lanemask_lt());
        const unsigned pos = valid ? sm.wcnt[wave][d] + r : 0u;
        if (valid) {
          k1[pos] = key[b];
          v1[pos] = val[b];
        }
        wave_lds_fence();
        if (valid && r == 0) sm.wcnt[wave][d] = pos + __popcll(peers);
        wave_lds_fence();
      }
    }
    __syncthreads();
    uint32_t* t;
    t = k0; k0 = k1; k1 = t;
    t = v0; v0 = v1; v1 = t;
  }
  return passes & 1;
}

__device__ unsigned block_max(unsigned v, unsigned* sm32) {
  for (int o = 32; o > 0; o >>= 1) v = max(v, (unsigned)__shfl_xor((int)v, o, 64));
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) sm32[wave] = v;
  __syncthreads();
  unsigned r = 0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) r = max(r, sm32[w]);
  __syncthreads();
  return r;
}

// Exclusive scan of one value per thread over the 1024-thread block.
__device__ unsigned block_excl_scan(unsigned v, unsigned* sm32, unsigned* total) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  unsigned x = v;
  for (int o = 1; o < 64; o <<= 1) {
    const unsigned y = (unsigned)__shfl_up((int)x, o, 64);
    if (lane >= o) x += y;
  }
  __syncthreads();
  if (lane == 63) sm32[wave] = x;
  __syncthreads();
  unsigned before = 0, tot = 0;
  for (int w = 0; w < 16; ++w) {
    if (w < wave) before += sm32[w];
    tot += sm32[w];
  }
  __syncthreads();
  *total = tot;
  return before + x - v;
}

// ---------------------------------------------------------------- codebook
constexpr int kWin = 12288;  // LDS window per queue in a merge round
static_assert(kWin < 2 * 8192, "window counts search from 8192 down");
constexpr int kMaxRounds = 256;
constexpr int kSortTile = 2048;                  // items per block of the multi-block sort
constexpr int kSortTiles = kDict / kSortTile;    // tiles (and blocks) per pass
constexpr int kSortPasses = 4;                   // 8-bit digits of a 32-bit frequency
static_assert(kSortTiles % 4 == 0 && kSortPasses * 256 * kSortTiles <= kDict / 2,
              "sort count table fits its scratch");

// Large LDS of the codebook build: the sort's tables, then the merge windows.
union CbBig {
  SortSmem sort;
  struct {
    uint32_t Lwin[kWin], Iwin[kWin], newI[kWin + 1];
  } mw;
};

static_assert(sizeof(CbBig) >= 2 * kDict, "depth and length bytes fit the merge windows");

struct CbSmem {
  unsigned round_lo[kMaxRounds];
  unsigned sm32[16];
  unsigned m, li, ii, nI, lastw, rounds, cntL, cntI;
  unsigned long long t;
  unsigned lcount[34];
  unsigned lfirst[34];
  unsigned wl[16][34];
};

// For four keys at once: pos[u] = count of a[0..n) below w[u] (LE: at most
// w[u]), a ascending, n >= 1.  Branch-free halving (the probe is always in
// range and the trip count depends on n only), so the four probes of a step
// are in flight together.
template <bool LE>
__device__ __forceinline__ void lds_count4(const uint32_t* a, unsigned n, const uint32_t (&w)[4],
                                           unsigned (&pos)[4]) {
  unsigned b[4] = {0u, 0u, 0u, 0u};
  for (unsigned len = n; len > 1;) {
    const unsigned half = len >> 1;
    uint32_t v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = a[b[u] + half];
#pragma unroll
    for (int u = 0; u < 4; ++u) b[u] = (LE ? v[u] <= w[u] : v[u] < w[u]) ? b[u] + half : b[u];
    len -= half;
  }
  uint32_t v[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) v[u] = a[b[u]];
#pragma unroll
  for (int u = 0; u < 4; ++u) pos[u] = b[u] + ((LE ? v[u] <= w[u] : v[u] < w[u]) ? 1u : 0u);
}

// Count of the entries <= t in a[lo, hi) (ascending), by the whole block:
// one probe per thread at a stride S = ceil((hi - lo) / 1024) finds the
// stride interval that holds the boundary, then one probe per thread inside
// it (S <= 1024 for the queue lengths here, at most 2^17).
__device__ unsigned block_count_le(const uint32_t* a, unsigned lo, unsigned hi,
                                   unsigned long long t) {
  const unsigned len = hi - lo, tid = threadIdx.x;
  if (len == 0) return 0;
  const unsigned S = (len + 1023) / 1024;
  const unsigned p = tid * S;
  const unsigned c1 = __syncthreads_count(p < len && (unsigned long long)a[lo + p] <= t);
  if (c1 == 0) return 0;
  const unsigned base = (c1 - 1) * S;  // a[lo + base] <= t < a[lo + base + S] (or the end)
  const unsigned q = base + 1 + tid;
  const unsigned c2 = __syncthreads_count(tid + 1 < S && q < len && (unsigned long long)a[lo + q] <= t);
  return base + 1 + c2;
}

// Weight bound of a merge round: with m nodes taken (a pending first child
// of weight lastw when m is odd), the next pair's weight; l0 <= l1 and
// i0 <= i1 are the fronts of the leaf and internal queues (~0 when empty).
__device__ __forceinline__ unsigned long long merge_threshold(unsigned m, uint32_t lastw,
                                                              unsigned long long l0,
                                                              unsigned long long l1,
                                                              unsigned long long i0,
                                                              unsigned long long i1) {
  if (m & 1) return (unsigned long long)lastw + (l0 < i0 ? l0 : i0);
  const unsigned long long a = l0 < i0 ? l0 : i0;
  const unsigned long long b = l0 < i0 ? (l1 < i0 ? l1 : i0) : (l0 < i1 ? l0 : i1);
  return a + b;
}

// 1. non-zero keys in ascending symbol order (each thread owns 64 symbols,
//    read as sixteen 16-byte vectors kept in registers); returns their count
__device__ unsigned compact_keys(const unsigned* __restrict__ hist, const CodebookScratch& s,
                                 CbSmem& sm) {
  const int tid = threadIdx.x;
  uint4 hv[16];
  const uint4* h4 = reinterpret_cast<const uint4*>(hist) + tid * 16;
#pragma unroll
  for (int k = 0; k < 16; ++k) hv[k] = h4[k];
  unsigned cnt = 0;
#pragma unroll
  for (int k = 0; k < 16; ++k)
    cnt += (hv[k].x != 0) + (hv[k].y != 0) + (hv[k].z != 0) + (hv[k].w != 0);
  unsigned total;
  unsigned off = block_excl_scan(cnt, sm.sm32, &total);
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const unsigned f4[4] = {hv[k].x, hv[k].y, hv[k].z, hv[k].w};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (f4[q]) {
        s.symAsc[off] = tid * 64 + 4 * k + q;
        s.freqAsc[off] = f4[q];
        ++off;
      }
    }
  }
  return total;
}

// Canonical codes (RFC 1951 construction): count per length, first code per
// length, then the rank of each symbol among equal lengths in ascending
// symbol order.  A wavefront takes a contiguous run [i0, i1) of the symbols
// in tiles of 64.  Its running count of each length d sits in lane d; a tile
// is taken one distinct length at a time (the lengths of neighbouring
// symbols mostly agree, so a tile holds few): the first remaining lane names
// the length, a ballot finds its peers, their ranks are the count read from
// lane d plus their order in the tile, and lane d advances.

// Lane d: the run's symbols of length d.
__device__ unsigned wave_len_counts(const uint8_t* lenAsc, unsigned i0, unsigned i1) {
  constexpr int B = 8;
  const int lane = threadIdx.x & 63;
  unsigned cnt = 0;
  for (unsigned t = i0; t < i1; t += 64 * B) {
    unsigned dl[B];
#pragma unroll
    for (int u = 0; u < B; ++u) dl[u] = lenAsc[min(t + u * 64 + lane, i1 - 1)];
#pragma unroll
    for (int u = 0; u < B; ++u) {
      uint64_t rem = __ballot(t + u * 64 + lane < i1);
      while (rem) {
        const int ld = __ffsll((unsigned long long)rem) - 1;
        const unsigned d = (unsigned)__builtin_amdgcn_readlane((int)dl[u], ld);
        const uint64_t m = __ballot(dl[u] == d) & rem;
        if (lane == (int)d) cnt += (unsigned)__popcll(m);
        rem &= ~m;
      }
    }
  }
  return cnt;
}

// The ranking pass over the run: lane d of cnt holds the symbols of length d
// before the run, lane d of fst a per-length value handed on (the first code
// of length d).  Calls out(i, symbol, d, rank among length d, fst of d) for
// each symbol i of the run; sym_of(i) loads symbol i.
template <typename SymFn, typename OutFn>
__device__ void wave_rank_pass(const uint8_t* lenAsc, unsigned i0, unsigned i1, unsigned cnt,
                               const unsigned fst, SymFn sym_of, OutFn out) {
  constexpr int B = 8;
  const int lane = threadIdx.x & 63;
  for (unsigned t = i0; t < i1; t += 64 * B) {
    unsigned dl[B], sy[B];
#pragma unroll
    for (int u = 0; u < B; ++u) {
      const unsigned i = min(t + u * 64 + lane, i1 - 1);
      dl[u] = lenAsc[i];
      sy[u] = sym_of(i);
    }
#pragma unroll
    for (int u = 0; u < B; ++u) {
      const unsigned i = t + u * 64 + lane;
      const bool valid = i < i1;
      uint64_t rem = __ballot(valid);
      unsigned rank = 0, first = 0;
      while (rem) {
        const int ld = __ffsll((unsigned long long)rem) - 1;
        const unsigned d = (unsigned)__builtin_amdgcn_readlane((int)dl[u], ld);
        const uint64_t m = __ballot(dl[u] == d) & rem;
        const unsigned base = (unsigned)__builtin_amdgcn_readlane((int)cnt, (int)d);
        const unsigned fd = (unsigned)__builtin_amdgcn_readlane((int)fst, (int)d);
        if ((m >> lane) & 1u) {
          rank = base + (unsigned)__popcll(m & lanemask_lt());
          first = fd;
        }
        if (lane == (int)d) cnt += (unsigned)__popcll(m);
        rem &= ~m;
      }
      if (valid) out(i, sy[u], dl[u], rank, first);
    }
  }
}

// The run's codes (fst: first codes): code[], the packed words s.pk and the
// codebook section (n symbols, then their lengths).
__device__ void wave_len_ranks(const uint8_t* lenAsc, unsigned i0, unsigned i1, unsigned cnt,
                               const unsigned fst, const CodebookScratch& s,
                               uint32_t* __restrict__ code, uint8_t* __restrict__ cb_out,
                               const unsigned n) {
  uint16_t* cs = reinterpret_cast<uint16_t*>(cb_out);
  wave_rank_pass(
      lenAsc, i0, i1, cnt, fst, [&](unsigned i) { return s.symAsc[i]; },
      [&](unsigned i, unsigned sy, unsigned d, unsigned rank, unsigned first) {
        code[sy] = first + rank;
        s.pk[sy] = (rank << 6) | d;
        cs[i] = (uint16_t)sy;
        cb_out[2 * n + i] = (uint8_t)d;
      });
}

// First code of each length from the counts per length (tot[l]); with
// write also stored behind the packed words, with lay->max_len.
__device__ __forceinline__ void first_codes(const unsigned* tot, unsigned* first, uint32_t* pk,
                                            Layout* lay, bool write) {
  unsigned c = 0, ml = 0;
  for (int l = 1; l <= kMaxCodeLen; ++l) {
    const unsigned cntl = tot[l];
    if (cntl) ml = l;
    first[l] = c;
    if (write) pk[kDict + l] = c;  // first code of each length, for the encoder
    c = (c + cntl) << 1;
  }
  if (write) lay->max_len = ml;
}

// The canonical codes of n symbols in one block of 1024 threads (lengths in
// symbol order in lenAsc): a counting pass, the scan of the counts over the
// wavefronts (which also gives the counts per length), the ranking pass.
__device__ void canonical_codes(const unsigned n, const uint8_t* lenAsc, const CodebookScratch& s,
                                uint32_t* __restrict__ code, uint8_t* __restrict__ cb_out,
                                Layout* __restrict__ lay, CbSmem& sm) {
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const unsigned run = ((n + 1023) / 1024) * 64;
  const unsigned i0 = min(n, (unsigned)wave * run), i1 = min(n, i0 + run);
  const unsigned cnt = wave_len_counts(lenAsc, i0, i1);
  if (lane < 34) sm.wl[wave][lane] = cnt;
  __syncthreads();
  if (tid < 34) {
    unsigned acc = 0;
    for (int w = 0; w < 16; ++w) {
      const unsigned c = sm.wl[w][tid];
      sm.wl[w][tid] = acc;
      acc += c;
    }
    sm.lcount[tid] = acc;
  }
  __syncthreads();
  if (tid == 0) first_codes(sm.lcount, sm.lfirst, s.pk, lay, true);
  __syncthreads();
  wave_len_ranks(lenAsc, i0, i1, lane < 34 ? sm.wl[wave][lane] : 0u,
                 lane < 34 ? sm.lfirst[lane] : 0u, s, code, cb_out, n);
}

// PRESORTED: the leaf sort of the first round was done by the multi-block
// sort (k_cbs_count / k_cbs_pass), which also wrote the non-zero keys in
// symbol order; otherwise the block compacts and sorts them itself.
template <bool PRESORTED, bool CANON>
__device__ __forceinline__ void codebook_body(const unsigned* __restrict__ hist,
                                              const CodebookScratch& s,
                                              uint32_t* __restrict__ code,
                                              uint8_t* __restrict__ clen,
                                              uint8_t* __restrict__ cb_out,
                                              Layout* __restrict__ lay) {
  __shared__ CbSmem sm;
  __shared__ __align__(16) CbBig big;
  const int tid = threadIdx.x;
  unsigned n, pre_passes = 0;
  if (PRESORTED) {
    // item count: every non-zero bin is counted once in the first pass's
    // (digit, tile) table
    unsigned c = 0;
    for (unsigned i = tid; i < 256u * kSortTiles; i += 1024) c += s.hcnt[i];
    unsigned fm = 0;
    for (int t = 0; t < kSortTiles; ++t) fm = max(fm, s.fmaxT[t]);
    pre_passes = (32 - __clz(fm) + 7) / 8;
    unsigned total;
    block_excl_scan(c, sm.sm32, &total);
    n = total;
  } else {
    n = compact_keys(hist, s, sm);
  }
  __syncthreads();

  if (n == 0) {
    uint4* clen4 = reinterpret_cast<uint4*>(clen);
    for (unsigned i = tid; i < kDict / 16; i += 1024) clen4[i] = make_uint4(0u, 0u, 0u, 0u);
    if (tid == 0) {
      lay->n_codes = 0;
      lay->max_len = 0;
    }
    return;
  }
  if (n == 1) {
    // one symbol: a one-bit code
    if (tid == 0) reinterpret_cast<uint8_t*>(&big)[kDict] = 1;
    __syncthreads();
  }
  const uint32_t root = n - 2;
  for (int flatten = 0; n >= 2; ++flatten) {
    if (flatten > 40) {  // 33 halvings bring every frequency to 1
      if (tid == 0) lay->status |= ST_INTERNAL;
      return;
    }
    // 2. sort leaves by (frequency, symbol): stable radix sort of indices
    //    into the ascending-symbol list, keyed by frequency
    bool inB;
    if (PRESORTED && flatten == 0) {
      inB = pre_passes & 1;  // passes alternate B, A, B, A
    } else {
      unsigned fmax = 0;
      for (unsigned i = tid; i < n; i += 1024) {
        s.keyA[i] = s.freqAsc[i];
        s.valA[i] = i;
        fmax = max(fmax, s.freqAsc[i]);
      }
      fmax = block_max(fmax, sm.sm32);
      const int bits = 32 - __clz(fmax);
      __syncthreads();
      inB = block_radix_sort(s.keyA, s.valA, s.keyB, s.valB, n, bits, big.sort);
    }
    const uint32_t* Lw = inB ? s.keyB : s.keyA;   // leaf weights, ascending
    const uint32_t* Lx = inB ? s.valB : s.valA;   // leaf -> index into symAsc
    __syncthreads();
    // 3. two-queue merge in rounds.  A round stages the fronts of both
    //    queues in LDS (up to kWin nodes each, 4096 at a time until a node
    //    above the threshold shows up), ranks every taken node in the merged
    //    order by a binary search in the other queue's window (ties to the
    //    leaf), and adds its weight into its parent's slot with LDS atomics
    //    (integer sums, so the order of the adds does not matter).  The next
    //    round's threshold is read from the same windows.  A round that
    //    takes more than a window's worth of one queue runs from global
    //    memory instead.
    if (tid == 0) {
      sm.m = 0;
      sm.li = 0;
      sm.ii = 0;
      sm.nI = 0;
      sm.lastw = 0;
      sm.rounds = 0;
      sm.cntL = 0;
      sm.cntI = 0;
      sm.t = (unsigned long long)Lw[0] + Lw[1];
    }
    __syncthreads();
    while (true) {
      const unsigned m = sm.m, li = sm.li, ii = sm.ii, nI = sm.nI;
      const unsigned long long t = sm.t;
      if (m == 2 * n - 2) break;
      // internal nodes created in this round: [nI, m_new / 2)
      if (tid == 0 && sm.rounds < kMaxRounds) sm.round_lo[sm.rounds] = nI;
      const unsigned availL = min((unsigned)kWin, n - li);
      const unsigned availI = min((unsigned)kWin, nI - ii);
      const uint32_t lastw0 = sm.lastw;
      for (unsigned k = tid; k <= (unsigned)kWin; k += 1024)
        big.mw.newI[k] = (k == 0 && (m & 1)) ? lastw0 : 0u;
      // window loads; the entries <= t are counted on the way (ballots, one
      // LDS add per wavefront), which the windows' order turns into nl, ni
      unsigned nLd = 0, nId = 0;
      bool moreL = availL > 0, moreI = availI > 0;
      while (moreL || moreI) {
        if (moreL) {
          uint32_t v[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) v[u] = Lw[li + min(nLd + u * 1024 + tid, availL - 1)];
          unsigned c = 0;
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const bool in = nLd + u * 1024 + tid < availL;
            if (in) big.mw.Lwin[nLd + u * 1024 + tid] = v[u];
            c += __popcll(__ballot(in && (unsigned long long)v[u] <= t));
          }
          if ((tid & 63) == 0 && c) atomicAdd(&sm.cntL, c);
        }
        if (moreI) {
          uint32_t v[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) v[u] = s.Iw[ii + min(nId + u * 1024 + tid, availI - 1)];
          unsigned c = 0;
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const bool in = nId + u * 1024 + tid < availI;
            if (in) big.mw.Iwin[nId + u * 1024 + tid] = v[u];
            c += __popcll(__ballot(in && (unsigned long long)v[u] <= t));
          }
          if ((tid & 63) == 0 && c) atomicAdd(&sm.cntI, c);
        }
        __syncthreads();
        if (moreL) {
          const unsigned e = min(nLd + 4096, availL);
          moreL = e < availL && (unsigned long long)big.mw.Lwin[e - 1] <= t;
          nLd = e;
        }
        if (moreI) {
          const unsigned e = min(nId + 4096, availI);
          moreI = e < availI && (unsigned long long)big.mw.Iwin[e - 1] <= t;
          nId = e;
        }
      }
      const unsigned nl = sm.cntL, ni = sm.cntI;
      const bool ovf = (nl == availL && availL < n - li) || (ni == availI && availI < nI - ii);
      if (!ovf) {
        const unsigned m_new = m + nl + ni;
        if (m_new == m) {  // every round takes at least the smallest node
          if (tid == 0) lay->status |= ST_INTERNAL;
          return;
        }
        const unsigned mh = m_new >> 1;  // internal nodes complete after the round
        const unsigned last = nl + ni - 1;
        // leaves: rank = own index + internal nodes lighter than it
        for (unsigned k0 = tid; k0 < nl; k0 += 4096) {
          uint32_t w[4];
          unsigned pos[4] = {0u, 0u, 0u, 0u};
#pragma unroll
          for (int u = 0; u < 4; ++u) w[u] = big.mw.Lwin[min(k0 + u * 1024, nl - 1)];
          if (ni) lds_count4<false>(big.mw.Iwin, ni, w, pos);
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const unsigned k = k0 + u * 1024;
            if (k < nl) {
              const unsigned r = k + pos[u];
              const unsigned par = (m + r) >> 1;
              s.leafPar[li + k] = par;
              if (par < mh) atomicAdd(&big.mw.newI[par - nI], w[u]);
              if (r == last) sm.lastw = w[u];
            }
          }
        }
        // internal nodes: rank = own index + leaves at most as heavy
        for (unsigned k0 = tid; k0 < ni; k0 += 4096) {
          uint32_t w[4];
          unsigned pos[4] = {0u, 0u, 0u, 0u};
#pragma unroll
          for (int u = 0; u < 4; ++u) w[u] = big.mw.Iwin[min(k0 + u * 1024, ni - 1)];
          if (nl) lds_count4<true>(big.mw.Lwin, nl, w, pos);
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const unsigned k = k0 + u * 1024;
            if (k < ni) {
              const unsigned r = k + pos[u];
              const unsigned par = (m + r) >> 1;
              s.parA[ii + k] = par;
              if (par < mh) atomicAdd(&big.mw.newI[par - nI], w[u]);
              if (r == last) sm.lastw = w[u];
            }
          }
        }
        __syncthreads();
        for (unsigned k = tid; k < mh - nI; k += 1024) s.Iw[nI + k] = big.mw.newI[k];
        if (tid == 0) {
          const unsigned long long INF = ~0ull;
          const unsigned li2 = li + nl, ii2 = ii + ni;
          auto lw = [&](unsigned x) -> unsigned long long {
            if (x >= n) return INF;
            return x - li < nLd ? big.mw.Lwin[x - li] : Lw[x];
          };
          auto iw = [&](unsigned y) -> unsigned long long {
            if (y >= mh) return INF;
            if (y >= nI) return big.mw.newI[y - nI];
            return y - ii < nId ? big.mw.Iwin[y - ii] : s.Iw[y];
          };
          sm.t = merge_threshold(m_new, sm.lastw, lw(li2), lw(li2 + 1), iw(ii2), iw(ii2 + 1));
          sm.cntL = 0;
          sm.cntI = 0;
          sm.m = m_new;
          sm.li = li2;
          sm.ii = ii2;
          sm.nI = mh;
          ++sm.rounds;
        }
        __syncthreads();
        continue;
      }
      // global-memory round: leaves and internal nodes of weight <= t
      // (prefixes of the sorted queues, found by a two-level block search),
      // four nodes per thread in flight
      const unsigned la = li + block_count_le(Lw, li, n, t);
      const unsigned ib = ii + block_count_le(s.Iw, ii, nI, t);
      const unsigned nl2 = la - li, ni2 = ib - ii;
      const unsigned m_new = m + nl2 + ni2;
      for (unsigned x0 = li + tid; x0 < la; x0 += 4096) {
        uint32_t w[4];
        unsigned pos[4] = {0u, 0u, 0u, 0u};
#pragma unroll
        for (int u = 0; u < 4; ++u) w[u] = Lw[min(x0 + 1024u * u, la - 1)];
        if (ni2) lds_count4<false>(s.Iw + ii, ni2, w, pos);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const unsigned x = x0 + 1024u * u;
          if (x < la) {
            const unsigned p = m + (x - li) + pos[u];
            s.Sw[p] = w[u];
            s.leafPar[x] = p >> 1;
          }
        }
      }
      for (unsigned y0 = ii + tid; y0 < ib; y0 += 4096) {
        uint32_t w[4];
        unsigned pos[4] = {0u, 0u, 0u, 0u};
#pragma unroll
        for (int u = 0; u < 4; ++u) w[u] = s.Iw[min(y0 + 1024u * u, ib - 1)];
        if (nl2) lds_count4<true>(Lw + li, nl2, w, pos);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const unsigned y = y0 + 1024u * u;
          if (y < ib) {
            const unsigned p = m + (y - ii) + pos[u];
            s.Sw[p] = w[u];
            s.parA[y] = p >> 1;
          }
        }
      }
      __syncthreads();
      const unsigned mh2 = m_new / 2;
      for (unsigned j0 = nI + tid; j0 < mh2; j0 += 4096) {
        uint32_t a[4], b[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const unsigned j = min(j0 + 1024u * u, mh2 - 1);
          a[u] = s.Sw[2 * j];
          b[u] = s.Sw[2 * j + 1];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const unsigned j = j0 + 1024u * u;
          if (j < mh2) s.Iw[j] = (2 * j + 1 == m ? lastw0 : a[u]) + b[u];
        }
      }
      __syncthreads();
      if (tid == 0) {
        const unsigned long long INF = ~0ull;
        const unsigned mh = m_new / 2;
        const uint32_t lw_new = s.Sw[m_new - 1];
        sm.lastw = lw_new;
        sm.t = merge_threshold(m_new, lw_new, la < n ? Lw[la] : INF, la + 1 < n ? Lw[la + 1] : INF,
                               ib < mh ? s.Iw[ib] : INF, ib + 1 < mh ? s.Iw[ib + 1] : INF);
        sm.cntL = 0;
        sm.cntI = 0;
        sm.m = m_new;
        sm.li = la;
        sm.ii = ib;
        sm.nI = mh;
        ++sm.rounds;
      }
      __syncthreads();
    }
    // 4. depths of internal nodes, in LDS as bytes saturated at 255 (a depth
    //    that large only shows that the code must be flattened).  A node
    //    created in round r is taken in a later round, so its parent is
    //    created later still: walking the rounds backwards, each round's
    //    nodes are resolved in parallel.  The parent indices of as many of
    //    the remaining rounds as fit are first staged in LDS (over the length
    //    bytes, written only later) in one copy, so the rounds of a batch
    //    wait on LDS only; a round larger than the stage reads them directly.
    uint8_t* dep = reinterpret_cast<uint8_t*>(&big);  // [n - 1] internal nodes
    uint8_t* lenAsc = dep + kDict;                     // [n] lengths in symbol order
    const unsigned rounds = sm.rounds;
    if (rounds <= (unsigned)kMaxRounds) {
      constexpr unsigned kStage = (unsigned)((sizeof(CbBig) - kDict) / 4);
      uint32_t* pst = reinterpret_cast<uint32_t*>(lenAsc);
      auto round_hi = [&](int r) { return r + 1 < (int)rounds ? sm.round_lo[r + 1] : root + 1; };
      for (int r = (int)rounds - 1; r >= 0;) {
        const unsigned bhi = round_hi(r);
        int r0 = r;
        while (r0 > 0 && bhi - sm.round_lo[r0 - 1] <= kStage) --r0;
        const unsigned blo = sm.round_lo[r0];
        if (bhi - blo <= kStage) {
          for (unsigned y0 = blo + tid; y0 < bhi; y0 += 8192) {
            uint32_t v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = s.parA[min(y0 + 1024u * u, bhi - 1)];
#pragma unroll
            for (int u = 0; u < 8; ++u)
              if (y0 + 1024u * u < bhi) pst[y0 + 1024u * u - blo] = v[u];
          }
          __syncthreads();
          for (int rr = r; rr >= r0; --rr) {
            const unsigned lo = sm.round_lo[rr], hi = round_hi(rr);
            for (unsigned y0 = lo + tid; y0 < hi; y0 += 4096) {
              uint32_t pv[4], dv[4];
#pragma unroll
              for (int u = 0; u < 4; ++u) pv[u] = pst[min(y0 + 1024u * u, hi - 1) - blo];
#pragma unroll
              for (int u = 0; u < 4; ++u) dv[u] = dep[min(pv[u], root)];  // (the root has no parent)
#pragma unroll
              for (int u = 0; u < 4; ++u) {
                const unsigned y = y0 + 1024u * u;
                if (y < hi) dep[y] = y == root ? 0 : (uint8_t)min(dv[u] + 1u, 255u);
              }
            }
            __syncthreads();
          }
          r = r0 - 1;
        } else {
          const unsigned lo = sm.round_lo[r];
          for (unsigned y0 = lo + tid; y0 < bhi; y0 += 8192) {
            uint32_t pv[8], dv[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) pv[u] = s.parA[min(y0 + 1024u * u, bhi - 1)];
#pragma unroll
            for (int u = 0; u < 8; ++u) dv[u] = dep[min(pv[u], root)];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
              const unsigned y = y0 + 1024u * u;
              if (y < bhi) dep[y] = y == root ? 0 : (uint8_t)min(dv[u] + 1u, 255u);
            }
          }
          __syncthreads();
          r -= 1;
        }
      }
    } else {
      // pointer jumping towards the root (global memory), then saturated
      for (unsigned y = tid; y <= root; y += 1024) {
        if (y == root) s.parA[y] = root;
        s.dstA[y] = y == root ? 0u : 1u;
      }
      __syncthreads();
      uint32_t *pa = s.parA, *pb = s.parB, *da = s.dstA, *db = s.dstB;
      for (int jump = 0;; ++jump) {
        if (jump > 40) {  // depth <= n - 1 < 2^17: 18 jumps suffice
          if (tid == 0) lay->status |= ST_INTERNAL;
          return;
        }
        bool more = false;
        for (unsigned y = tid; y <= root; y += 1024) {
          const uint32_t p = pa[y];
          db[y] = da[y] + da[p];
          pb[y] = pa[p];
          more |= pa[p] != root;
        }
        const int any = __syncthreads_or(more);
        uint32_t* tmp;
        tmp = pa; pa = pb; pb = tmp;
        tmp = da; da = db; db = tmp;
        if (!any) break;
      }
      for (unsigned y = tid; y <= root; y += 1024) dep[y] = (uint8_t)min(da[y], 255u);
      __syncthreads();
    }
    // 5. leaf lengths, stored by the leaf's position in symbol order
    //    (sixteen leaves per thread in flight)
    unsigned lmax = 0;
    for (unsigned x0 = tid; x0 < n; x0 += 16384) {
      uint32_t par[16], lx[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const unsigned x = min(x0 + 1024 * u, n - 1);
        par[u] = s.leafPar[x];
        lx[u] = Lx[x];
      }
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        if (x0 + 1024 * u < n) {
          const unsigned l = min(dep[par[u]] + 1u, 255u);
          lenAsc[lx[u]] = (uint8_t)l;
          lmax = max(lmax, l);
        }
      }
    }
    lmax = block_max(lmax, sm.sm32);
    if (lmax <= (unsigned)kMaxCodeLen) break;
    for (unsigned i = tid; i < n; i += 1024) s.freqAsc[i] = (s.freqAsc[i] + 1u) >> 1;
    __syncthreads();
  }
  // 5b. the code length of every symbol (zero for absent ones) through an
  //     LDS table over the depth bytes (dead now): cleared, filled from the
  //     leaves, then stored whole with 16-byte stores
  {
    uint8_t* lenAsc = reinterpret_cast<uint8_t*>(&big) + kDict;
    uint4* tab4 = reinterpret_cast<uint4*>(&big);
    for (unsigned i = tid; i < kDict / 16; i += 1024) tab4[i] = make_uint4(0u, 0u, 0u, 0u);
    __syncthreads();
    uint8_t* tab = reinterpret_cast<uint8_t*>(&big);
    for (unsigned i0 = tid; i0 < n; i0 += 8192) {
      unsigned sy[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) sy[u] = s.symAsc[min(i0 + 1024u * u, n - 1)];
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (i0 + 1024u * u < n) tab[sy[u]] = lenAsc[i0 + 1024u * u];
    }
    __syncthreads();
    uint4* clen4 = reinterpret_cast<uint4*>(clen);
    for (unsigned i = tid; i < kDict / 16; i += 1024) clen4[i] = tab4[i];
  }
  if (tid == 0) lay->n_codes = n;
  if (CANON) {
    // 6-7. canonical codes in this block (lengths in LDS)
    canonical_codes(n, reinterpret_cast<const uint8_t*>(&big) + kDict, s, code, cb_out, lay, sm);
  } else {
    // lengths in symbol order for the canonical pass (k_canon), as bytes
    // over the sort keys (dead now)
    const uint32_t* len4 = reinterpret_cast<const uint32_t*>(&big) + kDict / 4;
    for (unsigned i = tid; i < (n + 3) / 4; i += 1024) s.keyA[i] = len4[i];
  }
}

__global__ __launch_bounds__(1024) void k_codebook(const unsigned* __restrict__ hist,
                                                    CodebookScratch s, uint32_t* __restrict__ code,
                                                    uint8_t* __restrict__ clen,
                                                    uint8_t* __restrict__ cb_out,
                                                    Layout* __restrict__ lay,
                                                    const unsigned* __restrict__ gate) {
  if (gate_closed(gate)) return;
  codebook_body<true, false>(hist, s, code, clen, cb_out, lay);
}

// The canonical codes of the codebook k_codebook built (its lengths in
// symbol order as bytes over s.keyA) on kCanonBlocks blocks of four
// wavefronts, each wavefront a contiguous run of the symbols: the counts per
// length of every run (over s.valA), then the ranks, each block scanning the
// runs' counts before its own.
constexpr int kCanonBlocks = 64;
constexpr int kCanonRuns = kCanonBlocks * 4;

__device__ __forceinline__ void canon_run(unsigned n, unsigned& i0, unsigned& i1) {
  const unsigned gw = blockIdx.x * 4 + (threadIdx.x >> 6);
  const unsigned run = ((n + 64 * kCanonRuns - 1) / (64 * kCanonRuns)) * 64;
  i0 = min(n, gw * run);
  i1 = min(n, i0 + run);
}

// Per length, the counts before each of this block's four runs (off) and in
// all runs (tot), from the runs' counts (cw, `pitch` words per run): partial
// sums over seven groups of runs, then each length's prefix up to the block.
// All 256 threads; ends with a barrier.
struct RunScan {
  unsigned part[7][34];
  unsigned off[4][34];
  unsigned tot[34];
};
__device__ void run_offsets(const unsigned* cw, int pitch, RunScan& rs) {
  constexpr int G = (kCanonRuns + 6) / 7;
  const int tid = threadIdx.x;
  if (tid < 7 * 34) {
    const int d = tid % 34, g = tid / 34;
    unsigned acc = 0;
    for (int w = g * G; w < min((g + 1) * G, kCanonRuns); ++w) acc += cw[w * pitch + d];
    rs.part[g][d] = acc;
  }
  __syncthreads();
  if (tid < 34) {
    const int w0 = blockIdx.x * 4, gb = w0 / G;
    unsigned tot = 0, pre = 0;
    for (int g = 0; g < 7; ++g) {
      tot += rs.part[g][tid];
      if (g < gb) pre += rs.part[g][tid];
    }
    for (int w = gb * G; w < w0; ++w) pre += cw[w * pitch + tid];
    for (int k = 0; k < 4; ++k) {
      rs.off[k][tid] = pre;
      pre += cw[(w0 + k) * pitch + tid];
    }
    rs.tot[tid] = tot;
  }
  __syncthreads();
}

__global__ __launch_bounds__(256) void k_canon_count(CodebookScratch s, const Layout* __restrict__ lay,
                                                      const unsigned* __restrict__ gate) {
  if (gate_closed(gate) || lay->status) return;
  const unsigned n = (unsigned)lay->n_codes;
  if (n == 0) return;
  unsigned i0, i1;
  canon_run(n, i0, i1);
  const unsigned cnt = wave_len_counts(reinterpret_cast<const uint8_t*>(s.keyA), i0, i1);
  const int lane = threadIdx.x & 63;
  if (lane < 34) s.valA[(blockIdx.x * 4 + (threadIdx.x >> 6)) * 34 + lane] = cnt;
}

__global__ __launch_bounds__(256) void k_canon_rank(CodebookScratch s, uint32_t* __restrict__ code,
                                                     uint8_t* __restrict__ cb_out,
                                                     Layout* __restrict__ lay,
                                                     const unsigned* __restrict__ gate) {
  if (gate_closed(gate) || lay->status) return;
  const unsigned n = (unsigned)lay->n_codes;
  if (n == 0) return;
  __shared__ unsigned cw[kCanonRuns * 34];
  __shared__ RunScan rs;
  __shared__ unsigned first[34];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  for (int i = tid; i < kCanonRuns * 34; i += 256) cw[i] = s.valA[i];
  __syncthreads();
  run_offsets(cw, 34, rs);
  if (tid == 0) first_codes(rs.tot, first, s.pk, lay, blockIdx.x == 0);
  __syncthreads();
  unsigned i0, i1;
  canon_run(n, i0, i1);
  wave_len_ranks(reinterpret_cast<const uint8_t*>(s.keyA), i0, i1,
                 lane < 34 ? rs.off[wave][lane] : 0u, lane < 34 ? first[lane] : 0u, s, code, cb_out,
                 n);
}

// ------------------------------------------------- multi-block leaf sort
// Plain calls sort the leaves by (frequency, symbol) on many CUs before the
// one-block code construction: a stable LSD radix sort, 8 bits a pass, over
// tiles of kSortTile items, one 256-thread block per tile.  Pass 0 reads the
// non-zero histogram bins in place (tile t = symbols [kSortTile t,
// kSortTile (t + 1))) and also writes them compacted in symbol order; its
// values are those positions.  A block's output positions are the digit's
// start (counts of all smaller digits) plus the counts of its digit in
// earlier tiles, read from the (digit, tile) table; inside the tile each
// wavefront owns a contiguous run and ranks equal digits by ballots, so the
// sort is stable.  While it scatters, a pass counts the next pass's digits
// of its items by destination tile (global atomics), so every pass reads a
// complete table.  Passes beyond the largest frequency's width return at
// once; pass p writes (keyB, valB) for even p and (keyA, valA) for odd p.
__global__ __launch_bounds__(256) void k_cbs_count(const unsigned* __restrict__ hist,
                                                   CodebookScratch s,
                                                   const unsigned* __restrict__ gate) {
  if (gate_closed(gate)) return;
  __shared__ unsigned cnt[256];
  __shared__ unsigned wmax[4];
  const int t = blockIdx.x, tid = threadIdx.x;
  cnt[tid] = 0;
  __syncthreads();
  const uint4* h4 = reinterpret_cast<const uint4*>(hist + (size_t)t * kSortTile) + tid * 2;
  const uint4 a = h4[0], b = h4[1];
  const unsigned f[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
  unsigned fm = 0;
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    if (f[u]) atomicAdd(&cnt[f[u] & 255u], 1u);
    fm = max(fm, f[u]);
  }
  for (int o = 32; o > 0; o >>= 1) fm = max(fm, (unsigned)__shfl_xor((int)fm, o, 64));
  if ((tid & 63) == 0) wmax[tid >> 6] = fm;
  __syncthreads();
  s.hcnt[(size_t)tid * kSortTiles + t] = cnt[tid];
  for (int p = 1; p < kSortPasses; ++p) s.hcnt[((size_t)p * 256 + tid) * kSortTiles + t] = 0;
  if (tid == 0) s.fmaxT[t] = max(max(wmax[0], wmax[1]), max(wmax[2], wmax[3]));
}

template <int P>
__global__ __launch_bounds__(256) void k_cbs_pass(const unsigned* __restrict__ hist,
                                                  CodebookScratch s,
                                                  const unsigned* __restrict__ gate) {
  if (gate_closed(gate)) return;
  __shared__ unsigned wcnt[4][256];
  __shared__ unsigned sm32[16];
  __shared__ unsigned nzw[4];
  __shared__ unsigned ncnt[256 * kSortTiles];  // next pass: [digit][destination tile]
  const int t = blockIdx.x, tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  unsigned fm = 0;
  for (int k = 0; k < kSortTiles; ++k) fm = max(fm, s.fmaxT[k]);
  const int passes = (32 - __clz(fm) + 7) / 8;
  if (P >= passes) return;  // uniform over the grid
  // this digit's counts over the tiles: total, and in the tiles before t
  const uint4* hc = reinterpret_cast<const uint4*>(s.hcnt + ((size_t)P * 256 + tid) * kSortTiles);
  unsigned tot = 0, pre = 0;
#pragma unroll
  for (int q = 0; q < kSortTiles / 4; ++q) {
    const uint4 v = hc[q];
    const unsigned c4[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      tot += c4[r];
      pre += 4 * q + r < t ? c4[r] : 0u;
    }
  }
  // digit starts (exclusive scan of the totals over the 256 digits), item
  // count and, for pass 0, the items of the tiles before t
  unsigned x = tot, zp = pre;
  for (int o = 1; o < 64; o <<= 1) {
    const unsigned y = (unsigned)__shfl_up((int)x, o, 64);
    if (lane >= o) x += y;
  }
  for (int o = 32; o > 0; o >>= 1) zp += (unsigned)__shfl_xor((int)zp, o, 64);
  if (lane == 63) sm32[wave] = x;
  if (lane == 0) sm32[4 + wave] = zp;
  for (int d = lane; d < 256; d += 64) wcnt[wave][d] = 0;
  for (int i = tid; i < 256 * kSortTiles; i += 256) ncnt[i] = 0;
  __syncthreads();
  unsigned before = 0, n = 0, zbase = 0;
  for (int w = 0; w < 4; ++w) {
    before += w < wave ? sm32[w] : 0u;
    n += sm32[w];
    zbase += sm32[4 + w];
  }
  const unsigned start = before + x - tot + pre;  // digit tid's first slot for tile t
  if (P > 0 && (unsigned)t * kSortTile >= n) return;  // uniform over the block
  const uint32_t* ksrc = (P & 1) ? s.keyB : s.keyA;
  const uint32_t* vsrc = (P & 1) ? s.valB : s.valA;
  uint32_t* kdst = (P & 1) ? s.keyA : s.keyB;
  uint32_t* vdst = (P & 1) ? s.valA : s.valB;
  constexpr int K = kSortTile / 256;  // 64-item groups per wavefront
  const unsigned i0 = (unsigned)t * kSortTile + wave * (64 * K);
  uint32_t key[K], val[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const unsigned i = i0 + 64 * k + lane;
    if (P == 0) {
      key[k] = hist[i];
      val[k] = 0;
    } else {
      key[k] = ksrc[min(i, n - 1)];
      val[k] = vsrc[min(i, n - 1)];
    }
  }
  const int shift = 8 * P;
  unsigned nz = 0;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const bool valid = P == 0 ? key[k] != 0 : i0 + 64 * k + lane < n;
    const uint64_t peers = match_digit((key[k] >> shift) & 255u, 8, valid);
    if (valid && __popcll(peers & lanemask_lt()) == 0)
      wcnt[wave][(key[k] >> shift) & 255u] += __popcll(peers);
    nz += __popcll(__ballot(valid));
    wave_lds_fence();
  }
  if (lane == 0) nzw[wave] = nz;
  __syncthreads();
  {
    unsigned run = start;
    for (int w = 0; w < 4; ++w) {
      const unsigned c = wcnt[w][tid];
      wcnt[w][tid] = run;
      run += c;
    }
  }
  unsigned zrun = zbase;
  for (int w = 0; w < wave; ++w) zrun += nzw[w];
  __syncthreads();
  const bool count_next = P + 1 < kSortPasses && P + 1 < passes;
  uint32_t* hnext = s.hcnt + (size_t)(P + 1) * 256 * kSortTiles;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const bool valid = P == 0 ? key[k] != 0 : i0 + 64 * k + lane < n;
    const unsigned d = (key[k] >> shift) & 255u;
    const uint64_t peers = match_digit(d, 8, valid);
    const unsigned r = __popcll(peers & lanemask_lt());
    const unsigned pos = valid ? wcnt[wave][d] + r : 0u;
    if (P == 0) {
      const uint64_t vm = __ballot(valid);
      const unsigned zpos = zrun + __popcll(vm & lanemask_lt());
      zrun += __popcll(vm);
      if (valid) {
        s.symAsc[zpos] = i0 + 64 * k + lane;
        s.freqAsc[zpos] = key[k];
      }
      val[k] = zpos;
    }
    if (valid) {
      kdst[pos] = key[k];
      vdst[pos] = val[k];
      if (count_next)
        atomicAdd(&ncnt[((key[k] >> (shift + 8)) & 255u) * kSortTiles + pos / kSortTile], 1u);
    }
    wave_lds_fence();
    if (valid && r == 0) wcnt[wave][d] = pos + __popcll(peers);
    wave_lds_fence();
  }
  if (count_next) {
    __syncthreads();
    for (int i = tid; i < 256 * kSortTiles; i += 256)
      if (ncnt[i]) atomicAdd(&hnext[i], ncnt[i]);
  }
}

// ---------------------------------------------------------------- encoding
// Lane l of the chunk's wavefront owns symbols [l*per, (l+1)*per) of the
// chunk; symbols and their code lengths are fetched in groups of 8 with all
// loads in flight before use.
// With zc != nullptr (C = 1024, 16 symbols a lane) the pass also records
// where the escape symbol (0) occurs: zc[chunk] = escapes in the chunk and,
// for chunks that have any, zl[64 chunk + lane] = the lane's 16-bit mask of
// escapes | (escapes in the chunk's earlier lanes) << 16, from which the
// escaped values are put in stream order without sorting.
__device__ __forceinline__ void chunk_words_body(const uint16_t* __restrict__ sym, int64_t N,
                                                 int C, const uint8_t* __restrict__ clen,
                                                 uint32_t* __restrict__ cw,
                                                 const Layout* __restrict__ lay, uint32_t blk,
                                                 uint32_t nblk, uint32_t* __restrict__ zc = nullptr,
                                                 uint32_t* __restrict__ zl = nullptr) {
  // the code lengths of all 65536 symbols in LDS (one 16-byte load per
  // thread per 4 KiB), then chunk groups of four in a block-stride loop
  __shared__ __align__(16) uint8_t ln[kDict];
  if (lay->status) return;
  {
    const uint4* src = reinterpret_cast<const uint4*>(clen);
    uint4* dst = reinterpret_cast<uint4*>(ln);
    uint4 v[kDict / 16 / 256];
#pragma unroll
    for (int u = 0; u < kDict / 16 / 256; ++u) v[u] = src[u * 256 + threadIdx.x];
#pragma unroll
    for (int u = 0; u < kDict / 16 / 256; ++u) dst[u * 256 + threadIdx.x] = v[u];
  }
  __syncthreads();
  const int64_t n_chunks = (N + C - 1) / C;
  const int lane = threadIdx.x & 63;
  const int per = C / 64;
  for (int64_t chunk = (int64_t)blk * 4 + (threadIdx.x >> 6); chunk < n_chunks;
       chunk += (int64_t)nblk * 4) {
    const int64_t a = chunk * C + (int64_t)lane * per;
    const int64_t end = min<int64_t>(chunk * C + C, N);
    unsigned bits = 0, esc = 0;
    if (per == 16 && a + 16 <= end && (reinterpret_cast<uintptr_t>(sym) & 15) == 0) {
      const uint4* p = reinterpret_cast<const uint4*>(sym + a);
      const uint4 x0 = p[0], x1 = p[1];
      const unsigned w[8] = {x0.x, x0.y, x0.z, x0.w, x1.x, x1.y, x1.z, x1.w};
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        bits += (unsigned)ln[w[k] & 0xFFFFu] + ln[w[k] >> 16];
        esc |= ((w[k] & 0xFFFFu) == 0u ? 1u : 0u) << (2 * k);
        esc |= ((w[k] >> 16) == 0u ? 1u : 0u) << (2 * k + 1);
      }
    } else {
      for (int64_t i = a; i < min<int64_t>(a + per, end); ++i) {
        const uint16_t v = sym[i];
        bits += ln[v];
        if (v == 0 && i - a < 32) esc |= 1u << (i - a);
      }
    }
    for (int o = 32; o > 0; o >>= 1) bits += (unsigned)__shfl_xor((int)bits, o, 64);
    if (lane == 0) cw[chunk] = (bits + 31u) >> 5;
    if (zc) {
      const unsigned cnt = (unsigned)__popc(esc);
      unsigned incl = cnt;
      for (int o = 1; o < 64; o <<= 1) {
        const unsigned y = (unsigned)__shfl_up((int)incl, o, 64);
        if (lane >= o) incl += y;
      }
      const unsigned total = (unsigned)__shfl((int)incl, 63, 64);
      if (total) zl[chunk * 64 + lane] = esc | ((incl - cnt) << 16);
      if (lane == 0) zc[chunk] = total;
    }
  }
}

__global__ __launch_bounds__(256) void k_chunk_words(const uint16_t* __restrict__ sym, int64_t N,
                                                      int C, const uint8_t* __restrict__ clen,
                                                      uint32_t* __restrict__ cw,
                                                      const Layout* __restrict__ lay,
                                                      const unsigned* __restrict__ gate,
                                                      uint32_t* __restrict__ zc,
                                                      uint32_t* __restrict__ zl) {
  if (gate_closed(gate)) return;
  chunk_words_body(sym, N, C, clen, cw, lay, blockIdx.x, gridDim.x, zc, zl);
}

__device__ __forceinline__ void layout_scan_body(const uint32_t* __restrict__ cw,
                                                 int64_t n_chunks, uint8_t* __restrict__ out,
                                                 uint64_t cb_off, Layout* __restrict__ lay,
                                                 const unsigned long long* n_out,
                                                 uint64_t out_cap_n, int huff_only) {
  __shared__ unsigned long long carry;
  const int tid = threadIdx.x;
  const unsigned long long n_codes = lay->n_codes;
  const unsigned long long no = huff_only ? 0ull : *n_out;
  if (no > out_cap_n) {
    if (tid == 0) {
      lay->n_outliers = no;
      lay->status |= ST_OVERFLOW;
    }
    return;
  }
  const unsigned long long off = pad8(cb_off + 3 * n_codes);
  const unsigned long long opos = off + 8ull * (n_chunks + 1);
  const unsigned long long oval = opos + 8ull * no;
  const unsigned long long words = oval + 8ull * no;
  uint64_t* offs = reinterpret_cast<uint64_t*>(out + off);
  // batches of 16384 chunks: sub-tile s (4096 chunks) gives thread t the
  // four consecutive chunks 4t .. 4t+3, so every load and store of a wave
  // is contiguous; all sixteen loads of a thread are in flight together and
  // one block scan (four values per thread) serves the whole batch
  __shared__ unsigned wsum[16][4];
  const int wave = tid >> 6, lane = tid & 63;
  unsigned long long base = 0;
  const bool vec = (reinterpret_cast<uintptr_t>(cw) & 15) == 0;
  for (int64_t b0 = 0; b0 < n_chunks; b0 += 16384) {
    unsigned v[4][4];
#pragma unroll
    for (int sb = 0; sb < 4; ++sb) {
      const int64_t e = b0 + 4096 * sb + 4 * tid;
      if (vec && e + 3 < n_chunks) {
        const uint4 q = *reinterpret_cast<const uint4*>(cw + e);
        v[sb][0] = q.x;
        v[sb][1] = q.y;
        v[sb][2] = q.z;
        v[sb][3] = q.w;
      } else {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const unsigned x = cw[min<int64_t>(e + u, n_chunks - 1)];
          v[sb][u] = e + u < n_chunks ? x : 0u;
        }
      }
    }
    unsigned sum[4], incl[4];
#pragma unroll
    for (int sb = 0; sb < 4; ++sb) {
      sum[sb] = v[sb][0] + v[sb][1] + v[sb][2] + v[sb][3];
      incl[sb] = sum[sb];
    }
    for (int o = 1; o < 64; o <<= 1) {
#pragma unroll
      for (int sb = 0; sb < 4; ++sb) {
        const unsigned y = (unsigned)__shfl_up((int)incl[sb], o, 64);
        if (lane >= o) incl[sb] += y;
      }
    }
    if (lane == 63) {
#pragma unroll
      for (int sb = 0; sb < 4; ++sb) wsum[wave][sb] = incl[sb];
    }
    __syncthreads();
    unsigned before[4] = {0u, 0u, 0u, 0u}, tot[4] = {0u, 0u, 0u, 0u};
    for (int w = 0; w < 16; ++w) {
#pragma unroll
      for (int sb = 0; sb < 4; ++sb) {
        const unsigned c = wsum[w][sb];
        before[sb] += w < wave ? c : 0u;
        tot[sb] += c;
      }
    }
    unsigned long long run = base;
#pragma unroll
    for (int sb = 0; sb < 4; ++sb) {
      const int64_t e = b0 + 4096 * sb + 4 * tid;
      unsigned long long r = run + before[sb] + (incl[sb] - sum[sb]);
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (e + u < n_chunks) offs[e + u] = r;
        r += v[sb][u];
      }
      run += tot[sb];
    }
    base = run;
    __syncthreads();
  }
  const unsigned long long total = base;
  if (tid == 0) carry = total;
  __syncthreads();
  if (tid == 0) {
    const unsigned long long nw = carry;
    offs[n_chunks] = nw;
    lay->n_outliers = no;
    lay->n_words = nw;
    lay->cb = cb_off;
    lay->off = off;
    lay->opos = opos;
    lay->oval = oval;
    lay->words = words;
    lay->end = pad8(words + 4ull * nw);
  }
}

__global__ __launch_bounds__(1024) void k_layout_scan(const uint32_t* __restrict__ cw,
                                                       int64_t n_chunks, uint8_t* __restrict__ out,
                                                       uint64_t cb_off, Layout* __restrict__ lay,
                                                       const unsigned long long* n_out,
                                                       uint64_t out_cap_n, int huff_only,
                                                       const unsigned* __restrict__ gate) {
  if (gate_closed(gate)) return;
  layout_scan_body(cw, n_chunks, out, cb_off, lay, n_out, out_cap_n, huff_only);
}

// The same layout and offsets from many blocks (large arrays): block b owns
// the chunks [b R, (b + 1) R).  k_scan_sums writes each range's word total;
// k_scan_offsets adds the totals of the ranges before its own to an
// exclusive scan of its range (256 threads, four consecutive chunks each,
// sixteen loads in flight), and block 0 writes the layout.
constexpr int kScanThreads = 256;
constexpr int kScanBlocksMax = kScanSumWords / 2;

__device__ __forceinline__ unsigned long long block_sum_u64(unsigned long long v,
                                                            unsigned long long* sm) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = v;
  __syncthreads();
  unsigned long long t = 0;
  for (int w = 0; w < kScanThreads / 64; ++w) t += sm[w];
  __syncthreads();
  return t;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_sums(const uint32_t* __restrict__ cw,
                                                            int64_t n_chunks, int64_t R,
                                                            unsigned long long* __restrict__ sums,
                                                            const unsigned* __restrict__ gate) {
  if (gate_closed(gate)) return;
  __shared__ unsigned long long sm[kScanThreads / 64];
  const int64_t lo = (int64_t)blockIdx.x * R, hi = min<int64_t>(lo + R, n_chunks);
  unsigned long long acc = 0;
  for (int64_t i0 = lo + threadIdx.x; i0 < hi; i0 += 8 * kScanThreads) {
    uint32_t v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = cw[min<int64_t>(i0 + u * kScanThreads, hi - 1)];
#pragma unroll
    for (int u = 0; u < 8; ++u) acc += i0 + u * kScanThreads < hi ? v[u] : 0u;
  }
  acc = block_sum_u64(acc, sm);
  if (threadIdx.x == 0) sums[blockIdx.x] = acc;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_offsets(
    const uint32_t* __restrict__ cw, int64_t n_chunks, int64_t R,
    const unsigned long long* __restrict__ sums, uint8_t* __restrict__ out, uint64_t cb_off,
    Layout* __restrict__ lay, const unsigned long long* n_out, uint64_t out_cap_n,
    int huff_only, const unsigned* __restrict__ gate) {
  if (gate_closed(gate)) return;
  __shared__ unsigned long long sm[kScanThreads / 64];
  __shared__ unsigned wsum[kScanThreads / 64][4];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const unsigned long long n_codes = lay->n_codes;
  const unsigned long long no = huff_only ? 0ull : *n_out;
  if (no > out_cap_n) {
    if (blockIdx.x == 0 && tid == 0) {
      lay->n_outliers = no;
      lay->status |= ST_OVERFLOW;
    }
    return;
  }
  const unsigned long long off = pad8(cb_off + 3 * n_codes);
  const unsigned long long opos = off + 8ull * (n_chunks + 1);
  const unsigned long long oval = opos + 8ull * no;
  const unsigned long long words = oval + 8ull * no;
  uint64_t* offs = reinterpret_cast<uint64_t*>(out + off);
  // the word totals of the ranges before this block's, and of all ranges
  unsigned long long pre = 0, all = 0;
  for (int b = tid; b < (int)gridDim.x; b += kScanThreads) {
    const unsigned long long v = sums[b];
    all += v;
    pre += b < (int)blockIdx.x ? v : 0ull;
  }
  pre = block_sum_u64(pre, sm);
  all = block_sum_u64(all, sm);
  const int64_t lo = (int64_t)blockIdx.x * R, hi = min<int64_t>(lo + R, n_chunks);
  unsigned long long base = pre;
  constexpr int TB = 4 * kScanThreads;  // chunks per sub-tile
  for (int64_t b0 = lo; b0 < hi; b0 += 4 * TB) {
    unsigned v[4][4];
#pragma unroll
    for (int sb = 0; sb < 4; ++sb) {
      const int64_t e = b0 + TB * sb + 4 * tid;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const unsigned x = cw[min<int64_t>(e + u, hi - 1)];
        v[sb][u] = e + u < hi ? x : 0u;
      }
    }
    unsigned sum[4], incl[4];
#pragma unroll
    for (int sb = 0; sb < 4; ++sb) {
      sum[sb] = v[sb][0] + v[sb][1] + v[sb][2] + v[sb][3];
      incl[sb] = sum[sb];
    }
    for (int o = 1; o < 64; o <<= 1) {
#pragma unroll
      for (int sb = 0; sb < 4; ++sb) {
        const unsigned y = (unsigned)__shfl_up((int)incl[sb], o, 64);
        if (lane >= o) incl[sb] += y;
      }
    }
    if (lane == 63) {
#pragma unroll
      for (int sb = 0; sb < 4; ++sb) wsum[wave][sb] = incl[sb];
    }
    __syncthreads();
    unsigned before[4] = {0u, 0u, 0u, 0u}, tot[4] = {0u, 0u, 0u, 0u};
    for (int w = 0; w < kScanThreads / 64; ++w) {
#pragma unroll
      for (int sb = 0; sb < 4; ++sb) {
        const unsigned c = wsum[w][sb];
        before[sb] += w < wave ? c : 0u;
        tot[sb] += c;
      }
    }
    unsigned long long run = base;
#pragma unroll
    for (int sb = 0; sb < 4; ++sb) {
      const int64_t e = b0 + TB * sb + 4 * tid;
      unsigned long long r = run + before[sb] + (incl[sb] - sum[sb]);
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (e + u < hi) offs[e + u] = r;
        r += v[sb][u];
      }
      run += tot[sb];
    }
    base = run;
    __syncthreads();
  }
  if (blockIdx.x == 0 && tid == 0) {
    offs[n_chunks] = all;
    lay->n_outliers = no;
    lay->n_words = all;
    lay->cb = cb_off;
    lay->off = off;
    lay->opos = opos;
    lay->oval = oval;
    lay->words = words;
    lay->end = pad8(words + 4ull * all);
  }
}

__device__ __forceinline__ void outlier_sort_body(const OutlierBuf& ob, uint32_t* keyA,
                                                  uint32_t* valA, uint32_t* keyB,
                                                  uint32_t* valB, int key_bits,
                                                  uint8_t* __restrict__ out,
                                                  const Layout* __restrict__ lay) {
  __shared__ SortSmem sm;
  if (lay->status) return;
  const uint32_t n = (uint32_t)lay->n_outliers;
  if (n == 0) return;
  for (uint32_t i = threadIdx.x; i < n; i += 1024) {
    keyA[i] = ob.pos[i];
    valA[i] = i;
  }
  __syncthreads();
  const bool inB = block_radix_sort(keyA, valA, keyB, valB, n, key_bits, sm);
  const uint32_t* ks = inB ? keyB : keyA;
  const uint32_t* vs = inB ? valB : valA;
  uint64_t* op = reinterpret_cast<uint64_t*>(out + lay->opos);
  int64_t* ov = reinterpret_cast<int64_t*>(out + lay->oval);
  for (uint32_t i = threadIdx.x; i < n; i += 1024) {
    op[i] = ks[i];
    ov[i] = ob.val[vs[i]];
  }
}

__global__ __launch_bounds__(1024) void k_outlier_sort(const OutlierBuf ob, uint32_t* keyA,
                                                        uint32_t* valA, uint32_t* keyB,
                                                        uint32_t* valB, int key_bits,
                                                        uint8_t* __restrict__ out,
                                                        const Layout* __restrict__ lay,
                                                        const unsigned* __restrict__ gate) {
  if (gate_closed(gate)) return;
  outlier_sort_body(ob, keyA, valA, keyB, valB, key_bits, out, lay);
}

// --------------------------------------------- escaped values in stream order
// The level kernels append escaped values (stream position, value) in no
// particular order.  Their order in the stream is that of the escape
// symbols, so a value's rank is the number of escapes before its position:
// the exclusive sum of the per-chunk counts (zpre) plus the escapes of the
// chunk's earlier lanes and of the lane's symbols before it (zl).  The sums
// over chunks run on many blocks: range totals, then range scans offset by
// the totals before them.
constexpr int kEscThreads = 256;
__global__ __launch_bounds__(kEscThreads) void k_esc_sums(const uint32_t* __restrict__ zc,
                                                          int64_t n_chunks, int64_t R,
                                                          uint32_t* __restrict__ sums,
                                                          const Layout* __restrict__ lay,
                                                          const unsigned* __restrict__ gate) {
  if (gate_closed(gate) || lay->status) return;
  __shared__ unsigned long long sm[kScanThreads / 64];
  const int64_t lo = (int64_t)blockIdx.x * R, hi = min<int64_t>(lo + R, n_chunks);
  unsigned long long acc = 0;
  for (int64_t i = lo + threadIdx.x; i < hi; i += kEscThreads) acc += zc[i];
  acc = block_sum_u64(acc, sm);
  if (threadIdx.x == 0) sums[blockIdx.x] = (uint32_t)acc;
}

__global__ __launch_bounds__(kEscThreads) void k_esc_prefix(const uint32_t* __restrict__ zc,
                                                            int64_t n_chunks, int64_t R,
                                                            const uint32_t* __restrict__ sums,
                                                            uint32_t* __restrict__ zpre,
                                                            const Layout* __restrict__ lay,
                                                            const unsigned* __restrict__ gate) {
  if (gate_closed(gate) || lay->status) return;
  __shared__ unsigned long long sm[kScanThreads / 64];
  __shared__ uint32_t wtot[kEscThreads / 64];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  unsigned long long pre = 0;
  for (int b = tid; b < (int)blockIdx.x; b += kEscThreads) pre += sums[b];
  pre = block_sum_u64(pre, sm);
  const int64_t lo = (int64_t)blockIdx.x * R, hi = min<int64_t>(lo + R, n_chunks);
  uint32_t base = (uint32_t)pre;
  for (int64_t t0 = lo; t0 < hi; t0 += kEscThreads) {
    const int64_t i = t0 + tid;
    const uint32_t v = i < hi ? zc[i] : 0u;
    uint32_t incl = v;
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = (uint32_t)__shfl_up((int)incl, o, 64);
      if (lane >= o) incl += y;
    }
    if (lane == 63) wtot[wave] = incl;
    __syncthreads();
    uint32_t before = 0, all = 0;
    for (int w = 0; w < kEscThreads / 64; ++w) {
      before += w < wave ? wtot[w] : 0u;
      all += wtot[w];
    }
    if (i < hi) zpre[i] = base + before + incl - v;
    base += all;
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void k_esc_place(const OutlierBuf ob,
                                                   const uint32_t* __restrict__ zpre,
                                                   const uint32_t* __restrict__ zl,
                                                   uint8_t* __restrict__ out,
                                                   Layout* __restrict__ lay,
                                                   unsigned* __restrict__ status,
                                                   const unsigned* __restrict__ gate) {
  if (gate_closed(gate) || lay->status) return;
  const uint64_t n = lay->n_outliers;
  uint64_t* op = reinterpret_cast<uint64_t*>(out + lay->opos);
  int64_t* ov = reinterpret_cast<int64_t*>(out + lay->oval);
  for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * 256) {
    const uint32_t pos = ob.pos[i];
    const uint32_t chunk = pos >> 10, j = pos & 1023u;
    const uint32_t e = zl[(size_t)chunk * 64 + (j >> 4)];
    const uint32_t t = j & 15u;
    const uint64_t rank = (uint64_t)zpre[chunk] + (e >> 16) + (uint32_t)__popc(e & ((1u << t) - 1u));
    if (((e >> t) & 1u) == 0u || rank >= n) {
      atomicOr(status, ST_INTERNAL);
      continue;
    }
    op[rank] = pos;
    ov[rank] = ob.val[i];
  }
}

// One wavefront per chunk, four chunks per block; LDS holds each chunk's
// words while codes are OR-ed into place.
// wbuf: dynamic LDS of 4 * C words.
// OR code c of length l at bit position bitpos of the chunk's LDS words.
__device__ __forceinline__ void put_code(uint32_t* w, unsigned bitpos, uint32_t c, unsigned l) {
  const unsigned wi = bitpos >> 5, o = bitpos & 31u;
  if (o + l <= 32u) {
    atomicOr(&w[wi], c << (32u - o - l));
  } else {
    atomicOr(&w[wi], c >> (o + l - 32u));
    atomicOr(&w[wi + 1], c << (64u - o - l));
  }
}

__device__ __forceinline__ void encode_body(const uint16_t* __restrict__ sym, int64_t N, int C,
                                            const uint32_t* __restrict__ code,
                                            const uint8_t* __restrict__ clen,
                                            const uint32_t* __restrict__ pk,
                                            uint8_t* __restrict__ out,
                                            const Layout* __restrict__ lay, uint32_t blk,
                                            uint32_t* wbuf) {
  if (lay->status) return;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t n_chunks = (N + C - 1) / C;
  const int64_t chunk = (int64_t)blk * 4 + wave;
  uint32_t* w = wbuf + wave * C;
  __shared__ uint32_t fst[kMaxCodeLen + 1];  // first code of each length
  for (int i = lane; i < C; i += 64) w[i] = 0;
  if (threadIdx.x <= kMaxCodeLen) fst[threadIdx.x] = pk[kDict + threadIdx.x];
  __syncthreads();
  const uint64_t* offs = reinterpret_cast<const uint64_t*>(out + lay->off);
  uint32_t* words = reinterpret_cast<uint32_t*>(out + lay->words);
  const bool live = chunk < n_chunks;
  const int per = C / 64;
  const int64_t a = live ? chunk * C + (int64_t)lane * per : 0;
  const int64_t end = live ? min<int64_t>(chunk * C + C, N) : 0;
  if (per == 16) {
    // sixteen symbols per lane in two 16-byte loads (element loads at the
    // array's end), one packed (rank, length) word each
    uint32_t cl[16];
    if (a + 16 <= end && (reinterpret_cast<uintptr_t>(sym) & 15) == 0) {
      const uint4* p = reinterpret_cast<const uint4*>(sym + a);
      const uint4 x0 = p[0], x1 = p[1];
      const unsigned v[8] = {x0.x, x0.y, x0.z, x0.w, x1.x, x1.y, x1.z, x1.w};
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        cl[2 * k] = pk[v[k] & 0xFFFFu];
        cl[2 * k + 1] = pk[v[k] >> 16];
      }
    } else {
#pragma unroll
      for (int k = 0; k < 16; ++k) cl[k] = a + k < end ? pk[sym[a + k]] : 0u;
    }
    unsigned my_bits = 0;
#pragma unroll
    for (int k = 0; k < 16; ++k) my_bits += cl[k] & 63u;
    unsigned x = my_bits;
    for (int o = 1; o < 64; o <<= 1) {
      const unsigned y = (unsigned)__shfl_up((int)x, o, 64);
      if (lane >= o) x += y;
    }
    unsigned bitpos = x - my_bits;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const unsigned l = cl[k] & 63u;
      if (l == 0) continue;
      put_code(w, bitpos, fst[l] + (cl[k] >> 6), l);
      bitpos += l;
    }
    __syncthreads();
    if (live) {
      const uint64_t w0 = offs[chunk], nw = offs[chunk + 1] - w0;
      for (uint64_t i = lane; i < nw; i += 64) words[w0 + i] = w[i];
    }
    return;
  }
  // pass 1: bit count of this lane's symbols
  unsigned my_bits = 0;
  for (int k0 = 0; k0 < per; k0 += 8) {
    unsigned sy[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) sy[u] = (k0 + u < per && a + k0 + u < end) ? sym[a + k0 + u] : 0xFFFFFFFFu;
#pragma unroll
    for (int u = 0; u < 8; ++u) my_bits += sy[u] != 0xFFFFFFFFu ? clen[sy[u]] : 0u;
  }
  // exclusive prefix over lanes
  unsigned x = my_bits;
  for (int o = 1; o < 64; o <<= 1) {
    const unsigned y = (unsigned)__shfl_up((int)x, o, 64);
    if (lane >= o) x += y;
  }
  unsigned bitpos = x - my_bits;
  // pass 2: OR the codes into the chunk's words
  for (int k0 = 0; k0 < per; k0 += 8) {
    unsigned sy[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) sy[u] = (k0 + u < per && a + k0 + u < end) ? sym[a + k0 + u] : 0xFFFFFFFFu;
    uint32_t cd[8];
    unsigned ln[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      cd[u] = sy[u] != 0xFFFFFFFFu ? code[sy[u]] : 0u;
      ln[u] = sy[u] != 0xFFFFFFFFu ? clen[sy[u]] : 0u;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const unsigned l = ln[u];
      if (l == 0) continue;
      put_code(w, bitpos, cd[u], l);
      bitpos += l;
    }
  }
  __syncthreads();
  if (live) {
    const uint64_t w0 = offs[chunk], nw = offs[chunk + 1] - w0;
    for (uint64_t i = lane; i < nw; i += 64) words[w0 + i] = w[i];
  }
}

__global__ __launch_bounds__(256) void k_encode(const uint16_t* __restrict__ sym, int64_t N, int C,
                                                 const uint32_t* __restrict__ code,
                                                 const uint8_t* __restrict__ clen,
                                                 const uint32_t* __restrict__ pk,
                                                 uint8_t* __restrict__ out,
                                                 const Layout* __restrict__ lay,
                                                 const unsigned* __restrict__ gate) {
  if (gate_closed(gate)) return;
  extern __shared__ uint32_t wbuf[];  // 4 * C words
  encode_body(sym, N, C, code, clen, pk, out, lay, blockIdx.x, wbuf);
}

// Encoder for large arrays (chunks of 1024 symbols): persistent blocks of
// kEncWaves wavefronts, one chunk per wavefront at a time.  The packed
// (rank << 6 | length) words of the kEncWin symbols around the dictionary
// centre (|k| < kEncWin/2, nearly all of them) are copied into LDS once per
// block, so a symbol's code (the first code of its length plus its rank) is
// two LDS reads; the rest come from the global table.  Symbols are loaded two chunks ahead and the global look-ups of
// the next chunk are issued before the current chunk is coded, so neither
// waits on memory in the steady state (a look-up of an in-window symbol
// reads one shared, cached word instead).  Each wavefront ORs its chunk's
// codes into its own LDS words and copies them out; no block barriers.
constexpr int kEncWin = 20480;
constexpr uint32_t kEncLo = kHalf - kEncWin / 2;
constexpr int kEncWaves = 16;
constexpr int kEncC = 1024;

__host__ __device__ constexpr size_t enc_win_lds_bytes() {
  return (size_t)(kEncWin + kEncWaves * kEncC) * sizeof(uint32_t);
}

struct EncSyms {
  uint32_t v[8];  // 16 symbols, two per word (low half first)
  int n;          // symbols of this lane inside the array
};

__global__ __launch_bounds__(64 * kEncWaves) void k_encode_win(
    const uint16_t* __restrict__ sym, int64_t N, const uint32_t* __restrict__ pk,
    uint8_t* __restrict__ out, const Layout* __restrict__ lay, const unsigned* __restrict__ gate) {
  if (gate_closed(gate)) return;
  extern __shared__ __align__(16) uint32_t esm[];
  __shared__ uint32_t fst[kMaxCodeLen + 1];  // first code of each length
  if (lay->status) return;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  uint32_t* tab = esm;
  uint32_t* w = esm + kEncWin + wave * kEncC;
  const int64_t n_chunks = (N + kEncC - 1) / kEncC;
  const uint64_t* offs = reinterpret_cast<const uint64_t*>(out + lay->off);
  uint32_t* words = reinterpret_cast<uint32_t*>(out + lay->words);
  const int64_t stride = (int64_t)gridDim.x * kEncWaves;
  if (threadIdx.x <= kMaxCodeLen) fst[threadIdx.x] = pk[kDict + threadIdx.x];
  {
    const uint4* src = reinterpret_cast<const uint4*>(pk + kEncLo);
    uint4* dst = reinterpret_cast<uint4*>(tab);
    constexpr int NV = kEncWin / 4 / (64 * kEncWaves) + 1;
    uint4 t[NV];
#pragma unroll
    for (int u = 0; u < NV; ++u) {
      const int i = min<int>(u * 64 * kEncWaves + threadIdx.x, kEncWin / 4 - 1);
      t[u] = src[i];
    }
#pragma unroll
    for (int u = 0; u < NV; ++u) {
      const int i = u * 64 * kEncWaves + threadIdx.x;
      if (i < kEncWin / 4) dst[i] = t[u];
    }
  }
  __syncthreads();
  // 16 symbols of lane `lane` in chunk c (whole-vector loads inside the array)
  auto load_syms = [&](int64_t c, EncSyms& e) {
    const int64_t a = c * kEncC + lane * 16;
    const int64_t cl = min<int64_t>(c, n_chunks - 1);
    e.n = c < n_chunks ? (int)max<int64_t>(0, min<int64_t>(16, N - a)) : 0;
    if (e.n == 16) {
      const uint4* p = reinterpret_cast<const uint4*>(sym + a);
      const uint4 x0 = p[0], x1 = p[1];
      e.v[0] = x0.x; e.v[1] = x0.y; e.v[2] = x0.z; e.v[3] = x0.w;
      e.v[4] = x1.x; e.v[5] = x1.y; e.v[6] = x1.z; e.v[7] = x1.w;
    } else {
      const int64_t b = cl * kEncC + lane * 16;
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const uint32_t lo = 2 * k < e.n ? sym[b + 2 * k] : 0u;
        const uint32_t hi = 2 * k + 1 < e.n ? sym[b + 2 * k + 1] : 0u;
        e.v[k] = lo | (hi << 16);
      }
    }
  };
  auto sym_at = [](const EncSyms& e, int k) -> uint32_t {
    return (k & 1) ? (e.v[k >> 1] >> 16) : (e.v[k >> 1] & 0xFFFFu);
  };
  // global look-ups of the symbols outside the window (a shared word otherwise)
  auto gather = [&](const EncSyms& e, uint32_t (&g)[16]) {
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const uint32_t s = sym_at(e, k);
      g[k] = pk[s - kEncLo < (uint32_t)kEncWin ? kHalf : s];
    }
  };
  auto emit = [&](int64_t c, uint64_t w0, uint64_t nw) {
    wave_lds_fence();
    if (c < n_chunks)
      for (uint64_t i = lane; i < nw; i += 64) words[w0 + i] = w[i];
    wave_lds_fence();
  };
  auto zero_words = [&]() {
    uint4* z = reinterpret_cast<uint4*>(w);
#pragma unroll
    for (int k = 0; k < kEncC / 4 / 64; ++k) z[k * 64 + lane] = make_uint4(0u, 0u, 0u, 0u);
  };
  auto scan_bits = [&](unsigned my_bits) -> unsigned {
    unsigned x = my_bits;
    for (int o = 1; o < 64; o <<= 1) {
      const unsigned y = (unsigned)__shfl_up((int)x, o, 64);
      if (lane >= o) x += y;
    }
    return x - my_bits;
  };
  int64_t c = (int64_t)blockIdx.x * kEncWaves + wave;
  if (c >= n_chunks) return;
  EncSyms s0, s1, s2;
  uint32_t g0[16], g1[16];
  uint64_t o0a, o0b, o1a, o1b;
  load_syms(c, s0);
  load_syms(c + stride, s1);
  o0a = offs[c];
  o0b = offs[c + 1];
  {
    const int64_t cn = min<int64_t>(c + stride, n_chunks - 1);
    o1a = offs[cn];
    o1b = offs[cn + 1];
  }
  gather(s0, g0);
  for (; c < n_chunks; c += stride) {
    load_syms(c + 2 * stride, s2);
    gather(s1, g1);
    // code chunk c
    zero_words();
    uint32_t cl[16];
    unsigned my_bits = 0;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const uint32_t d = sym_at(s0, k) - kEncLo;
      const uint32_t e = d < (uint32_t)kEncWin ? tab[d] : g0[k];
      cl[k] = k < s0.n ? e : 0u;
      my_bits += cl[k] & 63u;
    }
    unsigned bitpos = scan_bits(my_bits);
    wave_lds_fence();
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const unsigned l = cl[k] & 63u;
      if (l == 0) continue;
      put_code(w, bitpos, fst[l] + (cl[k] >> 6), l);
      bitpos += l;
    }
    emit(c, o0a, o0b - o0a);
    // rotate the pipeline
    s0 = s1;
    s1 = s2;
#pragma unroll
    for (int k = 0; k < 16; ++k) g0[k] = g1[k];
    o0a = o1a;
    o0b = o1b;
    {
      const int64_t cn = min<int64_t>(c + 2 * stride, n_chunks - 1);
      o1a = offs[cn];
      o1b = offs[cn + 1];
    }
  }
}

// Header, bins and result words of one compression (thread 0 of a block),
// from the status bits st of the range pass and the quantiser and the
// stream layout.  Constant and empty arrays get the 136-byte trivial stream
// (header and one zero bin); a failed compression writes no stream and
// reports MGC_EINVAL (non-finite input), MGC_ERANGE (no budget left, or a
// quantised value out of range), MGC_ENOSPC with the escaped-value count it
// needs, or MGC_EDEVICE.  Results: *size_out = stream bytes (or that count),
// *status_out = the mgc_status.
template <typename St>
__device__ void header_body(Header h, uint8_t* __restrict__ out, const double* __restrict__ bud,
                            int L, unsigned st, const Layout* __restrict__ lay,
                            uint64_t* size_out, St* status_out) {
  if (st & (ST_EMPTY | ST_CONST)) {
    h.flags = (st & ST_EMPTY) ? FLAG_EMPTY : FLAG_CONSTANT;
    if (!(st & ST_EMPTY)) h.const_value = bud[0];
    h.L = 0;
    h.n_chunks = 0;
    h.total = kHeaderBytes + 8;
    const uint8_t* src = reinterpret_cast<const uint8_t*>(&h);
    for (int i = 0; i < kHeaderBytes; ++i) out[i] = src[i];
    for (int i = 0; i < 8; ++i) out[kHeaderBytes + i] = 0;
    *size_out = h.total;
    *status_out = MGC_OK;
    return;
  }
  if (st & ST_NONFINITE) {
    *size_out = 0;
    *status_out = MGC_EINVAL;
    return;
  }
  if (st & ST_BUDGET) {
    *size_out = 0;
    *status_out = MGC_ERANGE;
    return;
  }
  const unsigned all = st | lay->status;
  if (all) {
    *size_out = (all & ST_OVERFLOW) ? lay->n_outliers : 0;
    *status_out = (all & ST_OVERFLOW) ? MGC_ENOSPC : (all & ST_RANGE) ? MGC_ERANGE : MGC_EDEVICE;
    return;
  }
  h.tau = bud[4];
  h.tau_eff = bud[5];
  h.n_codes = lay->n_codes;
  h.n_outliers = lay->n_outliers;
  h.n_words = lay->n_words;
  h.total = lay->end;
  const uint8_t* src = reinterpret_cast<const uint8_t*>(&h);
  for (int i = 0; i < kHeaderBytes; ++i) out[i] = src[i];
  double* q = reinterpret_cast<double*>(out + kHeaderBytes);
  for (int l = 0; l <= L; ++l) q[l] = bud[bud_q(l)];
  // zero the padding bytes after the codebook and after the words
  for (uint64_t i = lay->cb + 3 * lay->n_codes; i < lay->off; ++i) out[i] = 0;
  for (uint64_t i = lay->words + 4 * lay->n_words; i < lay->end; ++i) out[i] = 0;
  *size_out = lay->end;
  *status_out = MGC_OK;
}

// Plain compression: res[0] = mgc_status, res[1] = stream bytes (or the
// escaped-value count needed).  `empty` marks an array without values (no
// range pass ran).
__global__ void k_header(uint8_t* __restrict__ out, Header h, const double* __restrict__ bud,
                         const Layout* __restrict__ lay, const unsigned* __restrict__ status,
                         int empty, unsigned long long* __restrict__ res) {
  if (threadIdx.x != 0) return;
  const unsigned st = empty ? (unsigned)ST_EMPTY : *status;
  header_body(h, out, bud, (int)h.L, st, lay, reinterpret_cast<uint64_t*>(res + 1),
              reinterpret_cast<uint64_t*>(res));
}

__global__ void k_huff_header(uint8_t* __restrict__ out, uint32_t C, uint64_t N, uint64_t n_chunks,
                              const Layout* __restrict__ lay, unsigned long long* info) {
  if (threadIdx.x != 0) return;
  info[0] = lay->status;
  info[1] = 0;
  info[2] = lay->end;
  HuffHeader h;
  h.magic = kHuffMagic;
  h.C = C;
  h.N = N;
  h.n_codes = lay->n_codes;
  h.n_chunks = n_chunks;
  h.n_words = lay->n_words;
  h.total = lay->end;
  const uint8_t* src = reinterpret_cast<const uint8_t*>(&h);
  for (int i = 0; i < kHuffHeaderBytes; ++i) out[i] = src[i];
  for (uint64_t i = lay->cb + 3 * lay->n_codes; i < lay->off; ++i) out[i] = 0;
  for (uint64_t i = lay->words + 4 * lay->n_words; i < lay->end; ++i) out[i] = 0;
}

// ---------------------------------------------------------------- decoding
// The decoding tables from a stream's codebook section (n symbols ascending,
// then their code lengths) on kCanonBlocks blocks of four wavefronts, each
// wavefront a contiguous run of the section (as the codebook's canonical
// pass): the runs' counts per length and validity, then the per-length
// tables, the symbols in (length, symbol) order and the prefix table.
static_assert(kCanonRuns == 256, "the tables' run scratch holds 256 runs");

__global__ __launch_bounds__(256) void k_dt_count(const uint8_t* __restrict__ cb, uint32_t n,
                                                   DecodeTables* __restrict__ t,
                                                   unsigned* status) {
  const int tid = threadIdx.x, lane = tid & 63;
  if (blockIdx.x == 0) {
    if (tid < 4) status[tid] = 0u;  // the call's status words start here (first kernel)
    if (tid == 0) t->valid = 0;
  }
  const uint16_t* syms = reinterpret_cast<const uint16_t*>(cb);
  const uint8_t* lens = cb + 2 * (size_t)n;
  unsigned i0, i1;
  canon_run(n, i0, i1);
  // (invalid lengths count in lanes that are never read)
  const unsigned cnt = wave_len_counts(lens, i0, i1);
  bool bad = false;
  for (unsigned i = i0 + lane; i < i1; i += 64) {
    const unsigned l = lens[i];
    bad |= l < 1 || l > (unsigned)kMaxCodeLen;
    if (i >= 1) bad |= syms[i] <= syms[i - 1];  // symbols strictly increasing
  }
  const bool any = __ballot(bad) != 0;
  const unsigned gw = blockIdx.x * 4 + (tid >> 6);
  if (lane < 34) t->runs[gw * 36 + lane] = cnt;
  if (lane == 34) t->runs[gw * 36 + 34] = any ? 1u : 0u;
}

__global__ __launch_bounds__(256) void k_dt_rank(const uint8_t* __restrict__ cb, uint32_t n,
                                                  DecodeTables* __restrict__ t,
                                                  unsigned* status) {
  __shared__ unsigned cw[kCanonRuns * 36];
  __shared__ RunScan rs;
  __shared__ unsigned lfirst[34], lbase[34];
  __shared__ unsigned long long llim[34];
  __shared__ unsigned lmax, flag;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  for (int i = tid; i < kCanonRuns * 36; i += 256) cw[i] = t->runs[i];
  if (tid == 0) flag = 0;
  __syncthreads();
  // validity of the runs (one thread per run)
  if (cw[tid * 36 + 34]) flag = 1;
  run_offsets(cw, 36, rs);
  const unsigned* tot = rs.tot;
  if (tid == 0) {
    unsigned c = 0, idx = 0, maxlen = 0;
    unsigned long long kraft = 0;
    for (int l = 1; l <= kMaxCodeLen; ++l) {
      const unsigned cnt = tot[l];
      llim[l] = ((unsigned long long)c + cnt) << (32 - l);
      lfirst[l] = c;
      lbase[l] = idx;
      kraft += (unsigned long long)cnt << (32 - l);
      idx += cnt;
      c = (c + cnt) << 1;
      if (cnt) maxlen = l;
    }
    lmax = maxlen;
    if (kraft > (1ull << 32) || (n >= 2 && kraft != (1ull << 32))) flag = 1;
    if (blockIdx.x == 0 && !flag) {
      for (int l = 1; l <= kMaxCodeLen; ++l) {
        t->first[l] = lfirst[l];
        t->count[l] = tot[l];
        t->base[l] = lbase[l];
        t->limit[l] = llim[l];
      }
      t->maxlen = maxlen;
    }
  }
  __syncthreads();
  if (flag) {
    if (blockIdx.x == 0 && tid == 0) atomicOr(status, ST_FORMAT);
    return;
  }
  // symbols in (length, symbol) order: slot = base of the length + rank
  {
    const uint16_t* syms = reinterpret_cast<const uint16_t*>(cb);
    unsigned i0, i1;
    canon_run(n, i0, i1);
    wave_rank_pass(
        cb + 2 * (size_t)n, i0, i1, lane < 34 ? rs.off[wave][lane] : 0u,
        lane < 34 ? lbase[lane] : 0u, [&](unsigned i) { return (unsigned)syms[i]; },
        [&](unsigned, unsigned sy, unsigned, unsigned rank, unsigned base) {
          t->sorted[base + rank] = (uint16_t)sy;
        });
  }
  // prefix table: the code length at a left-aligned 32-bit window W is one
  // more than the number of lengths whose limit is <= W (limits do not
  // decrease with the length); a prefix's windows span [lo, hi]
  constexpr unsigned kPer = (1u << kLutBits) / kCanonBlocks;
  const unsigned maxlen = lmax;
  for (unsigned p = blockIdx.x * kPer + tid; tid < kPer && p < (blockIdx.x + 1) * kPer; p += 256) {
    const uint64_t lo = (uint64_t)p << (32 - kLutBits);
    const uint64_t hi = lo + (1ull << (32 - kLutBits)) - 1;
    unsigned dlo = 1, dhi = 1;
    for (unsigned l = 1; l <= maxlen; ++l) {
      dlo += llim[l] <= lo ? 1u : 0u;
      dhi += llim[l] <= hi ? 1u : 0u;
    }
    uint32_t e;
    if (dhi > maxlen) e = kLutMixed;  // windows that start no code (one-symbol codebook)
    else if (dlo == dhi) e = (dlo << 16) | ((lbase[dlo] - lfirst[dlo]) & 0xFFFFu);
    else e = kLutMixed | (dlo << 16) | (dhi << 22);
    t->lut[p] = e;
  }
  if (blockIdx.x == 0 && tid == 0) t->valid = 1;
}

// One thread per chunk, 64 chunks per wavefront, blockDim/64 wavefronts per
// block (sized by the launcher so that one pass of blocks covers the CUs).
//
// A symbol costs two LDS lookups and no branch on the common path: the
// 12-bit prefix of the left-aligned window gives the code length d (and a
// 16-bit offset), the top d bits of the window plus the offset give the
// code's index in the (length, symbol)-ordered table.  Prefixes holding
// codes of several lengths (at most one per length boundary) count the
// canonical limits between their shortest and longest length.
//
// Every access to HBM covers whole pieces of a lane's own chunk, since 64
// lanes read and write 64 chunks far apart and L2 keeps few of their lines
// between two accesses of one lane:
//  * coded words arrive in aligned pieces of G words (4G bytes) into a ring
//    of RW words per lane in LDS; ring index i holds the word 4i bytes past
//    the lane's first piece, so the chunk's first word sits at index s0 < G
//    and indices past the chunk's last word read as zero;
//  * at fixed symbol counts (every P symbols, the same points for every
//    lane) a lane whose ring has room for G more words writes the piece it
//    loaded at its previous refill and loads the next one into the same
//    registers (no register copies, which would wait on the loads just
//    issued), so a wavefront waits only for loads issued P symbols before;
//    a refill point leaves at least min(G, RW - G + 1) >= P words in the
//    ring and P symbols take at most P words, so the word a symbol needs is
//    always there;
//  * decoded symbols stay in registers, kDecOB per lane, and leave as whole
//    128-byte rows (16-byte stores) at the next batch's first refill point.
constexpr int kDecOB = 64;
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

__host__ __device__ constexpr size_t dec_sorted_bytes(uint64_t n_codes) {
  return ((size_t)n_codes * sizeof(uint16_t) + 15) & ~size_t(15);
}
// dynamic LDS per wavefront beyond the sorted table: the rings
__host__ __device__ constexpr size_t dec_wave_bytes(int rw) {
  return (size_t)64 * (size_t)(rw + 1) * 4;
}

template <int RW, int G, int P>
__global__ __launch_bounds__(1024) void k_decode(
    const uint8_t* __restrict__ in, uint64_t off_sec, uint64_t words_sec, uint64_t n_chunks,
    uint64_t n_words, int C, int64_t N, uint32_t n_codes, const DecodeTables* __restrict__ t,
    uint16_t* __restrict__ sym, unsigned* status) {
  static_assert((RW & (RW - 1)) == 0 && (G & (G - 1)) == 0 && G >= 4 && 2 * G <= RW,
                "ring of two or more whole pieces");
  static_assert(G >= P && RW - G + 1 >= P && kDecOB % P == 0, "refill points keep P words");
  constexpr int RS = RW + 1;  // ring row pitch in words (odd: rows start on different banks)
  constexpr int NQ = G / 4;   // 16-byte loads per piece
  extern __shared__ __align__(16) unsigned char dsm[];
  __shared__ uint32_t lut[1 << kLutBits];
  __shared__ uint32_t lim[kMaxCodeLen + 1], offd[kMaxCodeLen + 1];
  __shared__ uint32_t valid;
  const int nthr = blockDim.x;
  uint16_t* sorted = reinterpret_cast<uint16_t*>(dsm);
  uint32_t* ring = reinterpret_cast<uint32_t*>(dsm + dec_sorted_bytes(n_codes));
  if (threadIdx.x == 0) valid = t->valid;
  __syncthreads();
  if (!valid) return;  // table build rejected the codebook (status already set)
  for (int i = threadIdx.x; i < (1 << kLutBits); i += nthr) lut[i] = t->lut[i];
  const uint32_t maxlen = t->maxlen > (uint32_t)kMaxCodeLen ? kMaxCodeLen : t->maxlen;
  if (threadIdx.x <= kMaxCodeLen) {
    // limits below the longest length are under 2^32 (the longest length's
    // codes lie above them)
    const int l = threadIdx.x;
    lim[l] = l >= 1 && (uint32_t)l < maxlen ? (uint32_t)t->limit[l] : 0xFFFFFFFFu;
    offd[l] = ((uint32_t)l << 16) | ((t->base[l] - t->first[l]) & 0xFFFFu);
  }
  for (uint32_t i = threadIdx.x; i < n_codes; i += nthr) sorted[i] = t->sorted[i];
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const uint64_t chunk = (uint64_t)blockIdx.x * nthr + wave * 64 + lane;
  const uint64_t* offs = reinterpret_cast<const uint64_t*>(in + off_sec);
  bool live = chunk < n_chunks;
  uint64_t w0 = 0, w1 = 0;
  if (live) {
    w0 = offs[chunk];
    w1 = offs[chunk + 1];
    if (w0 > w1 || w1 > n_words) {
      atomicOr(status, ST_FORMAT);
      live = false;
    }
  }
  const int64_t start = (int64_t)chunk * C;
  const int cnt = live ? (int)min<int64_t>(C, N - start) : 0;
  const uint64_t nwc = live ? w1 - w0 : 0;  // words of the chunk
  // byte offsets from `in` (4-byte aligned): the section [W, E), the first
  // and last 16-byte-aligned pieces that may be read whole, and the lane's
  // first 4G-byte-aligned piece rb
  const int64_t W = (int64_t)words_sec, E = W + 4 * (int64_t)n_words;
  const int64_t a16 = (int64_t)(reinterpret_cast<uintptr_t>(in) & 15);
  const int64_t aG = (int64_t)(reinterpret_cast<uintptr_t>(in) & (4 * G - 1));
  const int64_t lo = ((W + a16) & ~int64_t(15)) - a16;
  const int64_t hi = ((E + a16) & ~int64_t(15)) - a16 - 16;
  const int64_t b0 = W + 4 * (int64_t)w0;
  const int64_t rb = ((b0 + aG) & ~int64_t(4 * G - 1)) - aG;
  const uint32_t s0 = (uint32_t)((b0 - rb) >> 2);
  const uint32_t wend = s0 + (uint32_t)nwc;  // ring indices >= wend read as zero
  // the piece holding ring words i..i+3: pieces before the section read its
  // first piece (their words precede the chunk and are never used); a piece
  // that runs past the section's end is read word by word, clamped
  auto ldp = [&](uint32_t i) -> u32x4 {
    const int64_t b = max(lo, rb + 4 * (int64_t)i);
    if (b <= hi) return *reinterpret_cast<const u32x4*>(in + b);
    const int64_t e4 = E - 4;
    u32x4 r;
    r.x = *reinterpret_cast<const uint32_t*>(in + min(b, e4));
    r.y = *reinterpret_cast<const uint32_t*>(in + min(b + 4, e4));
    r.z = *reinterpret_cast<const uint32_t*>(in + min(b + 8, e4));
    r.w = *reinterpret_cast<const uint32_t*>(in + min(b + 12, e4));
    return r;
  };
  uint32_t* rg = ring + (size_t)threadIdx.x * RS;
  auto put4 = [&](uint32_t i, const u32x4& v) {
    rg[i % RW] = i < wend ? v.x : 0u;
    rg[(i + 1) % RW] = i + 1 < wend ? v.y : 0u;
    rg[(i + 2) % RW] = i + 2 < wend ? v.z : 0u;
    rg[(i + 3) % RW] = i + 3 < wend ? v.w : 0u;
  };
  // prologue: the first RW words into the ring, the next piece in flight
  u32x4 g[NQ];
  {
    u32x4 pre[RW / 4];
#pragma unroll
    for (int q = 0; q < RW / 4; ++q) pre[q] = ldp(4 * q);
#pragma unroll
    for (int q = 0; q < NQ; ++q) g[q] = ldp(RW + 4 * q);
#pragma unroll
    for (int q = 0; q < RW / 4; ++q) put4(4 * q, pre[q]);
  }
  uint64_t buf = ((uint64_t)rg[s0] << 32) | rg[s0 + 1];
  int nb = 64;                     // valid bits in buf (left-aligned)
  uint32_t rd = s0 + 2, wt = RW;   // next word into buf; ring words written
  uint32_t nextw = rg[rd % RW];
  bool bad = false;
  uint32_t ob[kDecOB / 2];  // the batch's symbols, two per register
  const bool vec = (C & 7) == 0 && (reinterpret_cast<uintptr_t>(sym) & 15) == 0;
  auto store_batch = [&](int kb) {
    const int64_t pos = start + kb;
    const int64_t n_here = live ? min<int64_t>(min<int64_t>(kDecOB, C - kb), N - pos) : 0;
    if (vec && n_here == kDecOB) {
      uint4* dst = reinterpret_cast<uint4*>(sym + pos);
#pragma unroll
      for (int q = 0; q < kDecOB / 8; ++q)
        dst[q] = make_uint4(ob[4 * q], ob[4 * q + 1], ob[4 * q + 2], ob[4 * q + 3]);
    } else {
#pragma unroll
      for (int j = 0; j < kDecOB; ++j)
        if (j < n_here) sym[pos + j] = (uint16_t)(ob[j >> 1] >> (16 * (j & 1)));
    }
  };
  auto top_up = [&]() {
    if (wt - rd <= (uint32_t)(RW - G)) {
#pragma unroll
      for (int q = 0; q < NQ; ++q) put4(wt + 4 * q, g[q]);
      wt += G;
#pragma unroll
      for (int q = 0; q < NQ; ++q) g[q] = ldp(wt + 4 * q);
    }
    nextw = rg[rd % RW];
  };
  // a prefix with codes of several lengths: count the limits the window
  // reaches; a window that starts no code marks the chunk bad
  auto mixed = [&](uint32_t e, uint32_t peek) -> uint32_t {
    unsigned d = (e >> 16) & 63u;
    const unsigned dhi = (e >> 22) & 63u;
    if (d == 0) {
      bad = true;
      return (1u << 16) | ((0u - (peek >> 31)) & 0xFFFFu);  // one bit, index 0
    }
    while (d < dhi && peek >= lim[d]) ++d;
    return offd[d];
  };
  for (int k0 = 0; k0 < C; k0 += kDecOB) {
    // the previous batch's stores follow the refill loads, so that the next
    // refill point, which waits for those loads, finds no later store
    top_up();
    if (k0 > 0) store_batch(k0 - kDecOB);
#pragma unroll
    for (int k1 = 0; k1 < kDecOB; k1 += P) {
      if (k1 > 0) top_up();
#pragma unroll
      for (int k2 = 0; k2 < P; ++k2) {
        const int k = k1 + k2;
        const uint32_t peek = (uint32_t)(buf >> 32);
        uint32_t e = lut[peek >> (32 - kLutBits)];
        if (e & kLutMixed) e = mixed(e, peek);
        unsigned d = (e >> 16) & 63u;
        const uint32_t v = (uint32_t)(((uint64_t)peek << d) >> 32);  // top d bits
        const uint32_t sv = sorted[(v + e) & 0xFFFFu];
        ob[k >> 1] = (k & 1) ? (ob[k >> 1] | (sv << 16)) : sv;
        d = k0 + k < cnt ? d : 0u;  // past the chunk's last symbol nothing is consumed
        buf <<= d;
        nb -= (int)d;
        const bool need = nb < 32;
        buf |= (uint64_t)(need ? nextw : 0u) << ((32 - nb) & 63);
        nb += need ? 32 : 0;
        rd += need ? 1u : 0u;
        nextw = rg[rd % RW];
      }
    }
  }
  store_batch(((C - 1) / kDecOB) * kDecOB);
  // bits taken from the chunk: the words moved into the buffer less those
  // still in it
  const int64_t used = ((int64_t)rd - s0) * 32 - nb;
  if (live && (bad || used > (int64_t)nwc * 32)) atomicOr(status, ST_FORMAT);
}

// ------------------------------------------------------------ batched form
// Same bodies as the plain kernels; the array comes from the block map (or
// the block index for one block per array).  Skipped arrays (constant, empty,
// non-finite, no budget) only get their trivial stream or status in kb_header.
__device__ __forceinline__ bool job_skipped_h(const Job& J) { return (*J.status & ST_SKIP) != 0; }
__device__ __forceinline__ uint64_t job_cb_off(const Job& J) {
  return kHeaderBytes + 8ull * (J.L + 1);
}

__global__ __launch_bounds__(1024) void kb_histogram(const Job* __restrict__ jobs,
                                                      const JobBlock* __restrict__ map,
                                                      uint32_t nb) {
  if (blockIdx.x >= nb) return;
  const JobBlock jb = map[blockIdx.x];
  const Job& J = jobs[jb.job];
  if (job_skipped_h(J)) return;
  histogram_body(J.sym, J.N, J.hist, jb.local, jb.count, kHistWinLo, 0u);
}

__global__ __launch_bounds__(1024) void kb_codebook(const Job* __restrict__ jobs) {
  const Job& J = jobs[blockIdx.x];
  if (job_skipped_h(J)) return;
  codebook_body<false, true>(J.hist, J.cbs, J.code, J.clen, J.out + job_cb_off(J), J.lay);
}

__global__ __launch_bounds__(256) void kb_chunk_words(const Job* __restrict__ jobs,
                                                       const JobBlock* __restrict__ map,
                                                       uint32_t nb) {
  if (blockIdx.x >= nb) return;
  const JobBlock jb = map[blockIdx.x];
  const Job& J = jobs[jb.job];
  if (job_skipped_h(J)) return;
  chunk_words_body(J.sym, J.N, (int)kChunkSyms, J.clen, J.cw, J.lay, jb.local, jb.count, J.zc,
                   J.zl);
}

__global__ __launch_bounds__(1024) void kb_layout_scan(const Job* __restrict__ jobs) {
  const Job& J = jobs[blockIdx.x];
  if (job_skipped_h(J)) return;
  layout_scan_body(J.cw, (int64_t)J.n_chunks, J.out, job_cb_off(J), J.lay, J.n_out, J.cap, 0);
}

// Escaped values of one array in stream order, one block per array: the
// exclusive prefix of the chunks' escape counts, then every record placed at
// its rank (the escapes of the chunks before its own, of its chunk's earlier
// lanes, and of its lane's symbols before it), as the plain path does.
__global__ __launch_bounds__(1024) void kb_escape_order(const Job* __restrict__ jobs) {
  const Job& J = jobs[blockIdx.x];
  if (job_skipped_h(J) || J.lay->status) return;
  __shared__ uint32_t wsum[16];
  __shared__ uint32_t carry;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint64_t nc = J.n_chunks;
  if (tid == 0) carry = 0;
  __syncthreads();
  for (uint64_t t0 = 0; t0 < nc; t0 += 1024) {
    const uint64_t i = t0 + tid;
    const uint32_t v = i < nc ? J.zc[i] : 0u;
    uint32_t incl = v;
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = (uint32_t)__shfl_up((int)incl, o, 64);
      if (lane >= o) incl += y;
    }
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    uint32_t before = carry, all = 0;
    for (int w = 0; w < 16; ++w) {
      before += w < wave ? wsum[w] : 0u;
      all += wsum[w];
    }
    if (i < nc) J.zpre[i] = before + incl - v;
    __syncthreads();
    if (tid == 0) carry += all;
    __syncthreads();
  }
  const uint64_t n = J.lay->n_outliers;
  uint64_t* op = reinterpret_cast<uint64_t*>(J.out + J.lay->opos);
  int64_t* ov = reinterpret_cast<int64_t*>(J.out + J.lay->oval);
  for (uint64_t i = tid; i < n; i += 1024) {
    const uint32_t pos = J.opos[i];
    const uint32_t chunk = pos >> 10, j = pos & 1023u;
    const uint32_t e = J.zl[(size_t)chunk * 64 + (j >> 4)];
    const uint32_t t = j & 15u;
    const uint64_t rank = (uint64_t)J.zpre[chunk] + (e >> 16) + (uint32_t)__popc(e & ((1u << t) - 1u));
    if (((e >> t) & 1u) == 0u || rank >= n) {
      atomicOr(J.status, ST_INTERNAL);
      continue;
    }
    op[rank] = pos;
    ov[rank] = J.oval[i];
  }
}

__global__ __launch_bounds__(1024) void kb_outlier_sort(const Job* __restrict__ jobs) {
  const Job& J = jobs[blockIdx.x];
  if (job_skipped_h(J)) return;
  const OutlierBuf ob{J.opos, J.oval, J.n_out, J.cap};
  outlier_sort_body(ob, J.okA, J.ovA, J.okB, J.ovB, J.key_bits, J.out, J.lay);
}

__global__ __launch_bounds__(256) void kb_encode(const Job* __restrict__ jobs,
                                                  const JobBlock* __restrict__ map,
                                                  uint32_t nb) {
  extern __shared__ uint32_t wbuf[];  // 4 * C words
  if (blockIdx.x >= nb) return;
  const JobBlock jb = map[blockIdx.x];
  const Job& J = jobs[jb.job];
  if (job_skipped_h(J)) return;
  encode_body(J.sym, J.N, (int)kChunkSyms, J.code, J.clen, J.cbs.pk, J.out, J.lay, jb.local,
              wbuf);
}

// Header, bins and result-table entries of one array (thread 0).
__global__ void kb_header(const Job* __restrict__ jobs) {
  if (threadIdx.x != 0) return;
  const Job& J = jobs[blockIdx.x];
  header_body(J.hdr, J.out, J.bud, J.L, *J.status, J.lay, J.size_out, J.status_out);
}

}  // namespace

uint32_t hist_blocks(int64_t n) {
  int64_t blocks = (n + 1024 * 64 - 1) / (1024 * 64);
  if (blocks < 1) blocks = 1;
  if (blocks > 256) blocks = 256;
  return (uint32_t)blocks;
}

void launch_histogram(const uint16_t* sym, int64_t n, unsigned* hist, hipStream_t s,
                      const unsigned* gate, uint32_t win_lo, uint32_t hot) {
  if (win_lo > (uint32_t)(kDict - kHistWin)) throw std::logic_error("histogram window out of range");
  hipLaunchKernelGGL(k_histogram, dim3(hist_blocks(n)), dim3(1024), 0, s, sym, n, hist, gate,
                     win_lo, hot);
}

void launch_b_histogram(const Job* jobs, const JobBlock* map, uint32_t nb, hipStream_t s) {
  hipLaunchKernelGGL(kb_histogram, dim3(nb), dim3(1024), 0, s, jobs, map, nb);
}
void launch_b_codebook(const Job* jobs, int n, hipStream_t s) {
  hipLaunchKernelGGL(kb_codebook, dim3((unsigned)n), dim3(1024), 0, s, jobs);
}
void launch_b_chunk_words(const Job* jobs, const JobBlock* map, uint32_t nb, hipStream_t s) {
  hipLaunchKernelGGL(kb_chunk_words, dim3(nb), dim3(256), 0, s, jobs, map, nb);
}
void launch_b_layout_scan(const Job* jobs, int n, hipStream_t s) {
  hipLaunchKernelGGL(kb_layout_scan, dim3((unsigned)n), dim3(1024), 0, s, jobs);
}
void launch_b_escape_order(const Job* jobs, int n, hipStream_t s) {
  hipLaunchKernelGGL(kb_escape_order, dim3((unsigned)n), dim3(1024), 0, s, jobs);
}
void launch_b_outlier_sort(const Job* jobs, int n, hipStream_t s) {
  hipLaunchKernelGGL(kb_outlier_sort, dim3((unsigned)n), dim3(1024), 0, s, jobs);
}
void launch_b_encode(const Job* jobs, const JobBlock* map, uint32_t nb, hipStream_t s) {
  hipLaunchKernelGGL(kb_encode, dim3(nb), dim3(256), (size_t)4 * kChunkSyms * sizeof(uint32_t),
                     s, jobs, map, nb);
}
void launch_b_header(const Job* jobs, int n, hipStream_t s) {
  hipLaunchKernelGGL(kb_header, dim3((unsigned)n), dim3(64), 0, s, jobs);
}

void launch_codebook(const unsigned* hist, const CodebookScratch& sc, uint32_t* code,
                     uint8_t* clen, uint8_t* cb_out_base, uint64_t cb_off, Layout* lay,
                     hipStream_t s, const unsigned* gate, bool canon) {
  hipLaunchKernelGGL(k_cbs_count, dim3(kSortTiles), dim3(256), 0, s, hist, sc, gate);
  hipLaunchKernelGGL(k_cbs_pass<0>, dim3(kSortTiles), dim3(256), 0, s, hist, sc, gate);
  hipLaunchKernelGGL(k_cbs_pass<1>, dim3(kSortTiles), dim3(256), 0, s, hist, sc, gate);
  hipLaunchKernelGGL(k_cbs_pass<2>, dim3(kSortTiles), dim3(256), 0, s, hist, sc, gate);
  hipLaunchKernelGGL(k_cbs_pass<3>, dim3(kSortTiles), dim3(256), 0, s, hist, sc, gate);
  hipLaunchKernelGGL(k_codebook, dim3(1), dim3(1024), 0, s, hist, sc, code, clen,
                     cb_out_base + cb_off, lay, gate);
  if (canon) launch_canon(sc, code, cb_out_base, cb_off, lay, s, gate);
}

void launch_canon(const CodebookScratch& sc, uint32_t* code, uint8_t* cb_out_base,
                  uint64_t cb_off, Layout* lay, hipStream_t s, const unsigned* gate) {
  hipLaunchKernelGGL(k_canon_count, dim3(kCanonBlocks), dim3(256), 0, s, sc, lay, gate);
  hipLaunchKernelGGL(k_canon_rank, dim3(kCanonBlocks), dim3(256), 0, s, sc, code,
                     cb_out_base + cb_off, lay, gate);
}

// Each block first copies the 64 KiB length table, so it takes at least 16
// groups of four chunks (128 KiB of symbols at C = 1024).
uint32_t chunk_words_blocks(int64_t N, int C) {
  const int64_t groups = ((N + C - 1) / C + 3) / 4;
  return (uint32_t)std::max<int64_t>(1, std::min<int64_t>((groups + 15) / 16, 512));
}

void launch_chunk_words(const uint16_t* sym, int64_t N, int C, const uint8_t* clen,
                        uint32_t* cw, Layout* lay, hipStream_t s, const unsigned* gate,
                        uint32_t* zc, uint32_t* zl) {
  if (zc && C != 1024) throw std::logic_error("launch_chunk_words: escape counts need C = 1024");
  hipLaunchKernelGGL(k_chunk_words, dim3(chunk_words_blocks(N, C)), dim3(256), 0, s, sym, N, C,
                     clen, cw, lay, gate, zc, zl);
}

int64_t esc_sum_blocks(int64_t n_chunks) {
  return std::max<int64_t>(1, std::min<int64_t>(kEscSumsMax, (n_chunks + 1023) / 1024));
}

void launch_chunk_prefix(const uint32_t* zc, uint32_t* zpre, uint32_t* sums, int64_t n_chunks,
                         const Layout* lay, hipStream_t s) {
  const int64_t nb = esc_sum_blocks(n_chunks);
  const int64_t R = (n_chunks + nb - 1) / nb;
  const int64_t blocks = (n_chunks + R - 1) / R;
  hipLaunchKernelGGL(k_esc_sums, dim3((unsigned)blocks), dim3(kEscThreads), 0, s, zc, n_chunks,
                     R, sums, lay, nullptr);
  hipLaunchKernelGGL(k_esc_prefix, dim3((unsigned)blocks), dim3(kEscThreads), 0, s, zc,
                     n_chunks, R, sums, zpre, lay, nullptr);
}

void launch_escape_order(const OutlierBuf& ob, const uint32_t* zc, const uint32_t* zl,
                         uint32_t* zpre, uint32_t* sums, int64_t n_chunks, uint8_t* out,
                         Layout* lay, unsigned* status, hipStream_t s, const unsigned* gate) {
  const int64_t nb = esc_sum_blocks(n_chunks);
  const int64_t R = (n_chunks + nb - 1) / nb;
  const int64_t blocks = (n_chunks + R - 1) / R;
  hipLaunchKernelGGL(k_esc_sums, dim3((unsigned)blocks), dim3(kEscThreads), 0, s, zc, n_chunks,
                     R, sums, lay, gate);
  hipLaunchKernelGGL(k_esc_prefix, dim3((unsigned)blocks), dim3(kEscThreads), 0, s, zc,
                     n_chunks, R, sums, zpre, lay, gate);
  const unsigned grid = (unsigned)std::max<uint64_t>(1, std::min<uint64_t>((ob.cap + 255) / 256, 2048));
  hipLaunchKernelGGL(k_esc_place, dim3(grid), dim3(256), 0, s, ob, zpre, zl, out, lay, status,
                     gate);
}

void launch_layout_scan(const uint32_t* cw, int64_t n_chunks, uint8_t* out, uint64_t cb_off,
                        Layout* lay, const unsigned long long* n_out, uint64_t out_cap_n,
                        bool huff_only, hipStream_t s, const unsigned* gate) {
  // ranges of at least 4096 chunks; the range totals follow the counts
  const int64_t nb = std::min<int64_t>(kScanBlocksMax, (n_chunks + 4095) / 4096);
  if (nb <= 1) {
    hipLaunchKernelGGL(k_layout_scan, dim3(1), dim3(1024), 0, s, cw, n_chunks, out, cb_off, lay,
                       n_out, out_cap_n, huff_only ? 1 : 0, gate);
    return;
  }
  const int64_t R = ((n_chunks + nb - 1) / nb + 3) & ~int64_t(3);
  const int64_t blocks = (n_chunks + R - 1) / R;
  unsigned long long* sums =
      reinterpret_cast<unsigned long long*>(const_cast<uint32_t*>(cw) + scan_sums_at(n_chunks));
  hipLaunchKernelGGL(k_scan_sums, dim3((unsigned)blocks), dim3(kScanThreads), 0, s, cw, n_chunks,
                     R, sums, gate);
  hipLaunchKernelGGL(k_scan_offsets, dim3((unsigned)blocks), dim3(kScanThreads), 0, s, cw,
                     n_chunks, R, sums, out, cb_off, lay, n_out, out_cap_n, huff_only ? 1 : 0,
                     gate);
}

void launch_outlier_sort(const OutlierBuf& ob, uint32_t* keyA, uint32_t* valA, uint32_t* keyB,
                         uint32_t* valB, int key_bits, uint8_t* out, Layout* lay,
                         hipStream_t s, const unsigned* gate) {
  hipLaunchKernelGGL(k_outlier_sort, dim3(1), dim3(1024), 0, s, ob, keyA, valA, keyB, valB,
                     key_bits, out, lay, gate);
}

void launch_encode(const uint16_t* sym, int64_t N, int C, const uint32_t* code,
                   const uint8_t* clen, const uint32_t* pk, uint8_t* out, const Layout* lay,
                   hipStream_t s, const unsigned* gate) {
  const int64_t n_chunks = (N + C - 1) / C;
  // large arrays: the persistent encoder with the code window in LDS (one
  // block per CU); the window copy needs 16-byte aligned symbol and table
  // arrays
  constexpr int64_t kCUs = 256;
  if (C == kEncC && n_chunks >= 2 * kCUs * kEncWaves &&
      (reinterpret_cast<uintptr_t>(sym) & 15) == 0 && (reinterpret_cast<uintptr_t>(pk) & 15) == 0) {
    static bool attr = false;
    if (!attr) {
      MGC_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(k_encode_win),
                                  hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)enc_win_lds_bytes()));
      attr = true;
    }
    const int64_t blocks = std::min<int64_t>(kCUs, (n_chunks + kEncWaves - 1) / kEncWaves);
    hipLaunchKernelGGL(k_encode_win, dim3((unsigned)blocks), dim3(64 * kEncWaves),
                       enc_win_lds_bytes(), s, sym, N, pk, out, lay, gate);
    return;
  }
  hipLaunchKernelGGL(k_encode, dim3((unsigned)((n_chunks + 3) / 4)), dim3(256),
                     (size_t)4 * C * sizeof(uint32_t), s, sym, N, C, code, clen, pk, out, lay,
                     gate);
}

void launch_header(uint8_t* out, const Header& h, const double* bud, const Layout* lay,
                   const unsigned* status, bool empty, unsigned long long* res, hipStream_t s) {
  hipLaunchKernelGGL(k_header, dim3(1), dim3(64), 0, s, out, h, bud, lay, status, empty ? 1 : 0,
                     res);
}

void launch_huff_header(uint8_t* out, uint32_t C, uint64_t N, uint64_t n_chunks,
                        const Layout* lay, unsigned long long* info, hipStream_t s) {
  hipLaunchKernelGGL(k_huff_header, dim3(1), dim3(64), 0, s, out, C, N, n_chunks, lay, info);
}

void launch_decode_tables(const uint8_t* cb, uint64_t n_codes, DecodeTables* t,
                          unsigned* status, hipStream_t s) {
  hipLaunchKernelGGL(k_dt_count, dim3(kCanonBlocks), dim3(256), 0, s, cb, (uint32_t)n_codes, t,
                     status);
  hipLaunchKernelGGL(k_dt_rank, dim3(kCanonBlocks), dim3(256), 0, s, cb, (uint32_t)n_codes, t,
                     status);
}

namespace {
// decoder shapes (ring words, piece words, refill period), widest first
template <int RW, int G, int P>
size_t decode_room() {
  // the dynamic LDS the kernel can take on top of its static LDS (160 KiB per CU)
  static size_t room = 0;
  if (room == 0) {
    hipFuncAttributes fa;
    MGC_HIP(hipFuncGetAttributes(&fa, reinterpret_cast<const void*>(k_decode<RW, G, P>)));
    const size_t r = 163840 - fa.sharedSizeBytes;
    MGC_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(k_decode<RW, G, P>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)r));
    room = r;
  }
  return room;
}
}  // namespace

DecodeShape launch_decode(const uint8_t* in, uint64_t off_sec, uint64_t words_sec,
                          uint64_t n_chunks, uint64_t n_words, int C, int64_t N,
                          uint64_t n_codes, const DecodeTables* t, uint16_t* sym,
                          unsigned* status, hipStream_t s, DecodeShape force) {
  // the kernel reads whole 16-byte pieces of the word section
  if ((reinterpret_cast<uintptr_t>(in) & 3) != 0 || (words_sec & 3) != 0)
    fail(MGC_EINVAL, "compressed stream must start on a 4-byte boundary");
  // wavefronts per block: enough that one block per CU covers every chunk
  // (one pass over the 256 CUs), at most 16; then the widest ring that fits
  // in LDS beside the symbol table (64-, 32- or 16-byte pieces), else fewer
  // wavefronts with the narrowest ring.  A forced ring or wavefront count
  // replaces the automatic choice and must fit.
  constexpr uint64_t kCUs = 256;
  int waves = (int)std::min<uint64_t>(16, std::max<uint64_t>(1, (n_chunks + 64 * kCUs - 1) / (64 * kCUs)));
  if (force.waves > 0) waves = force.waves;
  const size_t tab = dec_sorted_bytes(n_codes);
  constexpr int kRW[3] = {32, 16, 8};
  const size_t room[3] = {decode_room<32, 16, 16>(), decode_room<16, 8, 8>(),
                          decode_room<8, 4, 4>()};
  int shape = force.ring > 0 ? force.ring - 1 : 0;
  while (tab + (size_t)waves * dec_wave_bytes(kRW[shape]) > room[shape]) {
    if (force.ring > 0)
      fail(MGC_EINVAL, "the forced decoder ring and wavefront count do not fit in LDS");
    if (shape < 2) ++shape;
    else if (force.waves > 0)
      fail(MGC_EINVAL, "the forced decoder wavefront count does not fit in LDS");
    else if (waves > 1) --waves;
    else fail(MGC_EDEVICE, "decode table does not fit in LDS");
  }
  const int nthr = 64 * waves;
  const dim3 grid((unsigned)((n_chunks + nthr - 1) / nthr));
  const size_t dyn = tab + (size_t)waves * dec_wave_bytes(kRW[shape]);
  if (shape == 0)
    hipLaunchKernelGGL((k_decode<32, 16, 16>), grid, dim3(nthr), dyn, s, in, off_sec, words_sec,
                       n_chunks, n_words, C, N, (uint32_t)n_codes, t, sym, status);
  else if (shape == 1)
    hipLaunchKernelGGL((k_decode<16, 8, 8>), grid, dim3(nthr), dyn, s, in, off_sec, words_sec,
                       n_chunks, n_words, C, N, (uint32_t)n_codes, t, sym, status);
  else
    hipLaunchKernelGGL((k_decode<8, 4, 4>), grid, dim3(nthr), dyn, s, in, off_sec, words_sec,
                       n_chunks, n_words, C, N, (uint32_t)n_codes, t, sym, status);
  return DecodeShape{shape + 1, waves};
}

}  // namespace mgc
