// Internal definitions shared by the host orchestration and the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "mgc.h"

namespace mgc {

constexpr uint32_t kDict = 65536;   // dictionary size S (16-bit symbols)
constexpr uint32_t kHalf = 32768;   // symbol = k + S/2 for |k| < S/2; 0 = escape
constexpr int kMaxCodeLen = 32;
constexpr int kPkFirstWords = 64;   // first-code table behind the packed code words
constexpr int kHeaderBytes = 128;
constexpr int kHuffHeaderBytes = 48;
constexpr uint32_t kMagic = 0x3143474Du;      // "MGC1"
constexpr uint32_t kHuffMagic = 0x3148474Du;  // "MGH1"
constexpr int kHxHeaderBytes = 64;
constexpr int kZfpHeaderBytes = 64;
constexpr uint32_t kZfpMagic = 0x465A474Du;   // "MGZF"
constexpr uint32_t kHxMagic = 0x5848474Du;    // "MGHX"
constexpr uint16_t kVersion = 1;
constexpr int kMaxLevels = 62;

// Device-side status bits (OR-ed by kernels, read once at the end of a call).
enum : uint32_t {
  ST_RANGE = 1u,      // a quantised value reached 2^62
  ST_OVERFLOW = 2u,   // more escaped values than the outlier capacity
  ST_FORMAT = 4u,     // corrupt code or table in a stream being decoded
  ST_INTERNAL = 8u,   // a bounded device loop hit its iteration guard
  ST_NONFINITE = 16u, // the input holds NaN or Inf
  ST_CONST = 32u,     // the input is constant (trivial stream)
  ST_BUDGET = 64u,    // the error budget vanishes below the output precision
  ST_EMPTY = 128u,    // the array has no values (trivial stream)
  ST_SKIP = ST_NONFINITE | ST_CONST | ST_BUDGET | ST_EMPTY,
};

// A compression's later kernels take its status word as a gate: once the
// range pass has flagged the input (constant, empty, non-finite, or a budget
// below the output precision) they return at once.  A null gate is open.
__device__ __forceinline__ bool gate_closed(const unsigned* gate) {
  return gate != nullptr && (*gate & ST_SKIP) != 0u;
}

// Error-budget block of a compression (device, doubles): [0..3] min, max, sum
// of squares, non-finite flag; [4] tau; [5] tau'; [6 .. 6+L] bins q_l;
// [7+L .. 7+2L] their reciprocals.
constexpr int kBudDoubles = 6 + 2 * (kMaxLevels + 1);
__host__ __device__ inline int bud_q(int l) { return 6 + l; }
__host__ __device__ inline int bud_r(int L, int l) { return 7 + L + l; }

// Inputs of the error budget: the request and the per-level bin factors K_l
// (q_l = tau' K_l; device table of L + 1 doubles).
struct BudgetIn {
  int dtype, norm, mode, L;
  double bound;
  int64_t N;
  const double* K;
};

// Per-axis tables of one level (device pointers into the plan's table block).
struct AxisTab {
  const double* wl;  // [nf] weight of the left coarse neighbour of new node i
  const double* wr;  // [nf] weight of the right coarse neighbour of new node i
  const double* W;   // [nc*5] restriction taps at fine p(j)-2 .. p(j)+2
  const double* ta;  // [nc] Thomas: sub-diagonal times reciprocal pivot (0 at j = 0)
  const double* tm;  // [nc] Thomas: reciprocal pivots
  const double* tc;  // [nc] Thomas: super-diagonal times reciprocal pivot (0 at the end)
  const double* WP;  // [nc*5] taps of P^T at fine p(j)-2 .. p(j)+2 (adjoint)
  const double* Mt;  // [nf*3] fine mass-matrix row (i-1, i, i+1) (adjoint)
};

// Geometry of level l (fine grid = level l, coarse grid = level l-1) in the
// internal 3-axis layout (squeezed axes first, length 1).  Passed by value.
struct LevelGeom {
  int64_t nf[3];
  int64_t nc[3];
  int bit[3];            // subband bit of internal axis k (-1: inactive axis)
  int64_t level_off;     // stream offset of the level's first coefficient
  int64_t sub_off[8];    // offset of subband m inside the level
  AxisTab ax[3];
};

// Escaped values appended by the quantiser: (stream position, k).
struct OutlierBuf {
  uint32_t* pos;
  int64_t* val;
  unsigned long long* count;
  uint64_t cap;
};

// Coefficient source for recomposition: quantised symbols or FP64 values.
struct CoeffSrc {
  const uint16_t* sym;   // symbols (nullptr when raw is used)
  const double* raw;     // FP64 coefficients in stream order
  const uint64_t* opos;  // sorted escape positions
  const int64_t* oval;   // their values
  int64_t n_out;
};

// Scratch of the single-block codebook construction (65536 entries each).
struct CodebookScratch {
  uint32_t *keyA, *valA, *keyB, *valB, *symAsc, *freqAsc, *Iw, *Sw, *leafPar, *parA, *parB,
      *dstA, *dstB;
  uint32_t* pk;  // per coded symbol: rank << 6 | length, the rank among the codes of
                 // that length (code = first code of the length + rank); then, at
                 // pk[kDict + l], the first code of each length l (kPkFirstWords)
  uint32_t* hcnt;   // multi-block leaf sort: [pass][digit][tile] item counts
  uint32_t* fmaxT;  // multi-block leaf sort: largest frequency per tile
};

// Stream layout computed on the device once counts are known.
struct Layout {
  unsigned long long n_codes;
  unsigned long long n_outliers;
  unsigned long long n_words;
  unsigned long long cb, off, opos, oval, words, end;
  unsigned int status;
  unsigned int max_len;   // longest code length (set with the codebook)
};

// Fixed 128-byte header of a compressed stream (little-endian on the host
// and the device alike).
#pragma pack(push, 1)
struct Header {
  uint32_t magic;
  uint16_t version;
  uint8_t dtype, norm, mode, ndim, flags, D;
  uint32_t L;
  uint64_t shape[3];
  double bound, tau, tau_eff, const_value;
  uint32_t S, C;
  uint64_t N, n_codes, n_outliers, n_chunks, n_words, total;
};
struct HuffHeader {
  uint32_t magic, C;
  uint64_t N, n_codes, n_chunks, n_words, total;
};
#pragma pack(pop)
static_assert(sizeof(Header) == kHeaderBytes, "header layout");
static_assert(sizeof(HuffHeader) == kHuffHeaderBytes, "huffman header layout");

// 64-byte header of a fixed-rate block-coded stream.
#pragma pack(push, 1)
struct ZfpHead {
  uint32_t magic;
  uint8_t dtype, ndim;
  uint16_t z0;
  uint32_t maxbits, z1;
  uint64_t shape[3];
  double rate;
  uint64_t blocks, total;
};
#pragma pack(pop)
static_assert(sizeof(ZfpHead) == kZfpHeaderBytes, "fixed-rate header layout");

enum : uint8_t { FLAG_CONSTANT = 1, FLAG_EMPTY = 2 };

// ------------------------------------------------------------ batched form
// One array of a batched compression: a device table entry written by the
// host (pointers into the caller's buffers and the plan's tables).  Work
// buffers are those of a plain compression of the same array.
struct Job {
  const void* in;
  uint8_t* out;             // this array's output slot
  int64_t N;
  int32_t L, dtype;
  uint64_t cap;             // outlier capacity
  uint64_t n_chunks;
  int32_t key_bits, pad0;
  const LevelGeom* geo;     // geo[l], l = 0..L
  BudgetIn bi;
  double *part, *bud;
  uint16_t* sym;
  double *gA, *gB;
  unsigned* status;
  unsigned long long* n_out;
  Layout* lay;
  unsigned* hist;
  uint32_t* code;
  uint8_t* clen;
  CodebookScratch cbs;
  uint32_t* cw;
  uint32_t* opos;
  int64_t* oval;
  uint32_t *okA, *ovA, *okB, *ovB;
  uint32_t *zc, *zpre, *zl;  // escape counts per chunk, their prefix, lane masks
  uint64_t* size_out;       // result tables of the call (device)
  int32_t* status_out;
  Header hdr;               // template: request and shape fields
};

// Block of a flattened batched launch: its array, its index among that
// array's blocks of the launch and their count.
struct JobBlock {
  uint32_t job, local, count;
};

__host__ __device__ inline uint64_t pad8(uint64_t n) { return (n + 7) & ~uint64_t(7); }

// ----------------------------------------------------------------- errors
void set_error(const std::string& msg);
struct Fail {
  mgc_status st;
};
#define MGC_HIP(call)                                                             \
  do {                                                                            \
    hipError_t e_ = (call);                                                       \
    if (e_ != hipSuccess) {                                                       \
      ::mgc::set_error(std::string(#call) + ": " + hipGetErrorString(e_));        \
      throw ::mgc::Fail{MGC_EDEVICE};                                             \
    }                                                                             \
  } while (0)

[[noreturn]] void fail(mgc_status st, const std::string& msg);

// ---------------------------------------------------------- stage timing
// Records events around a launch when profiling is enabled on the context.
struct Profiler;
struct StageScope {
  Profiler* p;
  int slot;
  hipStream_t s;
  hipEvent_t a;
  StageScope(Profiler* prof, const char* name, hipStream_t stream);
  ~StageScope();
};

}  // namespace mgc
