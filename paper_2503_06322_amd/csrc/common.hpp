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
constexpr int kHeaderBytes = 128;
constexpr int kHuffHeaderBytes = 48;
constexpr uint32_t kMagic = 0x3143474Du;      // "MGC1"
constexpr uint32_t kHuffMagic = 0x3148474Du;  // "MGH1"
constexpr uint16_t kVersion = 1;
constexpr int kMaxLevels = 62;

// Device-side status bits (OR-ed by kernels, read once at the end of a call).
enum : uint32_t {
  ST_RANGE = 1u,      // a quantised value reached 2^62
  ST_OVERFLOW = 2u,   // more escaped values than the outlier capacity
  ST_FORMAT = 4u,     // corrupt code or table in a stream being decoded
  ST_INTERNAL = 8u,   // a bounded device loop hit its iteration guard
};

// Per-axis tables of one level (device pointers into the plan's table block).
struct AxisTab {
  const double* wl;  // [nf] weight of the left coarse neighbour of new node i
  const double* wr;  // [nf] weight of the right coarse neighbour of new node i
  const double* W;   // [nc*5] restriction taps at fine p(j)-2 .. p(j)+2
  const double* ta;  // [nc] Thomas: sub-diagonal of the coarse mass matrix
  const double* tm;  // [nc] Thomas: reciprocal pivots
  const double* tc;  // [nc] Thomas: super-diagonal times reciprocal pivot
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

// Stream layout computed on the device once counts are known.
struct Layout {
  unsigned long long n_codes;
  unsigned long long n_outliers;
  unsigned long long n_words;
  unsigned long long cb, off, opos, oval, words, end;
  unsigned int status;
  unsigned int pad;
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

enum : uint8_t { FLAG_CONSTANT = 1, FLAG_EMPTY = 2 };

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
