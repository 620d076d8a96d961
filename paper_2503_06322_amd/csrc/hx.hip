// Huffman-X: the Huffman pipeline (Algorithm 2, Section IV-B) as a
// standalone lossless codec for byte and integer streams.
//
// Values become 16-bit keys: u8 and u16 values are their own keys; an i32 or
// i64 value v with lo <= v <= hi (lo = base, hi = base + D - 2) is key
// v - lo and every other value is the escape key D - 1, its value stored raw
// after the coded section in position order.  The keys then go through the
// Huffman stage of the compressor unchanged (histogram, codebook, chunk
// sizes, layout scan, encode; decode tables, decode).
//
// The kernels here work on chunks of 1024 values, one wavefront per chunk,
// value i of chunk c at c * 1024 + k * 64 + lane (k = 0..15), so every load
// and store instruction covers 64 consecutive values and position order is
// (k, lane) order: a value's rank among its chunk's escapes is the escapes of
// the earlier k plus those of the lower lanes at its k (one ballot each).
#include "kernels.hpp"

namespace mgc {
namespace {

constexpr int kHxWaves = 4;  // wavefronts per block
constexpr uint64_t kHxChunk = 1024;

__device__ __forceinline__ uint64_t hx_lanemask_lt() {
  const int lane = threadIdx.x & 63;
  return lane ? (~0ull >> (64 - lane)) : 0ull;
}

template <typename T>
__device__ __forceinline__ bool hx_inside(T v, int64_t lo, int64_t hi) {
  return (int64_t)v >= lo && (int64_t)v <= hi;
}

// Keys of the values; zc[chunk] = escapes in the chunk (ESC types only).
template <typename T, bool ESC>
__global__ __launch_bounds__(64 * kHxWaves) void k_hx_keys(const T* __restrict__ in, uint64_t n,
                                                           int64_t lo, int64_t hi, uint32_t esc,
                                                           uint16_t* __restrict__ key,
                                                           uint32_t* __restrict__ zc,
                                                           uint64_t n_chunks) {
  const int lane = threadIdx.x & 63;
  const uint64_t wave = (uint64_t)blockIdx.x * kHxWaves + (threadIdx.x >> 6);
  const uint64_t step = (uint64_t)gridDim.x * kHxWaves;
  for (uint64_t c = wave; c < n_chunks; c += step) {
    uint32_t cnt = 0;
#pragma unroll 4
    for (int k = 0; k < 16; ++k) {
      const uint64_t i = c * kHxChunk + (uint64_t)k * 64 + lane;
      bool e = false;
      if (i < n) {
        const T v = in[i];
        if (ESC) {
          e = !hx_inside(v, lo, hi);
          key[i] = e ? (uint16_t)esc : (uint16_t)((uint64_t)(int64_t)v - (uint64_t)lo);
        } else {
          key[i] = (uint16_t)v;
        }
      }
      if (ESC) cnt += (uint32_t)__popcll(__ballot(e));
    }
    if (ESC && lane == 0) zc[c] = cnt;
  }
}

// Byte keys, sixteen bytes a thread (one 16-byte load, two 16-byte stores);
// the tail of n mod 16 bytes one by one.  Needs a 16-byte aligned input.
__global__ __launch_bounds__(256) void k_hx_keys_u8(const uint8_t* __restrict__ in, uint64_t n,
                                                    uint16_t* __restrict__ key) {
  const uint64_t n16 = n / 16;
  const uint64_t stride = (uint64_t)gridDim.x * 256;
  const uint4* src = reinterpret_cast<const uint4*>(in);
  uint4* dst = reinterpret_cast<uint4*>(key);
  for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n16; i += stride) {
    const uint4 w = src[i];
    const uint32_t a[4] = {w.x, w.y, w.z, w.w};
    uint32_t o[8];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      o[2 * k] = (a[k] & 0xFFu) | ((a[k] & 0xFF00u) << 8);
      o[2 * k + 1] = ((a[k] >> 16) & 0xFFu) | ((a[k] >> 8) & 0xFF0000u);
    }
    dst[2 * i] = make_uint4(o[0], o[1], o[2], o[3]);
    dst[2 * i + 1] = make_uint4(o[4], o[5], o[6], o[7]);
  }
  for (uint64_t i = n16 * 16 + (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride)
    key[i] = in[i];
}

// Escaped values of each chunk at zpre[chunk] + rank in the escape section,
// which starts right after the coded section (sec + lay->end).
template <typename T>
__global__ __launch_bounds__(64 * kHxWaves) void k_hx_place(const T* __restrict__ in, uint64_t n,
                                                            int64_t lo, int64_t hi,
                                                            const uint32_t* __restrict__ zc,
                                                            const uint32_t* __restrict__ zpre,
                                                            uint64_t n_chunks, uint8_t* sec,
                                                            const Layout* __restrict__ lay) {
  if (lay->status) return;
  T* esc = reinterpret_cast<T*>(sec + lay->end);
  const int lane = threadIdx.x & 63;
  const uint64_t wave = (uint64_t)blockIdx.x * kHxWaves + (threadIdx.x >> 6);
  const uint64_t step = (uint64_t)gridDim.x * kHxWaves;
  for (uint64_t c = wave; c < n_chunks; c += step) {
    if (zc[c] == 0) continue;
    uint64_t run = zpre[c];
    for (int k = 0; k < 16; ++k) {
      const uint64_t i = c * kHxChunk + (uint64_t)k * 64 + lane;
      T v = 0;
      bool e = false;
      if (i < n) {
        v = in[i];
        e = !hx_inside(v, lo, hi);
      }
      const uint64_t m = __ballot(e);
      if (e) esc[run + __popcll(m & hx_lanemask_lt())] = v;
      run += __popcll(m);
    }
  }
}

// The 64-byte stream header, the zero padding after the escaped values, and
// res = {status, stream bytes}.
struct HxHead {
  uint32_t magic;
  uint8_t type, z0, z1, z2;
  uint32_t D, C;
  int64_t base;
  uint64_t n, n_escaped, section, total, z3;
};
static_assert(sizeof(HxHead) == kHxHeaderBytes, "Huffman-X header is 64 bytes");

__global__ void k_hx_header(uint8_t* __restrict__ out, uint32_t type, uint32_t D, uint32_t C,
                            int64_t base, uint64_t n, const uint32_t* __restrict__ zc,
                            const uint32_t* __restrict__ zpre, uint64_t n_chunks,
                            const Layout* __restrict__ lay, uint32_t width,
                            unsigned long long* __restrict__ res) {
  if (threadIdx.x != 0) return;
  const bool coded = n > 0;
  const unsigned st = coded ? lay->status : 0u;
  const uint64_t n_esc = (zc && n_chunks) ? (uint64_t)zpre[n_chunks - 1] + zc[n_chunks - 1] : 0;
  const uint64_t sec = coded ? lay->end : 0;
  const uint64_t total = kHxHeaderBytes + sec + pad8(n_esc * width);
  res[0] = st ? (unsigned long long)MGC_EDEVICE : 0ull;
  res[1] = st ? 0ull : total;
  if (st) return;
  HxHead h;
  h.magic = kHxMagic;
  h.type = (uint8_t)type;
  h.z0 = h.z1 = h.z2 = 0;
  h.D = D;
  h.C = C;
  h.base = base;
  h.n = n;
  h.n_escaped = n_esc;
  h.section = sec;
  h.total = total;
  h.z3 = 0;
  const uint8_t* src = reinterpret_cast<const uint8_t*>(&h);
  for (int i = 0; i < kHxHeaderBytes; ++i) out[i] = src[i];
  for (uint64_t i = kHxHeaderBytes + sec + n_esc * width; i < total; ++i) out[i] = 0;
}

// Escape keys per chunk of decoded keys.
__global__ __launch_bounds__(64 * kHxWaves) void k_hx_count(const uint16_t* __restrict__ key,
                                                            uint64_t n, uint32_t esc,
                                                            uint32_t* __restrict__ zc,
                                                            uint64_t n_chunks) {
  const int lane = threadIdx.x & 63;
  const uint64_t wave = (uint64_t)blockIdx.x * kHxWaves + (threadIdx.x >> 6);
  const uint64_t step = (uint64_t)gridDim.x * kHxWaves;
  for (uint64_t c = wave; c < n_chunks; c += step) {
    uint32_t cnt = 0;
#pragma unroll 4
    for (int k = 0; k < 16; ++k) {
      const uint64_t i = c * kHxChunk + (uint64_t)k * 64 + lane;
      cnt += (uint32_t)__popcll(__ballot(i < n && key[i] == esc));
    }
    if (lane == 0) zc[c] = cnt;
  }
}

// Values from decoded keys: lo + key, or the next escaped value (ESC types);
// the key itself for u8.  A key no value maps to (above kmax and not the
// escape key; above 255 for u8), an escape rank beyond the stream's escaped
// values, or an escape total that differs from it sets ST_FORMAT in *status.
template <typename T, bool ESC>
__global__ __launch_bounds__(64 * kHxWaves) void k_hx_values(
    const uint16_t* __restrict__ key, uint64_t n, int64_t lo, uint32_t kmax, uint32_t esc_key,
    const T* __restrict__ esc, uint64_t n_esc, const uint32_t* __restrict__ zc,
    const uint32_t* __restrict__ zpre, uint64_t n_chunks, T* __restrict__ out,
    unsigned* __restrict__ status) {
  const int lane = threadIdx.x & 63;
  const uint64_t wave = (uint64_t)blockIdx.x * kHxWaves + (threadIdx.x >> 6);
  const uint64_t step = (uint64_t)gridDim.x * kHxWaves;
  bool bad = false;
  for (uint64_t c = wave; c < n_chunks; c += step) {
    uint64_t run = ESC ? zpre[c] : 0;
    if (ESC && c == n_chunks - 1 && (uint64_t)zpre[c] + zc[c] != n_esc) bad = true;
#pragma unroll 4
    for (int k = 0; k < 16; ++k) {
      const uint64_t i = c * kHxChunk + (uint64_t)k * 64 + lane;
      const bool live = i < n;
      const uint32_t kv = live ? key[i] : 0u;
      if (ESC) {
        const bool e = live && kv == esc_key;
        const uint64_t m = __ballot(e);
        if (live) {
          if (e) {
            const uint64_t r = run + __popcll(m & hx_lanemask_lt());
            if (r < n_esc) out[i] = esc[r];
            else bad = true;
          } else {
            if (kv > kmax) bad = true;
            out[i] = (T)(int64_t)((uint64_t)lo + kv);
          }
        }
        run += __popcll(m);
      } else if (live) {
        if (kv > 255u) bad = true;
        out[i] = (T)kv;
      }
    }
  }
  if (__ballot(bad) && lane == 0) atomicOr(status, (unsigned)ST_FORMAT);
}

unsigned hx_blocks(uint64_t n_chunks) {
  const uint64_t b = (n_chunks + kHxWaves - 1) / kHxWaves;
  return (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(b, 8192));
}

}  // namespace

void launch_hx_keys(const void* in, uint64_t n, int type, int64_t lo, int64_t hi, uint32_t esc,
                    uint16_t* key, uint32_t* zc, hipStream_t s) {
  const uint64_t nc = (n + kHxChunk - 1) / kHxChunk;
  const dim3 grid(hx_blocks(nc)), blk(64 * kHxWaves);
  switch (type) {
    case MGC_HX_U8:
      if ((reinterpret_cast<uintptr_t>(in) | reinterpret_cast<uintptr_t>(key)) % 16 == 0) {
        const uint64_t b = (n / 16 + 255) / 256;
        hipLaunchKernelGGL(k_hx_keys_u8, dim3((unsigned)std::max<uint64_t>(1, std::min<uint64_t>(b, 8192))),
                           dim3(256), 0, s, static_cast<const uint8_t*>(in), n, key);
      } else {
        hipLaunchKernelGGL((k_hx_keys<uint8_t, false>), grid, blk, 0, s,
                           static_cast<const uint8_t*>(in), n, lo, hi, esc, key, zc, nc);
      }
      break;
    case MGC_HX_U16:
      hipLaunchKernelGGL((k_hx_keys<uint16_t, false>), grid, blk, 0, s,
                         static_cast<const uint16_t*>(in), n, lo, hi, esc, key, zc, nc);
      break;
    case MGC_HX_I32:
      hipLaunchKernelGGL((k_hx_keys<int32_t, true>), grid, blk, 0, s,
                         static_cast<const int32_t*>(in), n, lo, hi, esc, key, zc, nc);
      break;
    default:
      hipLaunchKernelGGL((k_hx_keys<int64_t, true>), grid, blk, 0, s,
                         static_cast<const int64_t*>(in), n, lo, hi, esc, key, zc, nc);
  }
}

void launch_hx_place(const void* in, uint64_t n, int type, int64_t lo, int64_t hi,
                     const uint32_t* zc, const uint32_t* zpre, uint8_t* sec, const Layout* lay,
                     hipStream_t s) {
  const uint64_t nc = (n + kHxChunk - 1) / kHxChunk;
  const dim3 grid(hx_blocks(nc)), blk(64 * kHxWaves);
  if (type == MGC_HX_I32)
    hipLaunchKernelGGL(k_hx_place<int32_t>, grid, blk, 0, s, static_cast<const int32_t*>(in), n,
                       lo, hi, zc, zpre, nc, sec, lay);
  else
    hipLaunchKernelGGL(k_hx_place<int64_t>, grid, blk, 0, s, static_cast<const int64_t*>(in), n,
                       lo, hi, zc, zpre, nc, sec, lay);
}

void launch_hx_header(uint8_t* out, int type, uint32_t D, uint32_t C, int64_t base, uint64_t n,
                      const uint32_t* zc, const uint32_t* zpre, const Layout* lay,
                      unsigned long long* res, hipStream_t s) {
  const uint64_t nc = (n + kHxChunk - 1) / kHxChunk;
  const uint32_t width = type == MGC_HX_U8 ? 1 : type == MGC_HX_U16 ? 2 : type == MGC_HX_I32 ? 4 : 8;
  hipLaunchKernelGGL(k_hx_header, dim3(1), dim3(64), 0, s, out, (uint32_t)type, D, C, base, n, zc,
                     zpre, nc, lay, width, res);
}

void launch_hx_count(const uint16_t* key, uint64_t n, uint32_t esc, uint32_t* zc, hipStream_t s) {
  const uint64_t nc = (n + kHxChunk - 1) / kHxChunk;
  hipLaunchKernelGGL(k_hx_count, dim3(hx_blocks(nc)), dim3(64 * kHxWaves), 0, s, key, n, esc, zc,
                     nc);
}

void launch_hx_values(const uint16_t* key, uint64_t n, int type, int64_t lo, uint32_t kmax,
                      uint32_t esc_key,
                      const void* esc, uint64_t n_esc, const uint32_t* zc, const uint32_t* zpre,
                      void* out, unsigned* status, hipStream_t s) {
  const uint64_t nc = (n + kHxChunk - 1) / kHxChunk;
  const dim3 grid(hx_blocks(nc)), blk(64 * kHxWaves);
  if (type == MGC_HX_U8)
    hipLaunchKernelGGL((k_hx_values<uint8_t, false>), grid, blk, 0, s, key, n, lo, kmax, esc_key,
                       static_cast<const uint8_t*>(esc), n_esc, zc, zpre, nc,
                       static_cast<uint8_t*>(out), status);
  else if (type == MGC_HX_I32)
    hipLaunchKernelGGL((k_hx_values<int32_t, true>), grid, blk, 0, s, key, n, lo, kmax, esc_key,
                       static_cast<const int32_t*>(esc), n_esc, zc, zpre, nc,
                       static_cast<int32_t*>(out), status);
  else
    hipLaunchKernelGGL((k_hx_values<int64_t, true>), grid, blk, 0, s, key, n, lo, kmax, esc_key,
                       static_cast<const int64_t*>(esc), n_esc, zc, zpre, nc,
                       static_cast<int64_t*>(out), status);
}

}  // namespace mgc
