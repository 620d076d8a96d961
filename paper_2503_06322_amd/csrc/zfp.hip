// Fixed-rate block transform coding (ZFP-X): Algorithm "ZFP Fix-Rate
// Compression" of Section IV-C.
//
// One thread per block of 4^D values.  A block's values are aligned to its
// largest exponent as P-bit integers (trunc(x 2^(q - e)), q = P - 2 - D),
// transformed per axis (the last axis first) by two levels of reversible
// integer Haar lifting, ordered by total frequency, mapped to negabinary and
// coded bit plane by bit plane under a fixed budget of maxbits bits: a
// "not zero" bit and the biased exponent, then per plane the bits of the
// coefficients already significant, then group tests over the others, each
// followed by their bits up to the next one (the last coefficient's one
// implied).  Every block's bits start at bit b * maxbits of the payload, so
// blocks are coded and decoded independently.  The coefficients stay in
// registers: the coder works on one 64-bit mask per plane (bit i =
// coefficient i's bit), so no register array is indexed at run time.
#include "kernels.hpp"

namespace mgc {
namespace {

constexpr int kZfpThreads = 128;

template <typename T>
struct ZfpType;
template <>
struct ZfpType<float> {
  using I = int32_t;
  using U = uint32_t;
  static constexpr int P = 32, EB = 9, BIAS = 149;
  static constexpr U M = 0xAAAAAAAAu;
};
template <>
struct ZfpType<double> {
  using I = int64_t;
  using U = uint64_t;
  static constexpr int P = 64, EB = 12, BIAS = 1074;
  static constexpr U M = 0xAAAAAAAAAAAAAAAAull;
};

// Block positions (row-major, last axis fastest) sorted by the sum of their
// per-axis frequencies (0, 1, 2, 2 for positions 0..3 of a line), stable.
template <int D>
struct ZfpOrder {
  int p[1 << (2 * D)];
};
template <int D>
constexpr ZfpOrder<D> make_order() {
  constexpr int n = 1 << (2 * D);
  ZfpOrder<D> o{};
  int key[n] = {};
  for (int i = 0; i < n; ++i) {
    int k = 0, r = i;
    for (int a = 0; a < D; ++a) {
      const int c = r & 3;
      k += c == 0 ? 0 : (c == 1 ? 1 : 2);
      r >>= 2;
    }
    key[i] = k;
    o.p[i] = i;
  }
  for (int i = 1; i < n; ++i) {
    const int v = o.p[i];
    int j = i - 1;
    while (j >= 0 && key[o.p[j]] > key[v]) {
      o.p[j + 1] = o.p[j];
      --j;
    }
    o.p[j + 1] = v;
  }
  return o;
}

template <typename I>
__device__ __forceinline__ void lift(I& a, I& b) {  // (a, b) -> (s, t)
  const I t = a - b;
  a = b + (t >> 1);
  b = t;
}
template <typename I>
__device__ __forceinline__ void unlift(I& s, I& t) {  // (s, t) -> (a, b)
  const I b = s - (t >> 1);
  s = b + t;
  t = b;
}

// Two lifting levels on the line (v0, v1, v2, v3) -> (S, T, t0, t1).
template <typename I>
__device__ __forceinline__ void fwd_line(I& v0, I& v1, I& v2, I& v3) {
  lift(v0, v1);  // v0 = s0, v1 = t0
  lift(v2, v3);  // v2 = s1, v3 = t1
  I S = v0, T = v2;
  lift(S, T);
  const I t0 = v1, t1 = v3;
  v0 = S;
  v1 = T;
  v2 = t0;
  v3 = t1;
}
template <typename I>
__device__ __forceinline__ void inv_line(I& c0, I& c1, I& c2, I& c3) {
  I s0 = c0, s1 = c1;
  unlift(s0, s1);  // (S, T) -> (s0, s1)
  I a0 = s0, b0 = c2;
  unlift(a0, b0);
  I a1 = s1, b1 = c3;
  unlift(a1, b1);
  c0 = a0;
  c1 = b0;
  c2 = a1;
  c3 = b1;
}

template <int D, typename I>
__device__ __forceinline__ void forward(I* v) {
  constexpr int n = 1 << (2 * D);
#pragma unroll
  for (int ax = D - 1; ax >= 0; --ax) {
    const int s = 1 << (2 * (D - 1 - ax));
#pragma unroll
    for (int i = 0; i < n; ++i)
      if (((i / s) & 3) == 0) fwd_line(v[i], v[i + s], v[i + 2 * s], v[i + 3 * s]);
  }
}
template <int D, typename I>
__device__ __forceinline__ void inverse(I* v) {
  constexpr int n = 1 << (2 * D);
#pragma unroll
  for (int ax = 0; ax < D; ++ax) {
    const int s = 1 << (2 * (D - 1 - ax));
#pragma unroll
    for (int i = 0; i < n; ++i)
      if (((i / s) & 3) == 0) inv_line(v[i], v[i + s], v[i + 2 * s], v[i + 3 * s]);
  }
}

// Global index of position i (row-major in the block) of the block at b0,
// the block's last value repeated past the end of every axis.
struct ZfpIdx {
  uint64_t n[3];   // extents of the ndim axes (axis 0 first)
  uint64_t nb[3];  // blocks per axis
};
template <int D>
__device__ __forceinline__ uint64_t zfp_src(const ZfpIdx& g, const uint64_t* b0, int i) {
  uint64_t off = 0;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    const int c = (i >> (2 * (D - 1 - a))) & 3;
    const uint64_t x = min(b0[a] + (uint64_t)c, g.n[a] - 1);
    off = off * g.n[a] + x;
  }
  return off;
}
__device__ __forceinline__ void block_origin(const ZfpIdx& g, int D, uint64_t b, uint64_t* b0) {
  for (int a = D - 1; a >= 0; --a) {
    b0[a] = (b % g.nb[a]) * 4;
    b /= g.nb[a];
  }
}

// Sequential writer of a block's bits at a global bit position.  Whole
// 64-bit words are stored directly when blocks are word-aligned; otherwise
// OR-ed (the payload is cleared first: neighbouring blocks share words).
struct BitWriter {
  unsigned long long* w;
  uint64_t pos;
  unsigned long long acc = 0;
  int nacc = 0;
  bool aligned;
  __device__ void flush() {
    if (nacc == 0) return;
    const uint64_t wi = pos >> 6;
    const int s = (int)(pos & 63);
    if (aligned) {
      w[wi] = acc;
    } else {
      atomicOr(&w[wi], acc << s);
      // the bits that spill into the next word (none past the block's last bit)
      if (s && s + nacc > 64) atomicOr(&w[wi + 1], acc >> (64 - s));
    }
    pos += 64;
    acc = 0;
    nacc = 0;
  }
  __device__ __forceinline__ void put(unsigned long long bit) {
    acc |= bit << nacc;
    if (++nacc == 64) flush();
  }
  // the low c bits of v (nothing above them set), c <= 64
  __device__ __forceinline__ void put_bits(unsigned long long v, int c) {
    if (c == 0) return;
    acc |= v << nacc;
    const int room = 64 - nacc;
    if (c < room) {
      nacc += c;
      return;
    }
    nacc = 64;
    flush();
    if (c > room) {
      acc = v >> room;
      nacc = c - room;
    }
  }
};

struct BitReader {
  const unsigned long long* w;
  uint64_t pos;
  // the next c bits (c <= 64, all within the block), the first in bit 0
  __device__ __forceinline__ unsigned long long peek(int c) const {
    if (c == 0) return 0ull;
    const uint64_t wi = pos >> 6;
    const int s = (int)(pos & 63);
    unsigned long long v = w[wi] >> s;
    if (s + c > 64) v |= w[wi + 1] << (64 - s);
    return c == 64 ? v : v & ((1ull << c) - 1ull);
  }
  __device__ __forceinline__ unsigned long long get_bits(int c) {
    const unsigned long long v = peek(c);
    pos += (uint64_t)c;
    return v;
  }
  __device__ __forceinline__ unsigned get() { return (unsigned)get_bits(1); }
};

template <typename T, int D>
__global__ __launch_bounds__(kZfpThreads) void k_zfp_encode(const T* __restrict__ in,
                                                            const ZfpIdx g, uint64_t nblocks,
                                                            uint32_t maxbits,
                                                            unsigned long long* __restrict__ words,
                                                            unsigned* __restrict__ status) {
  using Z = ZfpType<T>;
  using I = typename Z::I;
  using U = typename Z::U;
  constexpr int n = 1 << (2 * D);
  constexpr int q = Z::P - 2 - D;
  constexpr ZfpOrder<D> ord = make_order<D>();
  const uint64_t b = (uint64_t)blockIdx.x * kZfpThreads + threadIdx.x;
  if (b >= nblocks) return;
  uint64_t b0[3];
  block_origin(g, D, b, b0);
  T x[n];
#pragma unroll
  for (int i = 0; i < n; ++i) x[i] = in[zfp_src<D>(g, b0, i)];
  double mx = 0.0;
  bool bad = false;
#pragma unroll
  for (int i = 0; i < n; ++i) {
    const double a = fabs((double)x[i]);
    bad = bad || !(a <= 1.7976931348623157e308);
    mx = fmax(mx, a);
  }
  BitWriter bw{words, b * (uint64_t)maxbits, 0, 0, (maxbits & 63u) == 0};
  if (bad) {
    atomicOr(status, ST_NONFINITE);
    return;
  }
  int budget = (int)maxbits;
  if (mx == 0.0) {
    bw.put(0);
  } else {
    int e;
    (void)frexp(mx, &e);
    bw.put(1);
    const unsigned ebits = (unsigned)(e + Z::BIAS);
#pragma unroll
    for (int j = 0; j < Z::EB; ++j) bw.put((ebits >> j) & 1u);
    budget -= 1 + Z::EB;
    I v[n];
#pragma unroll
    for (int i = 0; i < n; ++i) v[i] = (I)trunc(ldexp((double)x[i], q - e));
    forward<D>(v);
    U u[n];
#pragma unroll
    for (int i = 0; i < n; ++i) u[i] = ((U)v[ord.p[i]] + Z::M) ^ Z::M;
    // Runs of bits go out in one write each: the significant coefficients'
    // bits of a plane, and for each group test the zeros up to the next one
    // with that one (a run stops early where the budget ends).
    int m = 0, B = budget;
    for (int k = Z::P - 1; k >= 0 && B > 0; --k) {
      unsigned long long xm = 0;
#pragma unroll
      for (int i = 0; i < n; ++i) xm |= (unsigned long long)((u[i] >> k) & 1u) << i;
      const int t = min(m, B);
      bw.put_bits(t == 64 ? xm : xm & ((1ull << t) - 1ull), t);
      B -= t;
      if (t < m) break;
      xm = m < 64 ? xm >> m : 0ull;
      while (m < n && B > 0) {
        if (!xm) {
          bw.put_bits(0ull, 1);
          --B;
          break;
        }
        bw.put_bits(1ull, 1);
        --B;
        const int z = __builtin_ctzll(xm);  // the next one is coefficient m + z
        if (m + z == n - 1) {               // the last coefficient: its one is implied
          const int c = min(z, B);
          bw.put_bits(0ull, c);
          B -= c;
          m += c < z ? c : z + 1;
          break;
        }
        if (B >= z + 1) {
          bw.put_bits(1ull << z, z + 1);
          B -= z + 1;
          m += z + 1;
          xm = z + 1 < 64 ? xm >> (z + 1) : 0ull;
        } else {
          bw.put_bits(0ull, B);
          m += B;
          B = 0;
        }
      }
    }
  }
  if (bw.aligned) {
    // the rest of the block's words hold zeros
    bw.flush();
    const uint64_t end = (b + 1) * (uint64_t)maxbits;
    for (uint64_t p = bw.pos; p < end; p += 64) words[p >> 6] = 0ull;
  } else {
    bw.flush();
  }
}

template <typename T, int D>
__global__ __launch_bounds__(kZfpThreads) void k_zfp_decode(
    const unsigned long long* __restrict__ words, const ZfpIdx g, uint64_t nblocks,
    uint32_t maxbits, T* __restrict__ out) {
  using Z = ZfpType<T>;
  using I = typename Z::I;
  using U = typename Z::U;
  constexpr int n = 1 << (2 * D);
  constexpr int q = Z::P - 2 - D;
  constexpr ZfpOrder<D> ord = make_order<D>();
  const uint64_t b = (uint64_t)blockIdx.x * kZfpThreads + threadIdx.x;
  if (b >= nblocks) return;
  uint64_t b0[3];
  block_origin(g, D, b, b0);
  BitReader br{words, b * (uint64_t)maxbits};
  I v[n];
  int e = 0;
  if (!br.get()) {
#pragma unroll
    for (int i = 0; i < n; ++i) v[i] = 0;
  } else {
    unsigned ebits = 0;
#pragma unroll
    for (int j = 0; j < Z::EB; ++j) ebits |= br.get() << j;
    e = (int)ebits - Z::BIAS;
    U u[n];
#pragma unroll
    for (int i = 0; i < n; ++i) u[i] = 0;
    int m = 0, B = (int)maxbits - 1 - Z::EB;
    for (int k = Z::P - 1; k >= 0 && B > 0; --k) {
      const int t = min(m, B);
      unsigned long long ym = br.get_bits(t);
      B -= t;
      const bool stop = t < m;
      while (!stop && m < n && B > 0) {
        const unsigned gbit = br.get();
        --B;
        if (!gbit) break;
        if (m == n - 1) {  // the last coefficient's one is implied
          ym |= 1ull << m;
          ++m;
          break;
        }
        // the next one within the budget and before the last coefficient
        const int L = min(B, n - 1 - m);
        const unsigned long long v = br.peek(L);
        if (v) {
          const int r = __builtin_ctzll(v);
          br.pos += (uint64_t)(r + 1);
          B -= r + 1;
          ym |= 1ull << (m + r);
          m += r + 1;
        } else {
          br.pos += (uint64_t)L;
          B -= L;
          m += L;
          if (m == n - 1) {
            ym |= 1ull << m;
            ++m;
          }
          break;
        }
      }
#pragma unroll
      for (int i = 0; i < n; ++i) u[i] |= (U)((ym >> i) & 1ull) << k;
      if (stop) break;
    }
#pragma unroll
    for (int i = 0; i < n; ++i) v[ord.p[i]] = (I)((u[i] ^ Z::M) - Z::M);
    inverse<D>(v);
  }
#pragma unroll
  for (int i = 0; i < n; ++i) {
    // positions past the end of an axis repeat values already written
    bool inside = true;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const int c = (i >> (2 * (D - 1 - a))) & 3;
      inside = inside && b0[a] + (uint64_t)c < g.n[a];
    }
    if (inside) out[zfp_src<D>(g, b0, i)] = (T)ldexp((double)v[i], e - q);
  }
}

__global__ void k_zfp_header(uint8_t* __restrict__ out, ZfpHead h, const unsigned* status,
                             unsigned long long* __restrict__ res) {
  if (threadIdx.x != 0) return;
  const unsigned st = status ? *status : 0u;
  res[0] = (st & ST_NONFINITE) ? (unsigned long long)MGC_EINVAL : 0ull;
  res[1] = (st & ST_NONFINITE) ? 0ull : h.total;
  const uint8_t* src = reinterpret_cast<const uint8_t*>(&h);
  for (int i = 0; i < (int)sizeof(ZfpHead); ++i) out[i] = src[i];
}

template <typename T, int D>
void enc(const void* in, const ZfpIdx& g, uint64_t nblocks, uint32_t maxbits,
         unsigned long long* words, unsigned* status, hipStream_t s) {
  const unsigned grid = (unsigned)((nblocks + kZfpThreads - 1) / kZfpThreads);
  hipLaunchKernelGGL((k_zfp_encode<T, D>), dim3(grid), dim3(kZfpThreads), 0, s,
                     static_cast<const T*>(in), g, nblocks, maxbits, words, status);
}
template <typename T, int D>
void dec(const unsigned long long* words, const ZfpIdx& g, uint64_t nblocks, uint32_t maxbits,
         void* out, hipStream_t s) {
  const unsigned grid = (unsigned)((nblocks + kZfpThreads - 1) / kZfpThreads);
  hipLaunchKernelGGL((k_zfp_decode<T, D>), dim3(grid), dim3(kZfpThreads), 0, s, words, g,
                     nblocks, maxbits, static_cast<T*>(out));
}

ZfpIdx zfp_idx(int ndim, const uint64_t* shape) {
  ZfpIdx g{};
  for (int a = 0; a < ndim; ++a) {
    g.n[a] = shape[a];
    g.nb[a] = (shape[a] + 3) / 4;
  }
  return g;
}

}  // namespace

void launch_zfp_encode(const void* in, bool f64, int ndim, const uint64_t* shape,
                       uint64_t nblocks, uint32_t maxbits, uint8_t* out, unsigned* status,
                       const ZfpHead& h, unsigned long long* res, hipStream_t s) {
  const ZfpIdx g = zfp_idx(ndim, shape);
  unsigned long long* words = reinterpret_cast<unsigned long long*>(out + kZfpHeaderBytes);
  if (nblocks > 0) {
    if (f64) {
      if (ndim == 1) enc<double, 1>(in, g, nblocks, maxbits, words, status, s);
      else if (ndim == 2) enc<double, 2>(in, g, nblocks, maxbits, words, status, s);
      else enc<double, 3>(in, g, nblocks, maxbits, words, status, s);
    } else {
      if (ndim == 1) enc<float, 1>(in, g, nblocks, maxbits, words, status, s);
      else if (ndim == 2) enc<float, 2>(in, g, nblocks, maxbits, words, status, s);
      else enc<float, 3>(in, g, nblocks, maxbits, words, status, s);
    }
  }
  hipLaunchKernelGGL(k_zfp_header, dim3(1), dim3(64), 0, s, out, h, status, res);
}

void launch_zfp_decode(const uint8_t* in, bool f64, int ndim, const uint64_t* shape,
                       uint64_t nblocks, uint32_t maxbits, void* out, hipStream_t s) {
  const ZfpIdx g = zfp_idx(ndim, shape);
  const unsigned long long* words =
      reinterpret_cast<const unsigned long long*>(in + kZfpHeaderBytes);
  if (f64) {
    if (ndim == 1) dec<double, 1>(words, g, nblocks, maxbits, out, s);
    else if (ndim == 2) dec<double, 2>(words, g, nblocks, maxbits, out, s);
    else dec<double, 3>(words, g, nblocks, maxbits, out, s);
  } else {
    if (ndim == 1) dec<float, 1>(words, g, nblocks, maxbits, out, s);
    else if (ndim == 2) dec<float, 2>(words, g, nblocks, maxbits, out, s);
    else dec<float, 3>(words, g, nblocks, maxbits, out, s);
  }
}

}  // namespace mgc
