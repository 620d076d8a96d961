// Multilevel transform kernels for gfx950 (wave64, no MFMA: every step is a
// short stencil or a tridiagonal recurrence, bound by HBM bandwidth).
//
// Decomposition of level l (Algorithm 1 and Section IV-A of the paper):
//  * lerp: coefficient of a new node = value minus the multilinear
//    interpolant from its coarse neighbours, quantised on the spot
//    (level-wise linear quantisation) and written in stream order;
//  * mass_trans: f = (P^T M_l) G_l on the coarse grid, a separable 5-tap
//    stencil per axis evaluated on an LDS tile with a halo of two nodes;
//  * tridiag: G_{l-1} = M_{l-1}^{-1} f along each axis (Thomas sweeps).
// Because P^T M_l P = M_{l-1} (Galerkin identity of nested hat spaces), the
// L2 projection M_{l-1}^{-1} P^T M_l G_l equals G_l[coarse] plus the
// correction of the coefficients, so the add step is folded into the solve.
//
// Recomposition inverts each level: f = (P^T M_l) c_l, z = M_{l-1}^{-1} f,
// G_l[coarse] = G_{l-1} - z (fused into the last sweep), then
// G_l = P G_l[coarse] + c_l.
#include "kernels.hpp"

#include <cmath>

namespace mgc {

namespace {

__device__ __forceinline__ int64_t cpos(int64_t j, int64_t nf) {
  int64_t p = 2 * j;
  return p < nf ? p : nf - 1;
}
__device__ __forceinline__ bool is_new(int64_t i, int64_t nf) {
  return (i & 1) && i != nf - 1;
}
__device__ __forceinline__ int64_t coarse_idx(int64_t i, int64_t nf) {
  return (i == nf - 1 && !(nf & 1)) ? (nf >> 1) : (i >> 1);
}

// Stream position of fine point (i0,i1,i2) with new-node flags n0,n1,n2.
__device__ __forceinline__ int64_t stream_index(const LevelGeom& g, int64_t i0, int64_t i1,
                                                int64_t i2, bool n0, bool n1, bool n2) {
  int m = (n0 ? (1 << g.bit[0]) : 0) | (n1 ? (1 << g.bit[1]) : 0) |
          (n2 ? (1 << g.bit[2]) : 0);
  const int64_t e1 = n1 ? g.nf[1] - g.nc[1] : g.nc[1];
  const int64_t e2 = n2 ? g.nf[2] - g.nc[2] : g.nc[2];
  const int64_t j0 = n0 ? (i0 >> 1) : coarse_idx(i0, g.nf[0]);
  const int64_t j1 = n1 ? (i1 >> 1) : coarse_idx(i1, g.nf[1]);
  const int64_t j2 = n2 ? (i2 >> 1) : coarse_idx(i2, g.nf[2]);
  return g.level_off + g.sub_off[m] + (j0 * e1 + j1) * e2 + j2;
}

// Linear quantisation of one coefficient: k = rint(c * r) in FP64 (round
// half to even).  |k| < S/2 -> symbol k + S/2; otherwise the escape symbol 0
// and an (position, k) record.
__device__ __forceinline__ void emit_q(int64_t pos, double c, double r, uint16_t* sym,
                                       const OutlierBuf& ob, unsigned* status) {
  const double t = rint(c * r);
  if (fabs(t) < 32768.0) {
    sym[pos] = (uint16_t)(int)(t + 32768.0);
    return;
  }
  sym[pos] = 0;
  int64_t k = 0;
  if (fabs(t) < 4611686018427387904.0) k = (int64_t)t;
  else atomicOr(status, ST_RANGE);
  unsigned long long i = atomicAdd(ob.count, 1ull);
  if (i < ob.cap) {
    ob.pos[i] = (uint32_t)pos;
    ob.val[i] = k;
  }
}

// Coefficient at stream position pos: raw FP64, or dequantised k * q with
// escaped values found by binary search in the sorted outlier positions.
template <bool RAW>
__device__ __forceinline__ double coeff_at(const CoeffSrc& s, int64_t pos, double q) {
  if (RAW) return s.raw[pos];
  const uint16_t v = s.sym[pos];
  int64_t k;
  if (v != 0) {
    k = (int64_t)v - 32768;
  } else {
    int64_t lo = 0, hi = s.n_out;
    while (lo < hi) {
      int64_t mid = (lo + hi) >> 1;
      if (s.opos[mid] < (uint64_t)pos) lo = mid + 1;
      else hi = mid;
    }
    k = (lo < s.n_out && s.opos[lo] == (uint64_t)pos) ? s.oval[lo] : 0;
  }
  return (double)k * q;
}

template <typename T>
__device__ __forceinline__ double wave_sum(T v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// ------------------------------------------------------------ range pass
template <typename T>
__global__ __launch_bounds__(256) void k_range_partial(const T* __restrict__ u, int64_t N,
                                                        double* __restrict__ part) {
  double mn = INFINITY, mx = -INFINITY, ss = 0.0, bad = 0.0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += stride) {
    const double v = (double)u[i];
    if (!isfinite(v)) {
      bad = 1.0;
    } else {
      mn = fmin(mn, v);
      mx = fmax(mx, v);
      ss += v * v;
    }
  }
  for (int o = 32; o > 0; o >>= 1) {
    mn = fmin(mn, __shfl_xor(mn, o, 64));
    mx = fmax(mx, __shfl_xor(mx, o, 64));
    ss += __shfl_xor(ss, o, 64);
    bad = fmax(bad, __shfl_xor(bad, o, 64));
  }
  __shared__ double sm[4][4];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0) {
    sm[w][0] = mn;
    sm[w][1] = mx;
    sm[w][2] = ss;
    sm[w][3] = bad;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 1; k < 4; ++k) {
      sm[0][0] = fmin(sm[0][0], sm[k][0]);
      sm[0][1] = fmax(sm[0][1], sm[k][1]);
      sm[0][2] += sm[k][2];
      sm[0][3] = fmax(sm[0][3], sm[k][3]);
    }
    for (int k = 0; k < 4; ++k) part[4 * blockIdx.x + k] = sm[0][k];
  }
}

__global__ __launch_bounds__(64) void k_range_final(const double* __restrict__ part, int nb,
                                                     double* __restrict__ out) {
  if (threadIdx.x != 0) return;
  double mn = INFINITY, mx = -INFINITY, ss = 0.0, bad = 0.0;
  for (int b = 0; b < nb; ++b) {
    mn = fmin(mn, part[4 * b + 0]);
    mx = fmax(mx, part[4 * b + 1]);
    ss += part[4 * b + 2];
    bad = fmax(bad, part[4 * b + 3]);
  }
  out[0] = mn;
  out[1] = mx;
  out[2] = ss;
  out[3] = bad;
}

// ----------------------------------------------- decomposition of one level
// Coarse output tile TZ x TY x TX (an extent of 1 marks an inactive axis).
template <int T>
struct Ext {
  static constexpr int v = T == 1 ? 1 : 2 * T + 3;
};

template <typename Tin, int TZ, int TY, int TX, bool QUANT>
__global__ __launch_bounds__(256) void k_dec_level(const Tin* __restrict__ G, const LevelGeom g,
                                                    double* __restrict__ fout,
                                                    uint16_t* __restrict__ sym,
                                                    double* __restrict__ raw, const double r,
                                                    const OutlierBuf ob,
                                                    unsigned* __restrict__ status) {
  constexpr int E0 = Ext<TZ>::v, E1 = Ext<TY>::v, E2 = Ext<TX>::v;
  constexpr int TILE_BYTES = E0 * E1 * E2 * (int)sizeof(Tin);
  constexpr int B_BYTES = E0 * TY * TX * (int)sizeof(double);
  static_assert(B_BYTES <= TILE_BYTES, "B aliases the tile");
  __shared__ __align__(16) unsigned char smem[TILE_BYTES];
  __shared__ double A[E0 * E1 * TX];
  Tin* tile = reinterpret_cast<Tin*>(smem);
  double* B = reinterpret_cast<double*>(smem);

  const int tid = threadIdx.x;
  const int T[3] = {TZ, TY, TX};
  const int64_t c0[3] = {(int64_t)blockIdx.z * TZ, (int64_t)blockIdx.y * TY,
                         (int64_t)blockIdx.x * TX};
  int tk[3], ext[3], olo_rel[3], oext[3];
  int64_t lo[3];
  for (int k = 0; k < 3; ++k) {
    const int64_t nf = g.nf[k], nc = g.nc[k];
    tk[k] = (int)min<int64_t>(T[k], nc - c0[k]);
    lo[k] = max<int64_t>(cpos(c0[k], nf) - 2, 0);
    const int64_t hi = min<int64_t>(cpos(c0[k] + tk[k] - 1, nf) + 2, nf - 1);
    ext[k] = (int)(hi - lo[k] + 1);
    const int64_t olo = 2 * c0[k];
    const int64_t ohi = (c0[k] + tk[k] >= nc) ? nf : 2 * (c0[k] + tk[k]);
    olo_rel[k] = (int)(olo - lo[k]);
    oext[k] = (int)(ohi - olo);
  }
  // load the fine tile with its halo
  const int n_ld = ext[0] * ext[1] * ext[2];
  const int e12 = ext[1] * ext[2];
  for (int i = tid; i < n_ld; i += 256) {
    const int z = i / e12, rem = i - z * e12, y = rem / ext[2], x = rem - y * ext[2];
    tile[(z * E1 + y) * E2 + x] =
        G[((lo[0] + z) * g.nf[1] + (lo[1] + y)) * g.nf[2] + lo[2] + x];
  }
  __syncthreads();

  // lerp: coefficients of the owned new nodes
  const int n_own = oext[0] * oext[1] * oext[2];
  const int o12 = oext[1] * oext[2];
  for (int i = tid; i < n_own; i += 256) {
    const int a = i / o12, rem = i - a * o12, b = rem / oext[2], c = rem - b * oext[2];
    const int z = olo_rel[0] + a, y = olo_rel[1] + b, x = olo_rel[2] + c;
    const int64_t i0 = lo[0] + z, i1 = lo[1] + y, i2 = lo[2] + x;
    const bool n0 = is_new(i0, g.nf[0]), n1 = is_new(i1, g.nf[1]), n2 = is_new(i2, g.nf[2]);
    if (!(n0 || n1 || n2)) continue;
    double w0[2] = {1.0, 0.0}, w1[2] = {1.0, 0.0}, w2[2] = {1.0, 0.0};
    int d0[2] = {0, 0}, d1[2] = {0, 0}, d2[2] = {0, 0};
    int k0 = 1, k1 = 1, k2 = 1;
    if (n0) { w0[0] = g.ax[0].wl[i0]; w0[1] = g.ax[0].wr[i0]; d0[0] = -1; d0[1] = 1; k0 = 2; }
    if (n1) { w1[0] = g.ax[1].wl[i1]; w1[1] = g.ax[1].wr[i1]; d1[0] = -1; d1[1] = 1; k1 = 2; }
    if (n2) { w2[0] = g.ax[2].wl[i2]; w2[1] = g.ax[2].wr[i2]; d2[0] = -1; d2[1] = 1; k2 = 2; }
    double interp = 0.0;
    for (int p = 0; p < k0; ++p)
      for (int q = 0; q < k1; ++q) {
        double acc = 0.0;
        for (int s = 0; s < k2; ++s)
          acc += w2[s] * (double)tile[((z + d0[p]) * E1 + y + d1[q]) * E2 + x + d2[s]];
        interp += w0[p] * w1[q] * acc;
      }
    const double cval = (double)tile[(z * E1 + y) * E2 + x] - interp;
    const int64_t pos = stream_index(g, i0, i1, i2, n0, n1, n2);
    if (QUANT) emit_q(pos, cval, r, sym, ob, status);
    else raw[pos] = cval;
  }

  // mass_trans along axis 2 (contiguous)
  {
    const double* W = g.ax[2].W;
    const int n = ext[0] * ext[1] * tk[2];
    const int per = ext[1] * tk[2];
    for (int i = tid; i < n; i += 256) {
      const int z = i / per, rem = i - z * per, y = rem / tk[2], cx = rem - y * tk[2];
      const int64_t j = c0[2] + cx, p = cpos(j, g.nf[2]);
      double acc = 0.0;
#pragma unroll
      for (int d = -2; d <= 2; ++d) {
        const int64_t f = p + d;
        if (f >= 0 && f < g.nf[2])
          acc += W[5 * j + d + 2] * (double)tile[(z * E1 + y) * E2 + (int)(f - lo[2])];
      }
      A[(z * E1 + y) * TX + cx] = acc;
    }
  }
  __syncthreads();
  // along axis 1
  {
    const double* W = g.ax[1].W;
    const int n = ext[0] * tk[1] * tk[2];
    const int per = tk[1] * tk[2];
    for (int i = tid; i < n; i += 256) {
      const int z = i / per, rem = i - z * per, cy = rem / tk[2], cx = rem - cy * tk[2];
      const int64_t j = c0[1] + cy, p = cpos(j, g.nf[1]);
      double acc = 0.0;
#pragma unroll
      for (int d = -2; d <= 2; ++d) {
        const int64_t f = p + d;
        if (f >= 0 && f < g.nf[1]) acc += W[5 * j + d + 2] * A[(z * E1 + (int)(f - lo[1])) * TX + cx];
      }
      B[(z * TY + cy) * TX + cx] = acc;
    }
  }
  __syncthreads();
  // along axis 0, to global memory
  {
    const double* W = g.ax[0].W;
    const int n = tk[0] * tk[1] * tk[2];
    const int per = tk[1] * tk[2];
    for (int i = tid; i < n; i += 256) {
      const int cz = i / per, rem = i - cz * per, cy = rem / tk[2], cx = rem - cy * tk[2];
      const int64_t j = c0[0] + cz, p = cpos(j, g.nf[0]);
      double acc = 0.0;
#pragma unroll
      for (int d = -2; d <= 2; ++d) {
        const int64_t f = p + d;
        if (f >= 0 && f < g.nf[0]) acc += W[5 * j + d + 2] * B[((int)(f - lo[0]) * TY + cy) * TX + cx];
      }
      fout[((c0[0] + cz) * g.nc[1] + c0[1] + cy) * g.nc[2] + c0[2] + cx] = acc;
    }
  }
}

// ------------------------------------------------------------- tridiagonal
// One thread per line; lines of the strided axes are adjacent across lanes.
template <int AXIS>
__global__ __launch_bounds__(256) void k_thomas(double* __restrict__ x, int64_t n0, int64_t n1,
                                                 int64_t n2, const double* __restrict__ ta,
                                                 const double* __restrict__ tm,
                                                 const double* __restrict__ tc,
                                                 const double* __restrict__ sub) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t len, stride, base;
  if (AXIS == 2) {
    if (t >= n0 * n1) return;
    len = n2;
    stride = 1;
    base = t * n2;
  } else if (AXIS == 1) {
    if (t >= n0 * n2) return;
    const int64_t i0 = t / n2, i2 = t - i0 * n2;
    len = n1;
    stride = n2;
    base = i0 * n1 * n2 + i2;
  } else {
    if (t >= n1 * n2) return;
    len = n0;
    stride = n1 * n2;
    base = t;
  }
  double* p = x + base;
  double prev = p[0] * tm[0];
  p[0] = prev;
  for (int64_t i = 1; i < len; ++i) {
    const double v = (p[i * stride] - ta[i] * prev) * tm[i];
    p[i * stride] = v;
    prev = v;
  }
  double nxt = prev;
  if (sub) p[(len - 1) * stride] = sub[base + (len - 1) * stride] - nxt;
  for (int64_t i = len - 2; i >= 0; --i) {
    const double v = p[i * stride] - tc[i] * nxt;
    p[i * stride] = sub ? sub[base + i * stride] - v : v;
    nxt = v;
  }
}

template <typename Tin, bool QUANT>
__global__ __launch_bounds__(256) void k_level0(const Tin* __restrict__ G0, int64_t m0,
                                                 uint16_t* __restrict__ sym,
                                                 double* __restrict__ raw, double r,
                                                 const OutlierBuf ob, unsigned* status) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m0; i += stride) {
    const double c = (double)G0[i];
    if (QUANT) emit_q(i, c, r, sym, ob, status);
    else raw[i] = c;
  }
}

// --------------------------------------------- recomposition of one level
template <int TZ, int TY, int TX, bool RAW>
__global__ __launch_bounds__(256) void k_rec_restrict(const LevelGeom g, const CoeffSrc src,
                                                       const double q,
                                                       double* __restrict__ fout) {
  constexpr int E0 = Ext<TZ>::v, E1 = Ext<TY>::v, E2 = Ext<TX>::v;
  __shared__ double tile[E0 * E1 * E2];
  __shared__ double A[E0 * E1 * TX];
  double* B = tile;
  static_assert(E0 * TY * TX <= E0 * E1 * E2, "B aliases the tile");
  const int tid = threadIdx.x;
  const int T[3] = {TZ, TY, TX};
  const int64_t c0[3] = {(int64_t)blockIdx.z * TZ, (int64_t)blockIdx.y * TY,
                         (int64_t)blockIdx.x * TX};
  int tk[3], ext[3];
  int64_t lo[3];
  for (int k = 0; k < 3; ++k) {
    const int64_t nf = g.nf[k], nc = g.nc[k];
    tk[k] = (int)min<int64_t>(T[k], nc - c0[k]);
    lo[k] = max<int64_t>(cpos(c0[k], nf) - 2, 0);
    const int64_t hi = min<int64_t>(cpos(c0[k] + tk[k] - 1, nf) + 2, nf - 1);
    ext[k] = (int)(hi - lo[k] + 1);
  }
  const int n_ld = ext[0] * ext[1] * ext[2];
  const int e12 = ext[1] * ext[2];
  for (int i = tid; i < n_ld; i += 256) {
    const int z = i / e12, rem = i - z * e12, y = rem / ext[2], x = rem - y * ext[2];
    const int64_t i0 = lo[0] + z, i1 = lo[1] + y, i2 = lo[2] + x;
    const bool n0 = is_new(i0, g.nf[0]), n1 = is_new(i1, g.nf[1]), n2 = is_new(i2, g.nf[2]);
    double v = 0.0;
    if (n0 || n1 || n2) v = coeff_at<RAW>(src, stream_index(g, i0, i1, i2, n0, n1, n2), q);
    tile[(z * E1 + y) * E2 + x] = v;
  }
  __syncthreads();
  {
    const double* W = g.ax[2].W;
    const int n = ext[0] * ext[1] * tk[2];
    const int per = ext[1] * tk[2];
    for (int i = tid; i < n; i += 256) {
      const int z = i / per, rem = i - z * per, y = rem / tk[2], cx = rem - y * tk[2];
      const int64_t j = c0[2] + cx, p = cpos(j, g.nf[2]);
      double acc = 0.0;
#pragma unroll
      for (int d = -2; d <= 2; ++d) {
        const int64_t f = p + d;
        if (f >= 0 && f < g.nf[2]) acc += W[5 * j + d + 2] * tile[(z * E1 + y) * E2 + (int)(f - lo[2])];
      }
      A[(z * E1 + y) * TX + cx] = acc;
    }
  }
  __syncthreads();
  {
    const double* W = g.ax[1].W;
    const int n = ext[0] * tk[1] * tk[2];
    const int per = tk[1] * tk[2];
    for (int i = tid; i < n; i += 256) {
      const int z = i / per, rem = i - z * per, cy = rem / tk[2], cx = rem - cy * tk[2];
      const int64_t j = c0[1] + cy, p = cpos(j, g.nf[1]);
      double acc = 0.0;
#pragma unroll
      for (int d = -2; d <= 2; ++d) {
        const int64_t f = p + d;
        if (f >= 0 && f < g.nf[1]) acc += W[5 * j + d + 2] * A[(z * E1 + (int)(f - lo[1])) * TX + cx];
      }
      B[(z * TY + cy) * TX + cx] = acc;
    }
  }
  __syncthreads();
  {
    const double* W = g.ax[0].W;
    const int n = tk[0] * tk[1] * tk[2];
    const int per = tk[1] * tk[2];
    for (int i = tid; i < n; i += 256) {
      const int cz = i / per, rem = i - cz * per, cy = rem / tk[2], cx = rem - cy * tk[2];
      const int64_t j = c0[0] + cz, p = cpos(j, g.nf[0]);
      double acc = 0.0;
#pragma unroll
      for (int d = -2; d <= 2; ++d) {
        const int64_t f = p + d;
        if (f >= 0 && f < g.nf[0]) acc += W[5 * j + d + 2] * B[((int)(f - lo[0]) * TY + cy) * TX + cx];
      }
      fout[((c0[0] + cz) * g.nc[1] + c0[1] + cy) * g.nc[2] + c0[2] + cx] = acc;
    }
  }
}

template <typename Tout, bool RAW>
__global__ __launch_bounds__(256) void k_rec_interp(const double* __restrict__ Gc,
                                                     const LevelGeom g, const CoeffSrc src,
                                                     const double q, Tout* __restrict__ out) {
  const int64_t i2 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i2 >= g.nf[2]) return;
  const int64_t rows = g.nf[0] * g.nf[1];
  const bool n2 = is_new(i2, g.nf[2]);
  int64_t j2[2];
  double w2[2];
  int k2 = 1;
  if (n2) {
    j2[0] = i2 >> 1;
    j2[1] = (i2 >> 1) + 1;
    w2[0] = g.ax[2].wl[i2];
    w2[1] = g.ax[2].wr[i2];
    k2 = 2;
  } else {
    j2[0] = coarse_idx(i2, g.nf[2]);
    w2[0] = 1.0;
  }
  for (int64_t row = blockIdx.y; row < rows; row += gridDim.y) {
    const int64_t i0 = row / g.nf[1], i1 = row - i0 * g.nf[1];
    const bool n0 = is_new(i0, g.nf[0]), n1 = is_new(i1, g.nf[1]);
    int64_t j0[2], j1[2];
    double w0[2], w1[2];
    int k0 = 1, k1 = 1;
    if (n0) { j0[0] = i0 >> 1; j0[1] = (i0 >> 1) + 1; w0[0] = g.ax[0].wl[i0]; w0[1] = g.ax[0].wr[i0]; k0 = 2; }
    else { j0[0] = coarse_idx(i0, g.nf[0]); w0[0] = 1.0; }
    if (n1) { j1[0] = i1 >> 1; j1[1] = (i1 >> 1) + 1; w1[0] = g.ax[1].wl[i1]; w1[1] = g.ax[1].wr[i1]; k1 = 2; }
    else { j1[0] = coarse_idx(i1, g.nf[1]); w1[0] = 1.0; }
    double v;
    if (!(n0 || n1 || n2)) {
      v = Gc[(j0[0] * g.nc[1] + j1[0]) * g.nc[2] + j2[0]];
    } else {
      double interp = 0.0;
      for (int a = 0; a < k0; ++a)
        for (int b = 0; b < k1; ++b) {
          double acc = 0.0;
          for (int c = 0; c < k2; ++c) acc += w2[c] * Gc[(j0[a] * g.nc[1] + j1[b]) * g.nc[2] + j2[c]];
          interp += w0[a] * w1[b] * acc;
        }
      v = interp + coeff_at<RAW>(src, stream_index(g, i0, i1, i2, n0, n1, n2), q);
    }
    out[row * g.nf[2] + i2] = (Tout)v;
  }
}

template <typename Tout, bool RAW>
__global__ __launch_bounds__(256) void k_rec_level0(const CoeffSrc src, int64_t m0, double q,
                                                     Tout* __restrict__ out) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m0; i += stride)
    out[i] = (Tout)coeff_at<RAW>(src, i, q);
}

template <typename Tout>
__global__ __launch_bounds__(256) void k_fill(Tout* __restrict__ out, int64_t N, double v) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += stride)
    out[i] = (Tout)v;
}

inline unsigned grid_for(int64_t n, int block = 256, int64_t cap = 65536) {
  int64_t b = (n + block - 1) / block;
  if (b < 1) b = 1;
  return (unsigned)(b < cap ? b : cap);
}

// Tile shapes per number of active axes (an extent of 1 = inactive axis).
template <typename Tin, bool QUANT>
void dec_dispatch(const void* G, const LevelGeom& g, double* fout, uint16_t* sym, double* raw,
                  double r, const OutlierBuf& ob, unsigned* status, hipStream_t s) {
  const Tin* Gp = static_cast<const Tin*>(G);
  const int D = (g.bit[0] >= 0) + (g.bit[1] >= 0) + (g.bit[2] >= 0);
  auto grid = [&](int tz, int ty, int tx) {
    return dim3((unsigned)((g.nc[2] + tx - 1) / tx), (unsigned)((g.nc[1] + ty - 1) / ty),
                (unsigned)((g.nc[0] + tz - 1) / tz));
  };
  if (D == 3) {
    constexpr int TX = sizeof(Tin) == 4 ? 16 : 8;
    hipLaunchKernelGGL((k_dec_level<Tin, 4, 8, TX, QUANT>), grid(4, 8, TX), dim3(256), 0, s, Gp,
                       g, fout, sym, raw, r, ob, status);
  } else if (D == 2) {
    constexpr int TY = sizeof(Tin) == 4 ? 16 : 8;
    hipLaunchKernelGGL((k_dec_level<Tin, 1, TY, 32, QUANT>), grid(1, TY, 32), dim3(256), 0, s,
                       Gp, g, fout, sym, raw, r, ob, status);
  } else {
    hipLaunchKernelGGL((k_dec_level<Tin, 1, 1, 256, QUANT>), grid(1, 1, 256), dim3(256), 0, s,
                       Gp, g, fout, sym, raw, r, ob, status);
  }
}

template <bool RAW>
void rec_restrict_dispatch(const LevelGeom& g, const CoeffSrc& src, double q, double* fout,
                           hipStream_t s) {
  const int D = (g.bit[0] >= 0) + (g.bit[1] >= 0) + (g.bit[2] >= 0);
  auto grid = [&](int tz, int ty, int tx) {
    return dim3((unsigned)((g.nc[2] + tx - 1) / tx), (unsigned)((g.nc[1] + ty - 1) / ty),
                (unsigned)((g.nc[0] + tz - 1) / tz));
  };
  if (D == 3)
    hipLaunchKernelGGL((k_rec_restrict<4, 8, 8, RAW>), grid(4, 8, 8), dim3(256), 0, s, g, src, q,
                       fout);
  else if (D == 2)
    hipLaunchKernelGGL((k_rec_restrict<1, 8, 32, RAW>), grid(1, 8, 32), dim3(256), 0, s, g, src,
                       q, fout);
  else
    hipLaunchKernelGGL((k_rec_restrict<1, 1, 256, RAW>), grid(1, 1, 256), dim3(256), 0, s, g,
                       src, q, fout);
}

}  // namespace

void launch_range(const void* u, mgc_dtype dt, int64_t N, double* part, double* out,
                  hipStream_t s) {
  if (dt == MGC_F32)
    hipLaunchKernelGGL(k_range_partial<float>, dim3(kRangeBlocks), dim3(256), 0, s,
                       static_cast<const float*>(u), N, part);
  else
    hipLaunchKernelGGL(k_range_partial<double>, dim3(kRangeBlocks), dim3(256), 0, s,
                       static_cast<const double*>(u), N, part);
  hipLaunchKernelGGL(k_range_final, dim3(1), dim3(64), 0, s, part, kRangeBlocks, out);
}

void launch_dec_level(const void* G, bool g_is_f32, const LevelGeom& g, double* fout,
                      uint16_t* sym, double* raw, double r, const OutlierBuf& ob,
                      unsigned* status, hipStream_t s) {
  if (sym) {
    if (g_is_f32) dec_dispatch<float, true>(G, g, fout, sym, raw, r, ob, status, s);
    else dec_dispatch<double, true>(G, g, fout, sym, raw, r, ob, status, s);
  } else {
    if (g_is_f32) dec_dispatch<float, false>(G, g, fout, sym, raw, r, ob, status, s);
    else dec_dispatch<double, false>(G, g, fout, sym, raw, r, ob, status, s);
  }
}

void launch_thomas(int axis, double* x, const int64_t nc[3], const AxisTab& t,
                   const double* sub, hipStream_t s) {
  int64_t lines = axis == 2 ? nc[0] * nc[1] : axis == 1 ? nc[0] * nc[2] : nc[1] * nc[2];
  unsigned blocks = (unsigned)((lines + 255) / 256);
  if (axis == 2)
    hipLaunchKernelGGL(k_thomas<2>, dim3(blocks), dim3(256), 0, s, x, nc[0], nc[1], nc[2], t.ta,
                       t.tm, t.tc, sub);
  else if (axis == 1)
    hipLaunchKernelGGL(k_thomas<1>, dim3(blocks), dim3(256), 0, s, x, nc[0], nc[1], nc[2], t.ta,
                       t.tm, t.tc, sub);
  else
    hipLaunchKernelGGL(k_thomas<0>, dim3(blocks), dim3(256), 0, s, x, nc[0], nc[1], nc[2], t.ta,
                       t.tm, t.tc, sub);
}

void launch_level0(const void* G0, bool g_is_f32, int64_t m0, uint16_t* sym, double* raw,
                   double r, const OutlierBuf& ob, unsigned* status, hipStream_t s) {
  const unsigned b = grid_for(m0);
  if (g_is_f32) {
    if (sym) hipLaunchKernelGGL((k_level0<float, true>), dim3(b), dim3(256), 0, s,
                                static_cast<const float*>(G0), m0, sym, raw, r, ob, status);
    else hipLaunchKernelGGL((k_level0<float, false>), dim3(b), dim3(256), 0, s,
                            static_cast<const float*>(G0), m0, sym, raw, r, ob, status);
  } else {
    if (sym) hipLaunchKernelGGL((k_level0<double, true>), dim3(b), dim3(256), 0, s,
                                static_cast<const double*>(G0), m0, sym, raw, r, ob, status);
    else hipLaunchKernelGGL((k_level0<double, false>), dim3(b), dim3(256), 0, s,
                            static_cast<const double*>(G0), m0, sym, raw, r, ob, status);
  }
}

void launch_rec_restrict(const LevelGeom& g, const CoeffSrc& src, double q, double* fout,
                         hipStream_t s) {
  if (src.raw) rec_restrict_dispatch<true>(g, src, q, fout, s);
  else rec_restrict_dispatch<false>(g, src, q, fout, s);
}

void launch_rec_interp(const double* Gc, const LevelGeom& g, const CoeffSrc& src, double q,
                       void* out, bool out_f32, hipStream_t s) {
  const int64_t rows = g.nf[0] * g.nf[1];
  dim3 grid((unsigned)((g.nf[2] + 255) / 256), (unsigned)(rows < 65535 ? rows : 65535));
  if (out_f32) {
    if (src.raw) hipLaunchKernelGGL((k_rec_interp<float, true>), grid, dim3(256), 0, s, Gc, g, src,
                                    q, static_cast<float*>(out));
    else hipLaunchKernelGGL((k_rec_interp<float, false>), grid, dim3(256), 0, s, Gc, g, src, q,
                            static_cast<float*>(out));
  } else {
    if (src.raw) hipLaunchKernelGGL((k_rec_interp<double, true>), grid, dim3(256), 0, s, Gc, g,
                                    src, q, static_cast<double*>(out));
    else hipLaunchKernelGGL((k_rec_interp<double, false>), grid, dim3(256), 0, s, Gc, g, src, q,
                            static_cast<double*>(out));
  }
}

void launch_rec_level0(const CoeffSrc& src, int64_t m0, double q, void* out, bool out_f32,
                       hipStream_t s) {
  const unsigned b = grid_for(m0);
  if (out_f32) {
    if (src.raw) hipLaunchKernelGGL((k_rec_level0<float, true>), dim3(b), dim3(256), 0, s, src, m0,
                                    q, static_cast<float*>(out));
    else hipLaunchKernelGGL((k_rec_level0<float, false>), dim3(b), dim3(256), 0, s, src, m0, q,
                            static_cast<float*>(out));
  } else {
    if (src.raw) hipLaunchKernelGGL((k_rec_level0<double, true>), dim3(b), dim3(256), 0, s, src,
                                    m0, q, static_cast<double*>(out));
    else hipLaunchKernelGGL((k_rec_level0<double, false>), dim3(b), dim3(256), 0, s, src, m0, q,
                            static_cast<double*>(out));
  }
}

void launch_fill(void* out, bool out_f32, int64_t N, double v, hipStream_t s) {
  if (N <= 0) return;
  const unsigned b = grid_for(N);
  if (out_f32) hipLaunchKernelGGL(k_fill<float>, dim3(b), dim3(256), 0, s, static_cast<float*>(out), N, v);
  else hipLaunchKernelGGL(k_fill<double>, dim3(b), dim3(256), 0, s, static_cast<double*>(out), N, v);
}

}  // namespace mgc
