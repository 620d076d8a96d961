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
#include <type_traits>

namespace mgc {

namespace {

// Linear quantisation of one coefficient: k = rint(c * r) in FP64 (round
// half to even).  |k| < S/2 -> symbol k + S/2; otherwise the escape symbol 0
// and an (position, k) record.  The escaping lanes of a wavefront reserve
// their records with one atomic (the records are sorted by position later,
// so their order here does not matter).
__device__ __forceinline__ void emit_q(int64_t pos, double c, double r, uint16_t* sym,
                                       const OutlierBuf& ob, unsigned* status) {
  const double t = rint(c * r);
  const bool esc = !(fabs(t) < 32768.0);
  sym[pos] = (uint16_t)(int)((esc ? -32768.0 : t) + 32768.0);
  const uint64_t m = __ballot(esc);
  if (m == 0) return;
  if (esc) {
    int64_t k = 0;
    if (fabs(t) < 4611686018427387904.0) k = (int64_t)t;
    else atomicOr(status, ST_RANGE);
    const int lane = (int)__lane_id();
    const int leader = __ffsll((unsigned long long)m) - 1;
    unsigned long long base = 0;
    if (lane == leader) base = atomicAdd(ob.count, (unsigned long long)__popcll(m));
    base = __shfl(base, leader, 64);
    const unsigned long long i = base + (unsigned long long)__popcll(m & ((1ull << lane) - 1));
    if (i < ob.cap) {
      ob.pos[i] = (uint32_t)pos;
      ob.val[i] = k;
    }
  }
}

// Coefficient at stream position pos: raw FP64, or dequantised k * q with
// escaped values found by binary search in the sorted outlier positions.
// w0 a + w1 b as one multiply and one fused multiply-add (every variant of
// the interpolation uses this exact form, so their results agree bit for bit)
__device__ __forceinline__ double lin2(double w0, double a, double w1, double b) {
  return fma(w0, a, w1 * b);
}

// Value of the escaped coefficient at stream position pos (binary search in
// the sorted outlier positions; 0 when there is no record).
__device__ __forceinline__ int64_t escaped_k(const CoeffSrc& s, uint64_t pos) {
  int64_t lo = 0, hi = s.n_out;
  while (lo < hi) {
    int64_t mid = (lo + hi) >> 1;
    if (s.opos[mid] < pos) lo = mid + 1;
    else hi = mid;
  }
  return (lo < s.n_out && s.opos[lo] == pos) ? s.oval[lo] : 0;
}
template <bool RAW>
__device__ __forceinline__ double coeff_at(const CoeffSrc& s, int64_t pos, double q) {
  if (RAW) return s.raw[pos];
  const uint16_t v = s.sym[pos];
  if (v != 0) return (double)((int)v - 32768) * q;
  return (double)escaped_k(s, (uint64_t)pos) * q;
}

// ------------------------------------------------------------ range pass
template <typename T>
__device__ __forceinline__ void range_acc(double v, double& mn, double& mx, double& ss,
                                          double& bad) {
  if (!isfinite(v)) {
    bad = 1.0;
  } else {
    mn = fmin(mn, v);
    mx = fmax(mx, v);
    ss += v * v;
  }
}

// Block `blk` of `nblk` reads 16-byte vectors in a grid-stride loop (the
// tail, fewer than one vector per thread of the grid, element by element) and
// writes its (min, max, sum of squares, non-finite flag) to part4.
template <typename T, bool VEC>
__device__ __forceinline__ void range_partial_body(const T* __restrict__ u, int64_t N,
                                                   double* __restrict__ part4, uint32_t blk,
                                                   uint32_t nblk) {
  constexpr int V = VEC ? 16 / sizeof(T) : 1;
  using Vec = typename std::conditional<sizeof(T) == 4, float4, double2>::type;
  double mn = INFINITY, mx = -INFINITY, ss = 0.0, bad = 0.0;
  const int64_t stride = (int64_t)nblk * 256;
  const int64_t nvec = VEC ? N / V : 0;
  const Vec* uv = reinterpret_cast<const Vec*>(u);
  auto acc = [&](const Vec& w) {
    if constexpr (sizeof(T) == 4) {
      range_acc<T>(w.x, mn, mx, ss, bad);
      range_acc<T>(w.y, mn, mx, ss, bad);
      range_acc<T>(w.z, mn, mx, ss, bad);
      range_acc<T>(w.w, mn, mx, ss, bad);
    } else {
      range_acc<T>(w.x, mn, mx, ss, bad);
      range_acc<T>(w.y, mn, mx, ss, bad);
    }
  };
  // four vectors per thread in flight, then the remainder one at a time
  int64_t i = (int64_t)blk * 256 + threadIdx.x;
  for (; i + 3 * stride < nvec; i += 4 * stride) {
    Vec w[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) w[k] = uv[i + k * stride];
#pragma unroll
    for (int k = 0; k < 4; ++k) acc(w[k]);
  }
  for (; i < nvec; i += stride) acc(uv[i]);
  for (int64_t i = nvec * V + (int64_t)blk * 256 + threadIdx.x; i < N; i += stride)
    range_acc<T>((double)u[i], mn, mx, ss, bad);
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
    for (int k = 0; k < 4; ++k) part4[k] = sm[0][k];
  }
}

template <typename T, bool VEC>
__global__ __launch_bounds__(256) void k_range_partial(const T* __restrict__ u, int64_t N,
                                                        double* __restrict__ part) {
  range_partial_body<T, VEC>(u, N, part + 4 * blockIdx.x, blockIdx.x, gridDim.x);
}

// Reduces the per-block partials in a fixed tree order (deterministic) into
// out[0..3]; thread 0 also receives them in r4.
__device__ __forceinline__ void range_final_body(const double* __restrict__ part, int nb,
                                                 double* __restrict__ out, double* r4) {
  __shared__ double sm[4][256];
  const int t = threadIdx.x;
  double mn = INFINITY, mx = -INFINITY, ss = 0.0, bad = 0.0;
  for (int b = t; b < nb; b += 256) {
    mn = fmin(mn, part[4 * b + 0]);
    mx = fmax(mx, part[4 * b + 1]);
    ss += part[4 * b + 2];
    bad = fmax(bad, part[4 * b + 3]);
  }
  sm[0][t] = mn;
  sm[1][t] = mx;
  sm[2][t] = ss;
  sm[3][t] = bad;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) {
      sm[0][t] = fmin(sm[0][t], sm[0][t + w]);
      sm[1][t] = fmax(sm[1][t], sm[1][t + w]);
      sm[2][t] += sm[2][t + w];
      sm[3][t] = fmax(sm[3][t], sm[3][t + w]);
    }
    __syncthreads();
  }
  if (t < 4) out[t] = sm[t][0];
  if (t == 0)
    for (int k = 0; k < 4; ++k) r4[k] = sm[k][0];
}

// Error budget of the quantiser from the data range (thread 0): the absolute
// bound tau (relative bounds scale by max - min for L-inf, by ||u||_2 for
// L2), the budget tau' left after the rounding of the output type, and the
// per-level bins q_l = tau' K_l with their reciprocals.  Sets ST_NONFINITE,
// ST_CONST or ST_BUDGET (tau' not positive) instead when they apply.
__device__ __forceinline__ void budget_from_range(const BudgetIn& b, const double* r4,
                                                  double* __restrict__ bud,
                                                  unsigned* __restrict__ status) {
  const double mn = r4[0], mx = r4[1], ss = r4[2], bad = r4[3];
  if (bad != 0.0) {
    atomicOr(status, ST_NONFINITE);
    return;
  }
  if (mn == mx) {
    atomicOr(status, ST_CONST);
    return;
  }
  const double eps = b.dtype == MGC_F32 ? 0x1p-24 : 0x1p-53;
  const double margin = 0x1p-36;
  const double amax = fmax(fabs(mx), fabs(mn));
  double t, A;
  if (b.norm == MGC_LINF) {
    t = b.mode == MGC_REL ? b.bound * (mx - mn) : b.bound;
    A = amax;
  } else {
    t = b.mode == MGC_REL ? b.bound * sqrt(ss) : b.bound;
    A = sqrt((double)b.N) * amax;
  }
  const double te = t - (eps + margin) * (A + t);
  bud[4] = t;
  bud[5] = te;
  if (!(te > 0.0)) {
    atomicOr(status, ST_BUDGET);
    return;
  }
  for (int l = 0; l <= b.L; ++l) {
    const double q = te * b.K[l];
    bud[6 + l] = q;
    bud[6 + b.L + 1 + l] = 1.0 / q;
  }
}

__global__ __launch_bounds__(256) void k_budget(const double* __restrict__ part, int nb,
                                                 const BudgetIn b, double* __restrict__ bud,
                                                 unsigned* __restrict__ status) {
  double r4[4];
  range_final_body(part, nb, bud, r4);
  if (threadIdx.x == 0) budget_from_range(b, r4, bud, status);
}

// ------------------------------------------------------------- tile helpers
// Coarse output tile TZ x TY x TX; an extent of 1 marks an inactive axis.
template <int T>
struct Ext {
  static constexpr int v = T == 1 ? 1 : 2 * T + 3;
};

__device__ __forceinline__ uint32_t cpos32(uint32_t j, uint32_t nf) {
  const uint32_t p = 2 * j;
  return p < nf ? p : nf - 1;
}
__device__ __forceinline__ bool is_new32(uint32_t i, uint32_t nf) {
  return (i & 1u) && i != nf - 1;
}
__device__ __forceinline__ uint32_t cidx32(uint32_t i, uint32_t nf) {
  return (i == nf - 1 && !(nf & 1u)) ? (nf >> 1) : (i >> 1);
}
// floor(r / d) for r < 2^16 with m = ceil(2^32 / d) (2^32 itself for d = 1)
__device__ __forceinline__ uint32_t div_small(uint32_t r, uint64_t m) {
  return (uint32_t)(((uint64_t)r * m) >> 32);
}
// ceil(2^32 / d) for d >= 1 (floor((2^32 - 1 + d) / d) = floor((2^32 - 1) / d) + 1):
// a 32-bit division instead of a 64-bit one, which costs about a hundred
// scalar instructions per call
__device__ __forceinline__ uint64_t div_magic(uint32_t d) { return (uint64_t)(0xFFFFFFFFu / d) + 1; }

// Workgroups are dispatched round-robin over the 8 XCDs; giving each XCD a
// contiguous range of tiles keeps neighbouring tiles (which share halos) in
// the same L2.  grid = n_tiles rounded up to a multiple of 8.
// Orders a wavefront's LDS accesses (its lanes exchange values through LDS).
__device__ __forceinline__ void wave_fence() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ uint32_t xcd_tile(uint32_t b, uint32_t grid) {
  return (b & 7u) * (grid >> 3) + (b >> 3);
}

// Geometry of one tile of level l, uniform over the block.
struct Tile {
  uint32_t nf[3], nc[3];
  uint32_t c0[3];   // first coarse index per axis
  int tk[3];        // coarse outputs per axis
  uint32_t lo[3];   // first fine index loaded (halo of two nodes)
  int ext[3];       // fine nodes loaded
  int olo[3];       // first owned fine node, relative to lo
  int oext[3];      // owned fine nodes
};

template <int TZ, int TY, int TX>
__device__ __forceinline__ bool make_tile(const LevelGeom& g, uint32_t t, uint32_t tiles_x,
                                          uint32_t tiles_y, Tile& tl) {
  const uint32_t tx = t % tiles_x, rest = t / tiles_x;
  const uint32_t ty = rest % tiles_y, tz = rest / tiles_y;
  const uint32_t cc[3] = {tz * TZ, ty * TY, tx * TX};
  const int T[3] = {TZ, TY, TX};
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const uint32_t nf = (uint32_t)g.nf[k], nc = (uint32_t)g.nc[k];
    tl.nf[k] = nf;
    tl.nc[k] = nc;
    tl.c0[k] = cc[k];
    if (cc[k] >= nc) return false;
    tl.tk[k] = (int)min<uint32_t>(T[k], nc - cc[k]);
    const uint32_t p0 = cpos32(cc[k], nf);
    tl.lo[k] = p0 >= 2 ? p0 - 2 : 0;
    const uint32_t hi = min<uint32_t>(cpos32(cc[k] + tl.tk[k] - 1, nf) + 2, nf - 1);
    tl.ext[k] = (int)(hi - tl.lo[k] + 1);
    const uint32_t olo = 2 * cc[k];
    const uint32_t ohi = (cc[k] + tl.tk[k] >= nc) ? nf : 2 * (cc[k] + tl.tk[k]);
    tl.olo[k] = (int)(olo - tl.lo[k]);
    tl.oext[k] = ohi > olo ? (int)(ohi - olo) : 0;
  }
  return true;
}

// Per-tile operator tables in LDS: interpolation weights of the loaded fine
// nodes, restriction taps of the tile's coarse outputs and the tile-relative
// position of each output's centre tap; subband offsets of the level.
template <int E0, int E1, int E2, int TZ, int TY, int TX>
struct TileTabs {
  // doubles: wl0[E0] wr0[E0] wl1[E1] wr1[E1] wl2[E2] wr2[E2] W0[TZ][5] W1[TY][5] W2[TX][5]
  static constexpr int O_WL0 = 0, O_WR0 = E0, O_WL1 = 2 * E0, O_WR1 = 2 * E0 + E1,
                       O_WL2 = 2 * (E0 + E1), O_WR2 = 2 * (E0 + E1) + E2,
                       O_W0 = 2 * (E0 + E1 + E2), O_W1 = O_W0 + 5 * TZ, O_W2 = O_W1 + 5 * TY,
                       ND = O_W2 + 5 * TX;
  double d[ND];
  int P0[TZ], P1[TY], P2[TX];
  uint32_t soff[8];
  __device__ double wl0(int i) const { return d[O_WL0 + i]; }
  __device__ double wr0(int i) const { return d[O_WR0 + i]; }
  __device__ double wl1(int i) const { return d[O_WL1 + i]; }
  __device__ double wr1(int i) const { return d[O_WR1 + i]; }
  __device__ double wl2(int i) const { return d[O_WL2 + i]; }
  __device__ double wr2(int i) const { return d[O_WR2 + i]; }
  __device__ double W0(int j, int t) const { return d[O_W0 + 5 * j + t]; }
  __device__ double W1(int j, int t) const { return d[O_W1 + 5 * j + t]; }
  __device__ double W2(int j, int t) const { return d[O_W2 + 5 * j + t]; }
};

// The tables are fetched as one flattened list (interpolation weights of
// the loaded nodes when need_w, then the restriction taps of the outputs),
// every load of a thread issued before any is used, so a tile pays one
// memory latency for them.  (A loop of load-then-store would wait once per
// table.)  The taps are those of P^T instead of P^T M when transpose_p.
template <int E0, int E1, int E2, int TZ, int TY, int TX>
__device__ void load_tabs(const LevelGeom& g, const Tile& tl, TileTabs<E0, E1, E2, TZ, TY, TX>& tb,
                          bool need_w, bool transpose_p = false) {
  constexpr int MAXN = 2 * (E0 + E1 + E2) + 5 * (TZ + TY + TX);
  constexpr int NT = (MAXN + 255) / 256;
  const int tid = threadIdx.x;
  const int n0 = tl.ext[0], n1 = tl.ext[1], n2 = tl.ext[2];
  // segment sizes, sources and destinations (offsets in the doubles of tb)
  const int sz[9] = {need_w ? n0 : 0, need_w ? n0 : 0, need_w ? n1 : 0, need_w ? n1 : 0,
                     need_w ? n2 : 0, need_w ? n2 : 0, 5 * tl.tk[0], 5 * tl.tk[1], 5 * tl.tk[2]};
  const double* src[9] = {g.ax[0].wl + tl.lo[0], g.ax[0].wr + tl.lo[0], g.ax[1].wl + tl.lo[1],
                          g.ax[1].wr + tl.lo[1], g.ax[2].wl + tl.lo[2], g.ax[2].wr + tl.lo[2],
                          (transpose_p ? g.ax[0].WP : g.ax[0].W) + 5 * tl.c0[0],
                          (transpose_p ? g.ax[1].WP : g.ax[1].W) + 5 * tl.c0[1],
                          (transpose_p ? g.ax[2].WP : g.ax[2].W) + 5 * tl.c0[2]};
  using TT = TileTabs<E0, E1, E2, TZ, TY, TX>;
  constexpr int dof[9] = {TT::O_WL0, TT::O_WR0, TT::O_WL1, TT::O_WR1, TT::O_WL2,
                          TT::O_WR2, TT::O_W0, TT::O_W1, TT::O_W2};
  double v[NT];
  int dst[NT];
#pragma unroll
  for (int u = 0; u < NT; ++u) {
    int i = tid + 256 * u;
    dst[u] = -1;
    const double* sp = src[8];  // a valid address for threads with no entry
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      if (dst[u] < 0 && i < sz[k]) {
        dst[u] = dof[k] + i;
        sp = src[k] + i;
      }
      if (dst[u] < 0) i -= sz[k];
    }
    v[u] = *sp;
  }
#pragma unroll
  for (int u = 0; u < NT; ++u)
    if (dst[u] >= 0) tb.d[dst[u]] = v[u];
  for (int i = tid; i < tl.tk[0]; i += 256) tb.P0[i] = (int)(cpos32(tl.c0[0] + i, tl.nf[0]) - tl.lo[0]);
  for (int i = tid; i < tl.tk[1]; i += 256) tb.P1[i] = (int)(cpos32(tl.c0[1] + i, tl.nf[1]) - tl.lo[1]);
  for (int i = tid; i < tl.tk[2]; i += 256) tb.P2[i] = (int)(cpos32(tl.c0[2] + i, tl.nf[2]) - tl.lo[2]);
  if (tid < 8) tb.soff[tid] = (uint32_t)(tid == 0 ? 0 : g.sub_off[tid]);
}

// Stream position of a fine node with new-node flags n0..n2 (32-bit: N < 2^32).
__device__ __forceinline__ uint32_t stream_pos(const LevelGeom& g, const Tile& tl,
                                               const uint32_t* soff, uint32_t i0, uint32_t i1,
                                               uint32_t i2, bool n0, bool n1, bool n2) {
  const int m = (n0 ? (1 << g.bit[0]) : 0) | (n1 ? (1 << g.bit[1]) : 0) | (n2 ? (1 << g.bit[2]) : 0);
  const uint32_t e1 = n1 ? tl.nf[1] - tl.nc[1] : tl.nc[1];
  const uint32_t e2 = n2 ? tl.nf[2] - tl.nc[2] : tl.nc[2];
  const uint32_t j0 = n0 ? (i0 >> 1) : cidx32(i0, tl.nf[0]);
  const uint32_t j1 = n1 ? (i1 >> 1) : cidx32(i1, tl.nf[1]);
  const uint32_t j2 = n2 ? (i2 >> 1) : cidx32(i2, tl.nf[2]);
  return (uint32_t)g.level_off + soff[m] + (j0 * e1 + j1) * e2 + j2;
}

// Offset of subband m from eight uniform values (no indexing of a register
// array, which would go through scratch memory).
__device__ __forceinline__ uint32_t sel8(const uint32_t (&so)[8], int m) {
  const uint32_t a = (m & 1) ? so[1] : so[0], b = (m & 1) ? so[3] : so[2];
  const uint32_t c = (m & 1) ? so[5] : so[4], d = (m & 1) ? so[7] : so[6];
  const uint32_t ab = (m & 2) ? b : a, cd = (m & 2) ? d : c;
  return (m & 4) ? cd : ab;
}

// stream_pos with the subband offsets held in registers (no LDS table).
__device__ __forceinline__ uint32_t stream_pos_r(const LevelGeom& g, const Tile& tl,
                                                 const uint32_t (&so)[8], uint32_t i0,
                                                 uint32_t i1, uint32_t i2, bool n0, bool n1,
                                                 bool n2) {
  const int m = (n0 ? (1 << g.bit[0]) : 0) | (n1 ? (1 << g.bit[1]) : 0) | (n2 ? (1 << g.bit[2]) : 0);
  const uint32_t e1 = n1 ? tl.nf[1] - tl.nc[1] : tl.nc[1];
  const uint32_t e2 = n2 ? tl.nf[2] - tl.nc[2] : tl.nc[2];
  const uint32_t j0 = n0 ? (i0 >> 1) : cidx32(i0, tl.nf[0]);
  const uint32_t j1 = n1 ? (i1 >> 1) : cidx32(i1, tl.nf[1]);
  const uint32_t j2 = n2 ? (i2 >> 1) : cidx32(i2, tl.nf[2]);
  return (uint32_t)g.level_off + sel8(so, m) + (j0 * e1 + j1) * e2 + j2;
}

__device__ __forceinline__ void subband_offsets(const LevelGeom& g, uint32_t (&so)[8]) {
  so[0] = 0;
#pragma unroll
  for (int m = 1; m < 8; ++m) so[m] = (uint32_t)g.sub_off[m];
}

// Dequantised coefficient from an already loaded symbol v at stream position
// pos (escaped values: binary search in the sorted outlier positions).
// k q_l for symbol v (k = v - 32768 converts exactly through 32 bits).
__device__ __forceinline__ double dequant(const CoeffSrc& s, uint32_t v, uint32_t pos, double q) {
  if (v != 0) return (double)((int)v - 32768) * q;
  return (double)escaped_k(s, pos) * q;
}

// The separable restriction (P^T M_l along x, then y, then z) of a fine tile
// held in LDS (element type V, row pitch E2, plane pitch E1*E2) to the tile's
// coarse outputs, written to fout (coarse grid).  A and B are LDS scratch.
//
// A tap that falls outside the loaded region lies outside the grid, where the
// operator's weight is exactly zero; such taps read the nearest loaded node
// (clamped index) instead of being skipped, which adds a signed zero and
// leaves every sum unchanged.  Each thread keeps one output column (x) or one
// (y, x) pair for all its rows, so the taps' positions and weights are read
// from LDS once per thread.
template <typename V, int E0, int E1, int E2, int TZ, int TY, int TX>
__device__ void restrict_tile(const V* tile, double* A, double* B, const Tile& tl,
                              const TileTabs<E0, E1, E2, TZ, TY, TX>& tb, double* __restrict__ fout,
                              double* __restrict__ fout2 = nullptr) {
  const int tid = threadIdx.x;
  constexpr int CW = TX < 64 ? TX : 64;        // lanes per output row
  constexpr int RS = 256 / CW;                  // rows per block step
  const int col0 = tid % CW, rsub = tid / CW;
  // x: A[z][y][cx], rows (z, y)
  {
    const int rows = tl.ext[0] * tl.ext[1];
    const uint64_t m1 = div_magic((uint32_t)tl.ext[1]);
    const int last = tl.ext[2] - 1;
    for (int cx = col0; cx < tl.tk[2]; cx += CW) {
      const int p = tb.P2[cx];
      int f[5];
      double w[5];
#pragma unroll
      for (int d = 0; d < 5; ++d) {
        f[d] = min(max(p + d - 2, 0), last);
        w[d] = tb.W2(cx, d);
      }
      for (int rw = rsub; rw < rows; rw += RS) {
        const int z = (int)div_small((uint32_t)rw, m1), y = rw - z * tl.ext[1];
        const V* row = tile + (z * E1 + y) * E2;
        double acc = 0.0;
#pragma unroll
        for (int d = 0; d < 5; ++d) acc = fma(w[d], (double)row[f[d]], acc);
        A[(z * E1 + y) * TX + cx] = acc;
      }
    }
  }
  __syncthreads();
  constexpr int PAIRS = TY * TX;
  constexpr bool FIXED = PAIRS <= 256 && 256 % PAIRS == 0;
  // y: B[z][cy][cx]
  if constexpr (FIXED) {
    constexpr int G = 256 / PAIRS;   // threads sharing a (cy, cx) pair, over z
    const int pair = tid % PAIRS, z0 = tid / PAIRS;
    const int cy = pair / TX, cx = pair % TX;
    if (cy < tl.tk[1] && cx < tl.tk[2]) {
      const int p = tb.P1[cy], last = tl.ext[1] - 1;
      int f[5];
      double w[5];
#pragma unroll
      for (int d = 0; d < 5; ++d) {
        f[d] = min(max(p + d - 2, 0), last);
        w[d] = tb.W1(cy, d);
      }
      for (int z = z0; z < tl.ext[0]; z += G) {
        const double* col = A + z * E1 * TX + cx;
        double acc = 0.0;
#pragma unroll
        for (int d = 0; d < 5; ++d) acc = fma(w[d], col[f[d] * TX], acc);
        B[(z * TY + cy) * TX + cx] = acc;
      }
    }
  } else {
    const int rows = tl.ext[0] * tl.tk[1];
    const uint64_t m1 = div_magic((uint32_t)tl.tk[1]);
    const int last = tl.ext[1] - 1;
    for (int rw = rsub; rw < rows; rw += RS) {
      const int z = (int)div_small((uint32_t)rw, m1), cy = rw - z * tl.tk[1];
      const int p = tb.P1[cy];
      for (int cx = col0; cx < tl.tk[2]; cx += CW) {
        double acc = 0.0;
#pragma unroll
        for (int d = 0; d < 5; ++d)
          acc = fma(tb.W1(cy, d), A[(z * E1 + min(max(p + d - 2, 0), last)) * TX + cx], acc);
        B[(z * TY + cy) * TX + cx] = acc;
      }
    }
  }
  __syncthreads();
  // z: coarse outputs (cz, cy, cx)
  {
    const int last = tl.ext[0] - 1;
    if constexpr (FIXED) {
      constexpr int G = 256 / PAIRS;
      const int pair = tid % PAIRS, c0 = tid / PAIRS;
      const int cy = pair / TX, cx = pair % TX;
      if (cy < tl.tk[1] && cx < tl.tk[2]) {
        for (int cz = c0; cz < tl.tk[0]; cz += G) {
          const int p = tb.P0[cz];
          double acc = 0.0;
#pragma unroll
          for (int d = 0; d < 5; ++d)
            acc = fma(tb.W0(cz, d), B[(min(max(p + d - 2, 0), last) * TY + cy) * TX + cx], acc);
          const size_t o = ((size_t)(tl.c0[0] + cz) * tl.nc[1] + tl.c0[1] + cy) * tl.nc[2] +
                           tl.c0[2] + cx;
          fout[o] = acc;
          if (fout2) fout2[o] = acc;
        }
      }
    } else {
      const int rows = tl.tk[0] * tl.tk[1];
      const uint64_t m1 = div_magic((uint32_t)tl.tk[1]);
      for (int rw = rsub; rw < rows; rw += RS) {
        const int cz = (int)div_small((uint32_t)rw, m1), cy = rw - cz * tl.tk[1];
        const int p = tb.P0[cz];
        const size_t ro = ((size_t)(tl.c0[0] + cz) * tl.nc[1] + tl.c0[1] + cy) * tl.nc[2] + tl.c0[2];
        for (int cx = col0; cx < tl.tk[2]; cx += CW) {
          double acc = 0.0;
#pragma unroll
          for (int d = 0; d < 5; ++d)
            acc = fma(tb.W0(cz, d), B[(min(max(p + d - 2, 0), last) * TY + cy) * TX + cx], acc);
          fout[ro + cx] = acc;
          if (fout2) fout2[ro + cx] = acc;
        }
      }
    }
  }
}

// ------------------------------------------------------- lerp by cells
// Cell J (coarse indices J0, J1, J2) owns the fine nodes at cpos(J) and, on
// each axis where 2J+1 is a new node, 2J+1: up to seven new nodes, whose
// coefficients are the value minus the multilinear interpolant from the
// cell's corners cpos(J) and cpos(J+1) = 2J+2 (the coarse nodes around
// them).  The interpolant nests the axes as x innermost, then y, then z;
// along an axis where the node is not new the weights would be (1, 0), which
// reproduces the same value, so those factors are simply left out.  The
// seven stream positions share (J0*e1 + J1)*e2 + J2 with per-subband extents,
// and consecutive threads take consecutive cells along x, so each subband's
// stores are contiguous.
template <typename Tin, int TZ, int TY, int TX, int E1, int E2, bool QUANT, typename TT>
__device__ __forceinline__ void lerp_cells(const Tin* tile, const Tile& tl, const TT& tb,
                                           const LevelGeom& g, uint16_t* __restrict__ sym,
                                           double* __restrict__ raw, double r,
                                           const OutlierBuf& ob, unsigned* __restrict__ status) {
  constexpr int NC = TZ * TY * TX;
  const uint32_t e1c = tl.nc[1], e1n = tl.nf[1] - tl.nc[1];
  const uint32_t e2c = tl.nc[2], e2n = tl.nf[2] - tl.nc[2];
  const uint32_t lvl = (uint32_t)g.level_off;
  const int m0 = g.bit[0] >= 0 ? 1 << g.bit[0] : 0, m1 = g.bit[1] >= 0 ? 1 << g.bit[1] : 0,
            m2 = g.bit[2] >= 0 ? 1 << g.bit[2] : 0;
  auto T = [&](int z, int y, int x) -> double { return (double)tile[(z * E1 + y) * E2 + x]; };
  auto emit = [&](uint32_t pos, double v) {
    if (QUANT) emit_q(pos, v, r, sym, ob, status);
    else raw[pos] = v;
  };
  for (int e = threadIdx.x; e < NC; e += 256) {
    const int cx = e % TX, rest = e / TX, cy = rest % TY, cz = rest / TY;
    if (cz >= tl.tk[0] || cy >= tl.tk[1] || cx >= tl.tk[2]) continue;
    const uint32_t J0 = tl.c0[0] + cz, J1 = tl.c0[1] + cy, J2 = tl.c0[2] + cx;
    const bool h0 = 2 * J0 + 1 < tl.nf[0] - 1, h1 = 2 * J1 + 1 < tl.nf[1] - 1,
               h2 = 2 * J2 + 1 < tl.nf[2] - 1;
    if (!(h0 || h1 || h2)) continue;
    // tile-relative fine positions: cell origin p, new node p+1, next corner
    const int p0 = (int)(cpos32(J0, tl.nf[0]) - tl.lo[0]);
    const int p1 = (int)(cpos32(J1, tl.nf[1]) - tl.lo[1]);
    const int p2 = (int)(cpos32(J2, tl.nf[2]) - tl.lo[2]);
    const int s0 = h0 ? p0 + 2 : p0, s1 = h1 ? p1 + 2 : p1, s2 = h2 ? p2 + 2 : p2;
    const int q0 = h0 ? p0 + 1 : p0, q1 = h1 ? p1 + 1 : p1, q2 = h2 ? p2 + 1 : p2;
    const double wz0 = tb.wl0(q0), wz1 = tb.wr0(q0);
    const double wy0 = tb.wl1(q1), wy1 = tb.wr1(q1);
    const double wx0 = tb.wl2(q2), wx1 = tb.wr2(q2);
    const double c000 = T(p0, p1, p2), c001 = T(p0, p1, s2), c010 = T(p0, s1, p2),
                 c011 = T(p0, s1, s2), c100 = T(s0, p1, p2), c101 = T(s0, p1, s2),
                 c110 = T(s0, s1, p2), c111 = T(s0, s1, s2);
    const double ix00 = lin2(wx0, c000, wx1, c001), ix01 = lin2(wx0, c010, wx1, c011);
    const double ix10 = lin2(wx0, c100, wx1, c101), ix11 = lin2(wx0, c110, wx1, c111);
    const uint32_t base_cc = (J0 * e1c + J1) * e2c + J2, base_cn = (J0 * e1c + J1) * e2n + J2;
    const uint32_t base_nc = (J0 * e1n + J1) * e2c + J2, base_nn = (J0 * e1n + J1) * e2n + J2;
    if (h2) emit(lvl + tb.soff[m2] + base_cn, T(p0, p1, q2) - ix00);
    if (h1) emit(lvl + tb.soff[m1] + base_nc, T(p0, q1, p2) - (lin2(wy0, c000, wy1, c010)));
    if (h1 && h2)
      emit(lvl + tb.soff[m1 | m2] + base_nn, T(p0, q1, q2) - (lin2(wy0, ix00, wy1, ix01)));
    if (h0) emit(lvl + tb.soff[m0] + base_cc, T(q0, p1, p2) - (lin2(wz0, c000, wz1, c100)));
    if (h0 && h2)
      emit(lvl + tb.soff[m0 | m2] + base_cn, T(q0, p1, q2) - (lin2(wz0, ix00, wz1, ix10)));
    if (h0 && h1)
      emit(lvl + tb.soff[m0 | m1] + base_nc,
           T(q0, q1, p2) - (lin2(wz0, lin2(wy0, c000, wy1, c010), wz1, lin2(wy0, c100, wy1, c110))));
    if (h0 && h1 && h2)
      emit(lvl + tb.soff[m0 | m1 | m2] + base_nn,
           T(q0, q1, q2) - (lin2(wz0, lin2(wy0, ix00, wy1, ix01), wz1, lin2(wy0, ix10, wy1, ix11))));
  }
}

// ----------------------------------------------- decomposition of one level
// MODE: 0 quantise the coefficients, 1 write them as FP64, 2 adjoint (no
// coefficients; restriction with the P^T taps written to fout and fout2).
// Tile t (row-major over the level's coarse grid in tiles of TZ x TY x TX).
template <typename Tin, int TZ, int TY, int TX, int MODE>
__device__ __forceinline__ void dec_level_body(const Tin* __restrict__ G, const LevelGeom& g,
                                               double* __restrict__ fout,
                                               uint16_t* __restrict__ sym,
                                               double* __restrict__ raw, const double r,
                                               const OutlierBuf& ob,
                                               unsigned* __restrict__ status, uint32_t t) {
  constexpr int E0 = Ext<TZ>::v, E1 = Ext<TY>::v, E2 = Ext<TX>::v;
  constexpr int TILE_BYTES = E0 * E1 * E2 * (int)sizeof(Tin);
  static_assert(E0 * TY * TX * (int)sizeof(double) <= TILE_BYTES, "B aliases the tile");
  __shared__ __align__(16) unsigned char smem[TILE_BYTES];
  __shared__ double A[E0 * E1 * TX];
  __shared__ TileTabs<E0, E1, E2, TZ, TY, TX> tb;
  Tin* tile = reinterpret_cast<Tin*>(smem);

  const uint32_t tiles_x = (uint32_t)((g.nc[2] + TX - 1) / TX);
  const uint32_t tiles_y = (uint32_t)((g.nc[1] + TY - 1) / TY);
  Tile tl;
  if (!make_tile<TZ, TY, TX>(g, t, tiles_x, tiles_y, tl)) return;
  const int tid = threadIdx.x;
  // load the fine tile: flattened over the block, every load of a thread in
  // flight (with the operator tables' loads behind them) before the first
  // LDS store; offsets are 32-bit (arrays hold fewer than 2^32 values)
  {
    constexpr int NLD = (E0 * E1 * E2 + 255) / 256;
    const int e12 = tl.ext[1] * tl.ext[2], n_ld = tl.ext[0] * e12;
    const uint64_t m12 = div_magic((uint32_t)e12), m2 = div_magic((uint32_t)tl.ext[2]);
    const Tin* base = G + ((size_t)tl.lo[0] * tl.nf[1] + tl.lo[1]) * tl.nf[2] + tl.lo[2];
    const uint32_t pz = tl.nf[1] * tl.nf[2], py = tl.nf[2];
    Tin v[NLD];
    int dst[NLD];
#pragma unroll
    for (int u = 0; u < NLD; ++u) {
      const int e = min(u * 256 + tid, n_ld - 1);
      const int z = (int)div_small((uint32_t)e, m12), r = e - z * e12;
      const int y = (int)div_small((uint32_t)r, m2), x = r - y * tl.ext[2];
      v[u] = base[(uint32_t)z * pz + (uint32_t)y * py + (uint32_t)x];
      dst[u] = u * 256 + tid < n_ld ? (z * E1 + y) * E2 + x : -1;
    }
    load_tabs(g, tl, tb, MODE != 2, MODE == 2);
#pragma unroll
    for (int u = 0; u < NLD; ++u)
      if (dst[u] >= 0) tile[dst[u]] = v[u];
  }
  __syncthreads();

  // lerp + quantise the owned new nodes, one coarse cell (the 2x2x2 fine
  // nodes a coarse node owns) at a time
  if (MODE != 2) lerp_cells<Tin, TZ, TY, TX, E1, E2, MODE == 0>(tile, tl, tb, g, sym, raw, r, ob, status);
  // mass_trans (or P^T for the adjoint): separable restriction to the coarse outputs
  restrict_tile(tile, A, reinterpret_cast<double*>(smem), tl, tb, fout, MODE == 2 ? raw : nullptr);
}

template <typename Tin, int TZ, int TY, int TX, int MODE>
__global__ __launch_bounds__(256) void k_dec_level(const Tin* __restrict__ G, const LevelGeom g,
                                                    double* __restrict__ fout,
                                                    uint16_t* __restrict__ sym,
                                                    double* __restrict__ raw,
                                                    const double* __restrict__ rp,
                                                    const OutlierBuf ob,
                                                    unsigned* __restrict__ status,
                                                    const unsigned* __restrict__ gate,
                                                    const uint32_t n_tiles) {
  const uint32_t t = xcd_tile(blockIdx.x, gridDim.x);
  if (t >= n_tiles || gate_closed(gate)) return;
  const double r = rp ? *rp : 0.0;
  dec_level_body<Tin, TZ, TY, TX, MODE>(G, g, fout, sym, raw, r, ob, status, t);
}

// ------------------------------- decomposition of a 3-axis level, streamed
// A block owns a column of SY x SX coarse outputs (fine region with a
// two-node halo in y and x) and walks a segment of coarse z planes.  Each
// fine plane is loaded once (the next plane's loads in flight while the
// current one is processed), restricted along x and then y; the y results of
// the last five fine planes and the raw values of the last three stay in
// LDS rings.  When the five planes around a coarse plane are in, its outputs
// are restricted along z and its cells are interpolated and quantised.  The
// sums are formed in the same order as in the tiled kernel (x, y, z; taps in
// order), so the results are the same; the z halo is paid once per segment
// instead of once per tile.
constexpr int kStreamSY = 8, kStreamSX = 32;
constexpr int kStreamE1 = 2 * kStreamSY + 3, kStreamE2 = 2 * kStreamSX + 3;
constexpr int kStreamNLD = (kStreamE1 * kStreamE2 + 255) / 256;
constexpr int kStreamPF = 2;     // fine planes whose loads are in flight (recomposition)
constexpr int kDecStreamPF = 1;  // (decomposition: registers go to the cells)
// levels with fewer fine points use the tiled kernel (measured faster there)
constexpr int64_t kStreamMinPoints = int64_t(1) << 25;
// Recomposition's restriction (one value per coarse node from the dequantised
// new nodes) gains from streaming already at half that size.
constexpr int64_t kRecStreamMinPoints = int64_t(1) << 24;

template <typename Tin>
struct StreamSmem {
  Tin raw[3][kStreamE1][kStreamE2];
  double X[kStreamE1][kStreamSX];
  double Y[5][kStreamSY][kStreamSX];
  double wl1[kStreamE1], wr1[kStreamE1], wl2[kStreamE2], wr2[kStreamE2];
  double W1[kStreamSY][5], W2[kStreamSX][5];
  int P1[kStreamSY], P2[kStreamSX];
};

template <typename Tin, bool QUANT>
__global__ __launch_bounds__(256, 4) void k_dec_stream(const Tin* __restrict__ G, const LevelGeom g,
                                                     double* __restrict__ fout,
                                                     uint16_t* __restrict__ sym,
                                                     double* __restrict__ raw,
                                                     const double* __restrict__ rp,
                                                     const OutlierBuf ob,
                                                     unsigned* __restrict__ status,
                                                     const unsigned* __restrict__ gate,
                                                     const int seg, const uint32_t n_blocks) {
  constexpr int SY = kStreamSY, SX = kStreamSX, E2 = kStreamE2;
  __shared__ StreamSmem<Tin> sm;
  const uint32_t b = xcd_tile(blockIdx.x, gridDim.x);
  if (b >= n_blocks || gate_closed(gate)) return;
  const double r = rp ? *rp : 0.0;
  const uint32_t nf0 = (uint32_t)g.nf[0], nf1 = (uint32_t)g.nf[1], nf2 = (uint32_t)g.nf[2];
  const uint32_t nc0 = (uint32_t)g.nc[0], nc1 = (uint32_t)g.nc[1], nc2 = (uint32_t)g.nc[2];
  const uint32_t tiles_x = (nc2 + SX - 1) / SX, tiles_y = (nc1 + SY - 1) / SY;
  const uint32_t tx = b % tiles_x, rest = b / tiles_x;
  const uint32_t ty = rest % tiles_y, sg = rest / tiles_y;
  const uint32_t c0y = ty * SY, c0x = tx * SX;
  const int tky = (int)min<uint32_t>(SY, nc1 - c0y), tkx = (int)min<uint32_t>(SX, nc2 - c0x);
  const uint32_t py0 = cpos32(c0y, nf1), px0 = cpos32(c0x, nf2);
  const uint32_t lo1 = py0 >= 2 ? py0 - 2 : 0, lo2 = px0 >= 2 ? px0 - 2 : 0;
  const int ext1 = (int)(min<uint32_t>(cpos32(c0y + tky - 1, nf1) + 2, nf1 - 1) - lo1 + 1);
  const int ext2 = (int)(min<uint32_t>(cpos32(c0x + tkx - 1, nf2) + 2, nf2 - 1) - lo2 + 1);
  const uint32_t cz0 = sg * (uint32_t)seg, cz1 = min<uint32_t>(cz0 + seg, nc0);
  const uint32_t pz0 = cpos32(cz0, nf0);
  const uint32_t zs = pz0 >= 2 ? pz0 - 2 : 0;
  const uint32_t ze = min<uint32_t>(cpos32(cz1 - 1, nf0) + 2, nf0 - 1);
  const int tid = threadIdx.x;
  // per-block tables
  for (int i = tid; i < ext1; i += 256) {
    sm.wl1[i] = g.ax[1].wl[lo1 + i];
    sm.wr1[i] = g.ax[1].wr[lo1 + i];
  }
  for (int i = tid; i < ext2; i += 256) {
    sm.wl2[i] = g.ax[2].wl[lo2 + i];
    sm.wr2[i] = g.ax[2].wr[lo2 + i];
  }
  for (int i = tid; i < 5 * tky; i += 256) sm.W1[i / 5][i % 5] = g.ax[1].W[5 * c0y + i];
  for (int i = tid; i < 5 * tkx; i += 256) sm.W2[i / 5][i % 5] = g.ax[2].W[5 * c0x + i];
  for (int i = tid; i < tky; i += 256) sm.P1[i] = (int)(cpos32(c0y + i, nf1) - lo1);
  for (int i = tid; i < tkx; i += 256) sm.P2[i] = (int)(cpos32(c0x + i, nf2) - lo2);
  // the lane's values of a plane: offsets inside the plane and LDS slots
  const int n_pl = ext1 * ext2;
  const uint64_t m2 = div_magic((uint32_t)ext2);
  uint32_t goff[kStreamNLD];
  int ldst[kStreamNLD];
#pragma unroll
  for (int u = 0; u < kStreamNLD; ++u) {
    const int e = min(u * 256 + tid, n_pl - 1);
    const int y = (int)div_small((uint32_t)e, m2), x = e - y * ext2;
    goff[u] = (lo1 + y) * nf2 + lo2 + x;
    ldst[u] = u * 256 + tid < n_pl ? y * E2 + x : -1;
  }
  const size_t plane = (size_t)nf1 * nf2;
  // kDecStreamPF planes of loads in flight, one register set per plane in
  // fixed roles (the plane loop is unrolled by kDecStreamPF); a set is reloaded
  // with the plane kDecStreamPF ahead right after it has gone to LDS.
  Tin pv[kDecStreamPF][kStreamNLD];
  auto load_plane = [&](uint32_t z, Tin (&v)[kStreamNLD]) {
    const Tin* src = G + (size_t)z * plane;
#pragma unroll
    for (int u = 0; u < kStreamNLD; ++u) v[u] = src[goff[u]];
  };
  // x pass: thread column cx, rows y = rsub, rsub + 8, ...
  const int xcol = tid & 31, xrow = tid >> 5;
  int xf[5];
  double xw[5];
  {
    __syncthreads();  // tables
    const int p = xcol < tkx ? sm.P2[xcol] : 0;
#pragma unroll
    for (int d = 0; d < 5; ++d) {
      xf[d] = min(max(p + d - 2, 0), ext2 - 1);
      xw[d] = xcol < tkx ? sm.W2[xcol][d] : 0.0;
    }
  }
  // y pass / z pass / cells: thread (cy, cx)
  const int ocy = tid >> 5, ocx = tid & 31;
  const bool own = ocy < tky && ocx < tkx;
  int yf[5];
  double yw[5];
  {
    const int p = own ? sm.P1[ocy] : 0;
#pragma unroll
    for (int d = 0; d < 5; ++d) {
      yf[d] = min(max(p + d - 2, 0), ext1 - 1);
      yw[d] = own ? sm.W1[ocy][d] : 0.0;
    }
  }
  // cell geometry along y and x (fixed per thread)
  const uint32_t J1 = c0y + ocy, J2 = c0x + ocx;
  const bool h1 = own && 2 * J1 + 1 < nf1 - 1, h2 = own && 2 * J2 + 1 < nf2 - 1;
  const int p1 = own ? (int)(cpos32(J1, nf1) - lo1) : 0, p2 = own ? (int)(cpos32(J2, nf2) - lo2) : 0;
  const int q1 = h1 ? p1 + 1 : p1, q2 = h2 ? p2 + 1 : p2;
  const int s1 = h1 ? p1 + 2 : p1, s2 = h2 ? p2 + 2 : p2;
  const double wy0 = sm.wl1[q1], wy1 = sm.wr1[q1], wx0 = sm.wl2[q2], wx1 = sm.wr2[q2];
  const uint32_t e1c = nc1, e1n = nf1 - nc1, e2c = nc2, e2n = nf2 - nc2;
  const uint32_t lvl = (uint32_t)g.level_off;
  const int m0 = g.bit[0] >= 0 ? 1 << g.bit[0] : 0, m1 = g.bit[1] >= 0 ? 1 << g.bit[1] : 0,
            m2b = g.bit[2] >= 0 ? 1 << g.bit[2] : 0;
  // first stream position of each subband of the level (uniform)
  uint32_t so[8];
  subband_offsets(g, so);
  const uint32_t sb_x = lvl + sel8(so, m2b), sb_y = lvl + sel8(so, m1),
                 sb_yx = lvl + sel8(so, m1 | m2b), sb_z = lvl + sel8(so, m0),
                 sb_zx = lvl + sel8(so, m0 | m2b), sb_zy = lvl + sel8(so, m0 | m1),
                 sb_zyx = lvl + sel8(so, m0 | m1 | m2b);
  uint32_t next_cz = cz0;
#pragma unroll
  for (int d = 0; d < kDecStreamPF; ++d) load_plane(min<uint32_t>(zs + d, ze), pv[d]);
  for (uint32_t zb = zs; zb <= ze; zb += kDecStreamPF) {
#pragma unroll
  for (int d = 0; d < kDecStreamPF; ++d) {
    const uint32_t zf = zb + d;
    if (zf > ze) break;
    const int s3 = (int)(zf % 3u), s5 = (int)(zf % 5u);
#pragma unroll
    for (int u = 0; u < kStreamNLD; ++u)
      if (ldst[u] >= 0) (&sm.raw[s3][0][0])[ldst[u]] = pv[d][u];
    if (zf + kDecStreamPF <= ze) load_plane(zf + kDecStreamPF, pv[d]);
    __syncthreads();
    if (xcol < tkx) {
      for (int y = xrow; y < ext1; y += 8) {
        const Tin* row = sm.raw[s3][y];
        double acc = 0.0;
#pragma unroll
        for (int d = 0; d < 5; ++d) acc = fma(xw[d], (double)row[xf[d]], acc);
        sm.X[y][xcol] = acc;
      }
    }
    __syncthreads();
    if (own) {
      double acc = 0.0;
#pragma unroll
      for (int d = 0; d < 5; ++d) acc = fma(yw[d], sm.X[yf[d]][ocx], acc);
      sm.Y[s5][ocy][ocx] = acc;
    }
    __syncthreads();
    // coarse planes whose last fine plane is this one
    while (next_cz < cz1 && min<uint32_t>(cpos32(next_cz, nf0) + 2, nf0 - 1) == zf) {
      const uint32_t J0 = next_cz;
      const uint32_t P0 = cpos32(J0, nf0);
      const bool h0 = 2 * J0 + 1 < nf0 - 1;
      const double* W0 = g.ax[0].W + 5 * (size_t)J0;
      if (own) {
        double acc = 0.0;
#pragma unroll
        for (int d = 0; d < 5; ++d) {
          const int zz = min(max((int)P0 + d - 2, 0), (int)nf0 - 1);
          acc = fma(W0[d], sm.Y[zz % 5][ocy][ocx], acc);
        }
        fout[((size_t)J0 * nc1 + J1) * nc2 + J2] = acc;
      }
      if (own && (h0 || h1 || h2)) {
        const int r0 = (int)(P0 % 3u), rq = (int)((h0 ? P0 + 1 : P0) % 3u),
                  rs = (int)((h0 ? P0 + 2 : P0) % 3u);
        const double wz0 = h0 ? g.ax[0].wl[P0 + 1] : 1.0, wz1 = h0 ? g.ax[0].wr[P0 + 1] : 0.0;
        auto T = [&](int pz, int y, int x) -> double { return (double)sm.raw[pz][y][x]; };
        const double c000 = T(r0, p1, p2), c001 = T(r0, p1, s2), c010 = T(r0, s1, p2),
                     c011 = T(r0, s1, s2), c100 = T(rs, p1, p2), c101 = T(rs, p1, s2),
                     c110 = T(rs, s1, p2), c111 = T(rs, s1, s2);
        const double ix00 = lin2(wx0, c000, wx1, c001), ix01 = lin2(wx0, c010, wx1, c011);
        const double ix10 = lin2(wx0, c100, wx1, c101), ix11 = lin2(wx0, c110, wx1, c111);
        const uint32_t base_cc = (J0 * e1c + J1) * e2c + J2, base_cn = (J0 * e1c + J1) * e2n + J2;
        const uint32_t base_nc = (J0 * e1n + J1) * e2c + J2, base_nn = (J0 * e1n + J1) * e2n + J2;
        auto emit = [&](uint32_t pos, double v) {
          if (QUANT) emit_q(pos, v, r, sym, ob, status);
          else raw[pos] = v;
        };
        if (h2) emit(sb_x + base_cn, T(r0, p1, q2) - ix00);
        if (h1) emit(sb_y + base_nc, T(r0, q1, p2) - (lin2(wy0, c000, wy1, c010)));
        if (h1 && h2)
          emit(sb_yx + base_nn, T(r0, q1, q2) - (lin2(wy0, ix00, wy1, ix01)));
        if (h0) emit(sb_z + base_cc, T(rq, p1, p2) - (lin2(wz0, c000, wz1, c100)));
        if (h0 && h2)
          emit(sb_zx + base_cn, T(rq, p1, q2) - (lin2(wz0, ix00, wz1, ix10)));
        if (h0 && h1)
          emit(sb_zy + base_nc,
               T(rq, q1, p2) - (lin2(wz0, lin2(wy0, c000, wy1, c010), wz1, lin2(wy0, c100, wy1, c110))));
        if (h0 && h1 && h2)
          emit(sb_zyx + base_nn,
               T(rq, q1, q2) - (lin2(wz0, lin2(wy0, ix00, wy1, ix01), wz1, lin2(wy0, ix10, wy1, ix11))));
      }
      ++next_cz;
    }
    __syncthreads();
  }
  }
}

// ------------------------ recomposition restriction of a 3-axis level, streamed
// f = (P^T M_l) c_l with the same z streaming as k_dec_stream: each fine
// plane of the block's region is assembled from the dequantised coefficients
// (zero at the nodes coarse along every axis) and restricted along x and y;
// the y results of the last five planes stay in an LDS ring for the z pass.
// A lane's region slots are fixed, so a coefficient's stream position is a
// per-slot base (for the plane's new or coarse z) plus j0 times the
// subband's plane stride.
struct RecStreamSmem {
  double P[kStreamE1][kStreamE2];
  double X[kStreamE1][kStreamSX];
  double Y[5][kStreamSY][kStreamSX];
  double W1[kStreamSY][5], W2[kStreamSX][5];
  int P1[kStreamSY], P2[kStreamSX];
};

template <bool RAW>
__global__ __launch_bounds__(256, 4) void k_rec_stream(const LevelGeom g, const CoeffSrc src,
                                                     const double q, double* __restrict__ fout,
                                                     const int seg, const uint32_t n_blocks) {
  constexpr int SY = kStreamSY, SX = kStreamSX, E2 = kStreamE2;
  __shared__ RecStreamSmem sm;
  const uint32_t b = xcd_tile(blockIdx.x, gridDim.x);
  if (b >= n_blocks) return;
  const uint32_t nf0 = (uint32_t)g.nf[0], nf1 = (uint32_t)g.nf[1], nf2 = (uint32_t)g.nf[2];
  const uint32_t nc0 = (uint32_t)g.nc[0], nc1 = (uint32_t)g.nc[1], nc2 = (uint32_t)g.nc[2];
  const uint32_t tiles_x = (nc2 + SX - 1) / SX, tiles_y = (nc1 + SY - 1) / SY;
  const uint32_t tx = b % tiles_x, rest = b / tiles_x;
  const uint32_t ty = rest % tiles_y, sg = rest / tiles_y;
  const uint32_t c0y = ty * SY, c0x = tx * SX;
  const int tky = (int)min<uint32_t>(SY, nc1 - c0y), tkx = (int)min<uint32_t>(SX, nc2 - c0x);
  const uint32_t py0 = cpos32(c0y, nf1), px0 = cpos32(c0x, nf2);
  const uint32_t lo1 = py0 >= 2 ? py0 - 2 : 0, lo2 = px0 >= 2 ? px0 - 2 : 0;
  const int ext1 = (int)(min<uint32_t>(cpos32(c0y + tky - 1, nf1) + 2, nf1 - 1) - lo1 + 1);
  const int ext2 = (int)(min<uint32_t>(cpos32(c0x + tkx - 1, nf2) + 2, nf2 - 1) - lo2 + 1);
  const uint32_t cz0 = sg * (uint32_t)seg, cz1 = min<uint32_t>(cz0 + seg, nc0);
  const uint32_t pz0 = cpos32(cz0, nf0);
  const uint32_t zs = pz0 >= 2 ? pz0 - 2 : 0;
  const uint32_t ze = min<uint32_t>(cpos32(cz1 - 1, nf0) + 2, nf0 - 1);
  const int tid = threadIdx.x;
  for (int i = tid; i < 5 * tky; i += 256) sm.W1[i / 5][i % 5] = g.ax[1].W[5 * c0y + i];
  for (int i = tid; i < 5 * tkx; i += 256) sm.W2[i / 5][i % 5] = g.ax[2].W[5 * c0x + i];
  for (int i = tid; i < tky; i += 256) sm.P1[i] = (int)(cpos32(c0y + i, nf1) - lo1);
  for (int i = tid; i < tkx; i += 256) sm.P2[i] = (int)(cpos32(c0x + i, nf2) - lo2);
  // the lane's region slots: stream position = pbase[n0] + j0 * pstride
  // (n0: the plane's z is a new node); coarse along all axes -> no value
  const int n_pl = ext1 * ext2;
  const uint64_t m2 = div_magic((uint32_t)ext2);
  const uint32_t e1c = nc1, e1n = nf1 - nc1, e2c = nc2, e2n = nf2 - nc2;
  const int mb0 = g.bit[0] >= 0 ? 1 << g.bit[0] : 0, mb1 = g.bit[1] >= 0 ? 1 << g.bit[1] : 0,
            mb2 = g.bit[2] >= 0 ? 1 << g.bit[2] : 0;
  uint32_t so[8];
  subband_offsets(g, so);
  const uint32_t lvl = (uint32_t)g.level_off;
  // stream position of slot u on a plane that is new (n0) or coarse along z:
  // base + j0 * stride (j0: the plane's index among the planes of its kind)
  auto slot_base = [&](int u, bool n0, uint32_t& stride, bool& yx) -> uint32_t {
    const int e = min(u * 256 + tid, n_pl - 1);
    const int y = (int)div_small((uint32_t)e, m2), x = e - y * ext2;
    const uint32_t i1 = lo1 + y, i2 = lo2 + x;
    const bool n1 = is_new32(i1, nf1), n2 = is_new32(i2, nf2);
    const uint32_t j1 = n1 ? (i1 >> 1) : cidx32(i1, nf1);
    const uint32_t j2 = n2 ? (i2 >> 1) : cidx32(i2, nf2);
    const uint32_t ex1 = n1 ? e1n : e1c, ex2 = n2 ? e2n : e2c;
    const int myx = (n1 ? mb1 : 0) | (n2 ? mb2 : 0);
    stride = ex1 * ex2;
    yx = n1 || n2;
    return lvl + sel8(so, n0 ? (myx | mb0) : myx) + j1 * ex2 + j2;
  };
  // running positions of the next coarse and the next new plane to load
  // (planes are loaded once each, in order; the first coarse plane at or
  // after zs has j0 = (zs + 1) / 2, the first new one j0 = zs / 2)
  uint32_t pc[kStreamNLD], pn[kStreamNLD], pstride[kStreamNLD];
  int ldst[kStreamNLD];  // LDS slot | 1 << 30 when new along y or x; -1: none
#pragma unroll
  for (int u = 0; u < kStreamNLD; ++u) {
    uint32_t st;
    bool yx;
    const uint32_t bc = slot_base(u, false, st, yx), bn = slot_base(u, true, st, yx);
    pstride[u] = st;
    pc[u] = bc + ((zs + 1) >> 1) * st;
    pn[u] = bn + (zs >> 1) * st;
    const int e = min(u * 256 + tid, n_pl - 1);
    const int y = (int)div_small((uint32_t)e, m2), x = e - y * ext2;
    ldst[u] = u * 256 + tid < n_pl ? ((y * E2 + x) | (yx ? 1 << 30 : 0)) : -1;
  }
  const int xcol = tid & 31, xrow = tid >> 5;
  int xf[5];
  double xw[5];
  __syncthreads();  // tables
  {
    const int p = xcol < tkx ? sm.P2[xcol] : 0;
#pragma unroll
    for (int d = 0; d < 5; ++d) {
      xf[d] = min(max(p + d - 2, 0), ext2 - 1);
      xw[d] = xcol < tkx ? sm.W2[xcol][d] : 0.0;
    }
  }
  const int ocy = tid >> 5, ocx = tid & 31;
  const bool own = ocy < tky && ocx < tkx;
  int yf[5];
  double yw[5];
  {
    const int p = own ? sm.P1[ocy] : 0;
#pragma unroll
    for (int d = 0; d < 5; ++d) {
      yf[d] = min(max(p + d - 2, 0), ext1 - 1);
      yw[d] = own ? sm.W1[ocy][d] : 0.0;
    }
  }
  const uint32_t J1 = c0y + ocy, J2 = c0x + ocx;
  // coefficient loads of a plane (symbols or FP64 values): kStreamPF planes
  // in flight, one register set per plane in fixed roles (the plane loop is
  // unrolled by kStreamPF)
  // (a set holds only the loaded values: a slot's stream position and
  // whether it holds a coefficient are recomputed from the plane index)
  struct PlaneRegs {
    uint32_t sv[kStreamNLD];
    double rv[kStreamNLD];
  };
  PlaneRegs pr[kStreamPF];
  auto load_plane = [&](uint32_t z, PlaneRegs& R) {
    const bool n0 = is_new32(z, nf0);
#pragma unroll
    for (int u = 0; u < kStreamNLD; ++u) {
      const bool has = ldst[u] >= 0 && (n0 || (ldst[u] >> 30) != 0);
      const uint32_t pos = has ? (n0 ? pn[u] : pc[u]) : 0u;
      if (n0) pn[u] += pstride[u];
      else pc[u] += pstride[u];
      if (RAW) R.rv[u] = src.raw[pos];
      else R.sv[u] = src.sym[pos];
    }
  };
  uint32_t next_cz = cz0;
#pragma unroll
  for (int d = 0; d < kStreamPF; ++d)
    if (zs + d <= ze) load_plane(zs + d, pr[d]);
  for (uint32_t zb = zs; zb <= ze; zb += kStreamPF) {
#pragma unroll
  for (int d = 0; d < kStreamPF; ++d) {
    const uint32_t zf = zb + d;
    if (zf > ze) break;
    const int s5 = (int)(zf % 5u);
    const bool n0 = is_new32(zf, nf0);
#pragma unroll
    for (int u = 0; u < kStreamNLD; ++u) {
      if (ldst[u] < 0) continue;
      double v = 0.0;
      if (n0 || (ldst[u] >> 30) != 0) {
        if (RAW) {
          v = pr[d].rv[u];
        } else if (pr[d].sv[u] != 0) {
          v = (double)((int)pr[d].sv[u] - 32768) * q;
        } else {
          // escaped value (rare): its stream position from scratch
          uint32_t st;
          bool yx;
          const uint32_t j0 = n0 ? (zf >> 1) : cidx32(zf, nf0);
          v = (double)escaped_k(src, slot_base(u, n0, st, yx) + j0 * st) * q;
        }
      }
      (&sm.P[0][0])[ldst[u] & 0xFFFF] = v;
    }
    __syncthreads();
    if (zf + kStreamPF <= ze) load_plane(zf + kStreamPF, pr[d]);
    if (xcol < tkx) {
      for (int y = xrow; y < ext1; y += 8) {
        const double* row = sm.P[y];
        double acc = 0.0;
#pragma unroll
        for (int d = 0; d < 5; ++d) acc = fma(xw[d], row[xf[d]], acc);
        sm.X[y][xcol] = acc;
      }
    }
    __syncthreads();
    if (own) {
      double acc = 0.0;
#pragma unroll
      for (int d = 0; d < 5; ++d) acc = fma(yw[d], sm.X[yf[d]][ocx], acc);
      sm.Y[s5][ocy][ocx] = acc;
    }
    __syncthreads();
    while (next_cz < cz1 && min<uint32_t>(cpos32(next_cz, nf0) + 2, nf0 - 1) == zf) {
      const uint32_t J0 = next_cz;
      const uint32_t P0 = cpos32(J0, nf0);
      const double* W0 = g.ax[0].W + 5 * (size_t)J0;
      if (own) {
        double acc = 0.0;
#pragma unroll
        for (int d = 0; d < 5; ++d) {
          const int zz = min(max((int)P0 + d - 2, 0), (int)nf0 - 1);
          acc = fma(W0[d], sm.Y[zz % 5][ocy][ocx], acc);
        }
        fout[((size_t)J0 * nc1 + J1) * nc2 + J2] = acc;
      }
      ++next_cz;
    }
  }
  }
}


// --------------------------------------------- recomposition of one level
// f = (P^T M_l) c_l: the tile holds the dequantised coefficients (zero at the
// coarse nodes); then the same separable restriction.
// The tile of dequantised coefficients (zero at coarse nodes) is assembled by
// coarse cells (see lerp_cells): the cells whose nodes meet the loaded region
// are the tile's own plus one more on each side of each active axis.  Every
// coefficient load of a thread (coalesced per subband: consecutive threads,
// consecutive cells) and the tables' loads are in flight before any is used.
template <int TZ, int TY, int TX, bool RAW>
__device__ __forceinline__ void rec_restrict_body(const LevelGeom& g, const CoeffSrc& src,
                                                  const double q, double* __restrict__ fout,
                                                  uint32_t t) {
  constexpr int E0 = Ext<TZ>::v, E1 = Ext<TY>::v, E2 = Ext<TX>::v;
  static_assert(E0 * TY * TX <= E0 * E1 * E2, "B aliases the tile");
  constexpr int X0 = TZ == 1 ? 1 : TZ + 2, X1 = TY == 1 ? 1 : TY + 2, X2 = TX == 1 ? 1 : TX + 2;
  constexpr int NX = X0 * X1 * X2, NCR = (NX + 255) / 256;
  __shared__ double tile[E0 * E1 * E2];
  __shared__ double A[E0 * E1 * TX];
  __shared__ TileTabs<E0, E1, E2, TZ, TY, TX> tb;
  const uint32_t tiles_x = (uint32_t)((g.nc[2] + TX - 1) / TX);
  const uint32_t tiles_y = (uint32_t)((g.nc[1] + TY - 1) / TY);
  Tile tl;
  if (!make_tile<TZ, TY, TX>(g, t, tiles_x, tiles_y, tl)) return;
  const int tid = threadIdx.x;
  // On an axis of even length the last two coarse nodes are adjacent fine
  // nodes, so a tile that starts at the last coarse node loads one fine node
  // (its new node two coarse nodes back) that none of its cells covers.  The
  // restriction reads that node with weight zero; it must hold a number, not
  // whatever the LDS held before, so such tiles start from zeros.
  bool gap = false;
#pragma unroll
  for (int k = 0; k < 3; ++k)
    gap = gap || (tl.c0[k] >= 1 && cpos32(tl.c0[k], tl.nf[k]) - cpos32(tl.c0[k] - 1, tl.nf[k]) < 2);
  if (gap) {
    for (int i = tid; i < E0 * E1 * E2; i += 256) tile[i] = 0.0;
    __syncthreads();
  }
  uint32_t so[8];
  subband_offsets(g, so);
  const uint32_t e1c = tl.nc[1], e1n = tl.nf[1] - tl.nc[1];
  const uint32_t e2c = tl.nc[2], e2n = tl.nf[2] - tl.nc[2];
  const uint32_t lvl = (uint32_t)g.level_off;
  const int m0 = g.bit[0] >= 0 ? 1 << g.bit[0] : 0, m1 = g.bit[1] >= 0 ? 1 << g.bit[1] : 0,
            m2 = g.bit[2] >= 0 ? 1 << g.bit[2] : 0;
  uint32_t pos[NCR][8], sv[NCR][8];
  double rv[NCR][8];
  int dst[NCR][8];
#pragma unroll
  for (int u = 0; u < NCR; ++u) {
    const int eu = u * 256 + tid, e = min(eu, NX - 1);
    const int ex = e % X2, rest = e / X2, ey = rest % X1, ez = rest / X1;
    const int J0 = (int)tl.c0[0] + ez - (TZ == 1 ? 0 : 1);
    const int J1 = (int)tl.c0[1] + ey - (TY == 1 ? 0 : 1);
    const int J2 = (int)tl.c0[2] + ex - (TX == 1 ? 0 : 1);
    const bool live = eu < NX && J0 >= 0 && J1 >= 0 && J2 >= 0 && J0 < (int)tl.nc[0] &&
                      J1 < (int)tl.nc[1] && J2 < (int)tl.nc[2];
    const uint32_t j0 = live ? J0 : 0, j1 = live ? J1 : 0, j2 = live ? J2 : 0;
    const bool h0 = live && 2 * j0 + 1 < tl.nf[0] - 1, h1 = live && 2 * j1 + 1 < tl.nf[1] - 1,
               h2 = live && 2 * j2 + 1 < tl.nf[2] - 1;
    // tile-relative fine index of the cell origin and of its new node
    const int p0 = (int)cpos32(j0, tl.nf[0]) - (int)tl.lo[0];
    const int p1 = (int)cpos32(j1, tl.nf[1]) - (int)tl.lo[1];
    const int p2 = (int)cpos32(j2, tl.nf[2]) - (int)tl.lo[2];
    const bool iP0 = p0 >= 0 && p0 < tl.ext[0], iP1 = p1 >= 0 && p1 < tl.ext[1],
               iP2 = p2 >= 0 && p2 < tl.ext[2];
    const bool iN0 = h0 && p0 + 1 >= 0 && p0 + 1 < tl.ext[0];
    const bool iN1 = h1 && p1 + 1 >= 0 && p1 + 1 < tl.ext[1];
    const bool iN2 = h2 && p2 + 1 >= 0 && p2 + 1 < tl.ext[2];
    const uint32_t bcc = (j0 * e1c + j1) * e2c + j2, bcn = (j0 * e1c + j1) * e2n + j2;
    const uint32_t bnc = (j0 * e1n + j1) * e2c + j2, bnn = (j0 * e1n + j1) * e2n + j2;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const bool nx = k & 1, ny = k & 2, nz = k & 4;
      const bool ok = live && (nx ? iN2 : iP2) && (ny ? iN1 : iP1) && (nz ? iN0 : iP0);
      const int z = p0 + (nz ? 1 : 0), y = p1 + (ny ? 1 : 0), x = p2 + (nx ? 1 : 0);
      dst[u][k] = ok ? (z * E1 + y) * E2 + x : -1;
      const int m = (nz ? m0 : 0) | (ny ? m1 : 0) | (nx ? m2 : 0);
      const uint32_t bse = ny ? (nx ? bnn : bnc) : (nx ? bcn : bcc);
      pos[u][k] = k != 0 && ok ? lvl + sel8(so, m) + bse : 0u;
      if (k != 0) {
        if (RAW) rv[u][k] = src.raw[pos[u][k]];
        else sv[u][k] = src.sym[pos[u][k]];
      }
    }
  }
  load_tabs(g, tl, tb, false);
#pragma unroll
  for (int u = 0; u < NCR; ++u) {
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      if (dst[u][k] < 0) continue;
      double v = 0.0;
      if (k != 0) v = RAW ? rv[u][k] : dequant(src, sv[u][k], pos[u][k], q);
      tile[dst[u][k]] = v;
    }
  }
  __syncthreads();
  restrict_tile(tile, A, tile, tl, tb, fout);
}

template <int TZ, int TY, int TX, bool RAW>
__global__ __launch_bounds__(256) void k_rec_restrict(const LevelGeom g, const CoeffSrc src,
                                                       const double q, double* __restrict__ fout,
                                                       const uint32_t n_tiles) {
  const uint32_t t = xcd_tile(blockIdx.x, gridDim.x);
  if (t >= n_tiles) return;
  rec_restrict_body<TZ, TY, TX, RAW>(g, src, q, fout, t);
}

// G_l = P Gc + c_l on the tile's owned fine nodes; the coarse values the tile
// needs (its coarse outputs plus one more per axis) are staged in LDS.
// SRC: 0 dequantised symbols, 1 FP64 coefficients, 2 none (plain P Gc).
// Per coarse cell (see lerp_cells): the cell's coarse value and, at its new
// nodes, the multilinear interpolant of its corners plus the coefficient.
// The coarse values the tile needs (its cells and one more per axis) are
// staged in LDS; every global load (coarse values, coefficients, weights)
// is issued before any is used.
template <typename Tout, int TZ, int TY, int TX, int SRC>
__device__ __forceinline__ void rec_interp_body(const double* __restrict__ Gc, const LevelGeom& g,
                                                const CoeffSrc& src, const double q,
                                                Tout* __restrict__ out, uint32_t t) {
  constexpr int E0 = Ext<TZ>::v, E1 = Ext<TY>::v, E2 = Ext<TX>::v;
  constexpr int C0 = TZ == 1 ? 1 : TZ + 1, C1 = TY == 1 ? 1 : TY + 1, C2 = TX == 1 ? 1 : TX + 1;
  constexpr int NC = TZ * TY * TX, NCELL = (NC + 255) / 256;
  __shared__ double gc[C0 * C1 * C2];
  __shared__ TileTabs<E0, E1, E2, TZ, TY, TX> tb;
  const uint32_t tiles_x = (uint32_t)((g.nc[2] + TX - 1) / TX);
  const uint32_t tiles_y = (uint32_t)((g.nc[1] + TY - 1) / TY);
  Tile tl;
  if (!make_tile<TZ, TY, TX>(g, t, tiles_x, tiles_y, tl)) return;
  const int tid = threadIdx.x;
  uint32_t so[8];
  subband_offsets(g, so);
  // 1. coarse values
  constexpr int NGC = (C0 * C1 * C2 + 255) / 256;
  int ce[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) ce[k] = (int)min<uint32_t>(tl.tk[k] + 1, tl.nc[k] - tl.c0[k]);
  const int c12 = ce[1] * ce[2], n_gc = ce[0] * c12;
  const uint64_t mc12 = div_magic((uint32_t)c12), mc2 = div_magic((uint32_t)ce[2]);
  double gv[NGC];
  int gdst[NGC];
#pragma unroll
  for (int u = 0; u < NGC; ++u) {
    const int iu = u * 256 + tid, i = min(iu, n_gc - 1);
    const int a = (int)div_small((uint32_t)i, mc12), rem = i - a * c12;
    const int b = (int)div_small((uint32_t)rem, mc2), c = rem - b * ce[2];
    gv[u] = Gc[((tl.c0[0] + a) * tl.nc[1] + tl.c0[1] + b) * tl.nc[2] + tl.c0[2] + c];
    gdst[u] = iu < n_gc ? (a * C1 + b) * C2 + c : -1;
  }
  // 2. coefficients of the cells' new nodes (node k: bit 0 x, bit 1 y, bit 2 z new)
  const uint32_t e1c = tl.nc[1], e1n = tl.nf[1] - tl.nc[1];
  const uint32_t e2c = tl.nc[2], e2n = tl.nf[2] - tl.nc[2];
  const uint32_t lvl = (uint32_t)g.level_off;
  const int m0 = g.bit[0] >= 0 ? 1 << g.bit[0] : 0, m1 = g.bit[1] >= 0 ? 1 << g.bit[1] : 0,
            m2 = g.bit[2] >= 0 ? 1 << g.bit[2] : 0;
  uint32_t cpos[NCELL][8], csv[NCELL][8];
  double crv[NCELL][8];
#pragma unroll
  for (int u = 0; u < NCELL; ++u) {
    const int e = min(u * 256 + tid, NC - 1);
    const int cx = e % TX, rest = e / TX, cy = rest % TY, cz = rest / TY;
    const uint32_t J0 = tl.c0[0] + cz, J1 = tl.c0[1] + cy, J2 = tl.c0[2] + cx;
    const bool live = u * 256 + tid < NC && cz < tl.tk[0] && cy < tl.tk[1] && cx < tl.tk[2];
    const bool h0 = live && 2 * J0 + 1 < tl.nf[0] - 1, h1 = live && 2 * J1 + 1 < tl.nf[1] - 1,
               h2 = live && 2 * J2 + 1 < tl.nf[2] - 1;
    const uint32_t bcc = (J0 * e1c + J1) * e2c + J2, bcn = (J0 * e1c + J1) * e2n + J2;
    const uint32_t bnc = (J0 * e1n + J1) * e2c + J2, bnn = (J0 * e1n + J1) * e2n + J2;
#pragma unroll
    for (int k = 1; k < 8; ++k) {
      const bool nx = k & 1, ny = k & 2, nz = k & 4;
      const bool ok = (!nx || h2) && (!ny || h1) && (!nz || h0) && live;
      const int m = (nz ? m0 : 0) | (ny ? m1 : 0) | (nx ? m2 : 0);
      const uint32_t bse = ny ? (nx ? bnn : bnc) : (nx ? bcn : bcc);
      cpos[u][k] = SRC != 2 && ok ? lvl + sel8(so, m) + bse : 0u;
      if (SRC == 1) crv[u][k] = src.raw[cpos[u][k]];
      if (SRC == 0) csv[u][k] = src.sym[cpos[u][k]];
    }
  }
  // 3. interpolation weights
  load_tabs(g, tl, tb, true);
#pragma unroll
  for (int u = 0; u < NGC; ++u)
    if (gdst[u] >= 0) gc[gdst[u]] = gv[u];
  __syncthreads();
  // 4. outputs
  auto G = [&](int a, int b, int c) -> double { return gc[(a * C1 + b) * C2 + c]; };
#pragma unroll
  for (int u = 0; u < NCELL; ++u) {
    const int e = u * 256 + tid;
    if (e >= NC) break;
    const int cx = e % TX, rest = e / TX, cy = rest % TY, cz = rest / TY;
    if (cz >= tl.tk[0] || cy >= tl.tk[1] || cx >= tl.tk[2]) continue;
    const uint32_t J0 = tl.c0[0] + cz, J1 = tl.c0[1] + cy, J2 = tl.c0[2] + cx;
    const bool h0 = 2 * J0 + 1 < tl.nf[0] - 1, h1 = 2 * J1 + 1 < tl.nf[1] - 1,
               h2 = 2 * J2 + 1 < tl.nf[2] - 1;
    const uint32_t P0 = cpos32(J0, tl.nf[0]), P1 = cpos32(J1, tl.nf[1]), P2 = cpos32(J2, tl.nf[2]);
    // weights of the new nodes (tile-relative fine index of 2J+1)
    const int r0 = (int)(P0 - tl.lo[0]) + (h0 ? 1 : 0), r1 = (int)(P1 - tl.lo[1]) + (h1 ? 1 : 0),
              r2 = (int)(P2 - tl.lo[2]) + (h2 ? 1 : 0);
    const double wz0 = tb.wl0(r0), wz1 = tb.wr0(r0), wy0 = tb.wl1(r1), wy1 = tb.wr1(r1);
    const double wx0 = tb.wl2(r2), wx1 = tb.wr2(r2);
    const int a1 = h0 ? cz + 1 : cz, b1 = h1 ? cy + 1 : cy, c1 = h2 ? cx + 1 : cx;
    const double c000 = G(cz, cy, cx), c001 = G(cz, cy, c1), c010 = G(cz, b1, cx),
                 c011 = G(cz, b1, c1), c100 = G(a1, cy, cx), c101 = G(a1, cy, c1),
                 c110 = G(a1, b1, cx), c111 = G(a1, b1, c1);
    const double ix00 = lin2(wx0, c000, wx1, c001), ix01 = lin2(wx0, c010, wx1, c011);
    const double ix10 = lin2(wx0, c100, wx1, c101), ix11 = lin2(wx0, c110, wx1, c111);
    auto coef = [&](int k) -> double {
      if (SRC == 2) return 0.0;
      return SRC == 1 ? crv[u][k] : dequant(src, csv[u][k], cpos[u][k], q);
    };
    const uint32_t nf1 = tl.nf[1], nf2 = tl.nf[2];
    auto put = [&](uint32_t i0, uint32_t i1, uint32_t i2, double v) {
      out[(i0 * nf1 + i1) * nf2 + i2] = (Tout)v;
    };
    put(P0, P1, P2, c000);
    if (h2) put(P0, P1, P2 + 1, ix00 + coef(1));
    if (h1) put(P0, P1 + 1, P2, (lin2(wy0, c000, wy1, c010)) + coef(2));
    if (h1 && h2) put(P0, P1 + 1, P2 + 1, (lin2(wy0, ix00, wy1, ix01)) + coef(3));
    if (h0) put(P0 + 1, P1, P2, (lin2(wz0, c000, wz1, c100)) + coef(4));
    if (h0 && h2) put(P0 + 1, P1, P2 + 1, (lin2(wz0, ix00, wz1, ix10)) + coef(5));
    if (h0 && h1)
      put(P0 + 1, P1 + 1, P2,
          (lin2(wz0, lin2(wy0, c000, wy1, c010), wz1, lin2(wy0, c100, wy1, c110))) + coef(6));
    if (h0 && h1 && h2)
      put(P0 + 1, P1 + 1, P2 + 1,
          (lin2(wz0, lin2(wy0, ix00, wy1, ix01), wz1, lin2(wy0, ix10, wy1, ix11))) + coef(7));
  }
}

template <typename Tout, int TZ, int TY, int TX, int SRC>
__global__ __launch_bounds__(256) void k_rec_interp(const double* __restrict__ Gc,
                                                     const LevelGeom g, const CoeffSrc src,
                                                     const double q, Tout* __restrict__ out,
                                                     const uint32_t n_tiles) {
  const uint32_t t = xcd_tile(blockIdx.x, gridDim.x);
  if (t >= n_tiles) return;
  rec_interp_body<Tout, TZ, TY, TX, SRC>(Gc, g, src, q, out, t);
}

// --------------------------------------------------------- adjoint pieces
// cbar at the new nodes of level l: g - (M_l Pv), the fine mass matrix applied
// as a 3x3x3 stencil to the prolongated coarse solution Pv.
__global__ __launch_bounds__(256) void k_adj_mass(const double* __restrict__ Pv,
                                                   const double* __restrict__ gl,
                                                   const LevelGeom g, double* __restrict__ cbar) {
  const uint32_t nf0 = (uint32_t)g.nf[0], nf1 = (uint32_t)g.nf[1], nf2 = (uint32_t)g.nf[2];
  const uint32_t i2 = blockIdx.x * 256 + threadIdx.x;
  if (i2 >= nf2) return;
  Tile tl;
  for (int k = 0; k < 3; ++k) {
    tl.nf[k] = (uint32_t)g.nf[k];
    tl.nc[k] = (uint32_t)g.nc[k];
  }
  uint32_t soff[8];
#pragma unroll
  for (int m = 0; m < 8; ++m) soff[m] = (uint32_t)(m == 0 ? 0 : g.sub_off[m]);
  const bool n2 = is_new32(i2, nf2);
  const uint32_t rows = nf0 * nf1;
  for (uint32_t row = blockIdx.y; row < rows; row += gridDim.y) {
    const uint32_t i0 = row / nf1, i1 = row - i0 * nf1;
    const bool n0 = is_new32(i0, nf0), n1 = is_new32(i1, nf1);
    if (!(n0 || n1 || n2)) continue;
    double acc = 0.0;
    for (int a = -1; a <= 1; ++a) {
      const int64_t j0 = (int64_t)i0 + a;
      if (j0 < 0 || j0 >= nf0) continue;
      const double w0 = g.ax[0].Mt[3 * i0 + a + 1];
      for (int b = -1; b <= 1; ++b) {
        const int64_t j1 = (int64_t)i1 + b;
        if (j1 < 0 || j1 >= nf1) continue;
        const double w1 = g.ax[1].Mt[3 * i1 + b + 1];
        const double* prow = Pv + ((size_t)j0 * nf1 + j1) * nf2;
        double s2 = 0.0;
        for (int c = -1; c <= 1; ++c) {
          const int64_t j2 = (int64_t)i2 + c;
          if (j2 < 0 || j2 >= nf2) continue;
          s2 += g.ax[2].Mt[3 * i2 + c + 1] * prow[j2];
        }
        acc += w0 * w1 * s2;
      }
    }
    const uint32_t pos = stream_pos(g, tl, soff, i0, i1, i2, n0, n1, n2);
    cbar[pos] = gl[((size_t)i0 * nf1 + i1) * nf2 + i2] - acc;
  }
}

// ------------------------------------------------------------- tridiagonal
// Thomas sweeps with the pre-factored coarse mass matrix (pivot reciprocals
// m_i, sub- and super-diagonal scaled by them, a_i and c_i): forward
// y_i = m_i f_i - a_i y_{i-1}, backward x_i = y_i - c_i x_{i+1}, each one
// fused multiply-add on the dependence chain (the same arithmetic in every
// sweep kernel).  a_0 = c_{n-1} = 0 and the sweeps start from y_{-1} =
// x_n = 0, which leave the first and last steps exact.
__device__ __forceinline__ double thomas_fwd(double f, double a, double m, double prev) {
  return fma(-a, prev, m * f);
}
__device__ __forceinline__ double thomas_bwd(double y, double c, double nxt) {
  return fma(-c, nxt, y);
}
//
// Strided axes: one thread per line, adjacent lanes on adjacent lines (the
// contiguous index), so every access is coalesced; values are moved in blocks
// of U so that U loads are in flight before the recurrence consumes them.
// Line t of the axis (lines ordered by their contiguous index).
template <int AXIS, int U>
__device__ __forceinline__ void thomas_strided_body(double* __restrict__ x, int64_t n0,
                                                    int64_t n1, int64_t n2,
                                                    const double* __restrict__ ta,
                                                    const double* __restrict__ tm,
                                                    const double* __restrict__ tc,
                                                    const double* __restrict__ sub, int64_t t) {
  int64_t len, stride, base;
  if (AXIS == 1) {
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
  // each sweep keeps the next batch's loads in flight while it runs the
  // recurrence over the current batch.  Two register buffers alternate in
  // fixed roles (the loop takes two batches per iteration) and every load is
  // issued unconditionally from a clamped index, so no copy of freshly
  // loaded registers makes the wavefront wait for them; the batches a sweep
  // reads ahead are not yet written.
  double* p = x + base;
  const double* ps = sub ? sub + base : nullptr;
  const int64_t last = len - 1;
  double va[U], vb[U], sa[U], sb[U];
  auto fload = [&](int64_t i0, double (&v)[U]) {
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = p[min<int64_t>(i0 + u, last) * stride];
  };
  double prev = 0.0;
  auto fsweep = [&](int64_t i0, double (&v)[U]) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t i = min<int64_t>(i0 + u, last);
      v[u] = thomas_fwd(v[u], ta[i], tm[i], prev);
      prev = v[u];
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (i0 + u < len) p[(i0 + u) * stride] = v[u];
  };
  fload(0, va);
  for (int64_t i0 = 0; i0 < len; i0 += 2 * U) {
    fload(i0 + U, vb);
    fsweep(i0, va);
    if (i0 + U >= len) break;
    fload(i0 + 2 * U, va);
    fsweep(i0 + U, vb);
  }
  // backward: batch k covers i = hi, hi-1, ..., hi-U+1 (indices below 0 are
  // clamped reads whose results are not stored)
  auto bload = [&](int64_t hi, double (&v)[U], double (&sv)[U]) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t i = max<int64_t>(hi - u, 0);
      v[u] = p[i * stride];
      sv[u] = ps ? ps[i * stride] : 0.0;
    }
  };
  double nxt = 0.0;
  auto bsweep = [&](int64_t hi, double (&v)[U], const double (&sv)[U]) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t i = max<int64_t>(hi - u, 0);
      v[u] = thomas_bwd(v[u], tc[i], nxt);
      nxt = v[u];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t i = hi - u;
      if (i >= 0) p[i * stride] = ps ? sv[u] - v[u] : v[u];
    }
  };
  bload(last, va, sa);
  for (int64_t hi = last; hi >= 0; hi -= 2 * U) {
    bload(hi - U, vb, sb);
    bsweep(hi, va, sa);
    if (hi - U < 0) break;
    bload(hi - 2 * U, va, sa);
    bsweep(hi - U, vb, sb);
  }
}

template <int AXIS, int U>
__global__ __launch_bounds__(256) void k_thomas_strided(double* __restrict__ x, int64_t n0,
                                                         int64_t n1, int64_t n2,
                                                         const double* __restrict__ ta,
                                                         const double* __restrict__ tm,
                                                         const double* __restrict__ tc,
                                                         const double* __restrict__ sub) {
  thomas_strided_body<AXIS, U>(x, n0, n1, n2, ta, tm, tc, sub,
                               (int64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

// Contiguous axis: one wavefront per 64 rows.  Segments of SEG elements of
// the 64 rows are staged through LDS with coalesced loads and stores; each
// lane then runs the recurrence along its own row inside LDS.
// Value of lane l (uniform) of a double held by every lane of the wavefront.
__device__ __forceinline__ double readlane_d(double v, int l) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
  return __hiloint2double(hi, lo);
}

template <int SEG>
__device__ __forceinline__ void thomas_rows_body(double* __restrict__ x, int64_t nrows,
                                                 int64_t n, const double* __restrict__ ta,
                                                 const double* __restrict__ tm,
                                                 const double* __restrict__ tc,
                                                 const double* __restrict__ sub, int64_t blk) {
  static_assert(SEG <= 64 && 64 % SEG == 0, "segment divides the wavefront");
  constexpr int RP = 64 / SEG;  // rows per wavefront load (SEG lanes per row)
  constexpr int K = SEG;        // loads per lane per segment (64 rows)
  __shared__ double buf[64][SEG + 1];
  const int lane = threadIdx.x;
  const int64_t r0 = blk * 64;
  const int nr = (int)min<int64_t>(64, nrows - r0);
  const int c = lane % SEG, jr = lane / SEG;
  // a segment of the 64 rows: every load of a lane in flight at once, plus
  // the segment's factors (lane c holds entry s0 + c; the recurrence reads
  // them back with a uniform lane index).  The recurrence runs on all 64
  // lanes, also past the last row (those LDS rows hold clamped copies of a
  // real row and are never stored): under a lane-dependent branch the
  // compiler may move the factor loads into it, and a lane read back by
  // readlane would then be one that never loaded.
  // Segments move through two register sets in fixed roles (the loops take
  // two segments per iteration): the next segment's loads are in flight
  // while the current one is solved, and no copy of freshly loaded
  // registers makes the wavefront wait for them.  Indices are clamped to the
  // row, so a segment past either end reads valid, unused values.
  struct SegRegs {
    double v[K], w[K], fa, fm, fc;
  };
  auto seg_load = [&](int64_t s0, SegRegs& R, const double* src2) {
    const int64_t cc = min<int64_t>(max<int64_t>(s0, 0) + c, n - 1);
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int j = min(jr + k * RP, nr - 1);
      R.v[k] = x[(r0 + j) * n + cc];
      if (src2) R.w[k] = src2[(r0 + j) * n + cc];
    }
    R.fa = ta[cc];
    R.fm = tm[cc];
    R.fc = tc[cc];
  };
  double prev = 0.0;
  auto fwd_seg = [&](int64_t s0, const SegRegs& R) {
    const int ns = (int)min<int64_t>(SEG, n - s0);
#pragma unroll
    for (int k = 0; k < K; ++k) buf[jr + k * RP][c] = R.v[k];
    __syncthreads();
    for (int i = 0; i < ns; ++i) {
      const double a = readlane_d(R.fa, i), m = readlane_d(R.fm, i);
      const double y = thomas_fwd(buf[lane][i], a, m, prev);
      buf[lane][i] = y;
      prev = y;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int j = jr + k * RP;
      if (j < nr && c < ns) x[(r0 + j) * n + s0 + c] = buf[j][c];
    }
    __syncthreads();
  };
  double nxt = 0.0;
  auto bwd_seg = [&](int64_t s0, const SegRegs& R) {
    const int ns = (int)min<int64_t>(SEG, n - s0);
#pragma unroll
    for (int k = 0; k < K; ++k) buf[jr + k * RP][c] = R.v[k];
    __syncthreads();
    for (int i = ns - 1; i >= 0; --i) {
      const double cf = readlane_d(R.fc, i);
      const double y = thomas_bwd(buf[lane][i], cf, nxt);
      buf[lane][i] = y;
      nxt = y;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int j = jr + k * RP;
      if (j < nr && c < ns) {
        const int64_t gi = (r0 + j) * n + s0 + c;
        x[gi] = sub ? R.w[k] - buf[j][c] : buf[j][c];
      }
    }
    __syncthreads();
  };
  SegRegs A, B;
  seg_load(0, A, nullptr);
  for (int64_t s0 = 0; s0 < n; s0 += 2 * SEG) {
    seg_load(s0 + SEG, B, nullptr);
    fwd_seg(s0, A);
    if (s0 + SEG >= n) break;
    seg_load(s0 + 2 * SEG, A, nullptr);
    fwd_seg(s0 + SEG, B);
  }
  const int64_t sl = ((n - 1) / SEG) * SEG;
  seg_load(sl, A, sub);
  for (int64_t s0 = sl; s0 >= 0; s0 -= 2 * SEG) {
    seg_load(s0 - SEG, B, sub);
    bwd_seg(s0, A);
    if (s0 - SEG < 0) break;
    seg_load(s0 - 2 * SEG, A, sub);
    bwd_seg(s0 - SEG, B);
  }
}

template <int SEG>
__global__ __launch_bounds__(64) void k_thomas_rows(double* __restrict__ x, int64_t nrows,
                                                     int64_t n, const double* __restrict__ ta,
                                                     const double* __restrict__ tm,
                                                     const double* __restrict__ tc,
                                                     const double* __restrict__ sub) {
  thomas_rows_body<SEG>(x, nrows, n, ta, tm, tc, sub, blockIdx.x);
}


// Partitioned sweeps for coarse grids above the LDS-tile limit.  A line is
// cut into segments whose values stay in registers from their load to their
// store, so every value is read once and written once per axis.  The forward
// recurrence is affine in its start value: inside a segment starting at s it
// runs from zero (y^_i), and the true value is y_i = y^_i + alpha_i y_{s-1}
// with alpha_i = prod_{j=s..i} (-a_j).  The segments' end values chain the
// start values from segment to segment (one multiply-add each); the backward
// sweep splits the same way with beta_i = prod_{j=i..e-1} (-c_j) and the next
// segment's first value.  Results agree with the serial sweep up to rounding.
//
// Strided axes: lanes take 64 adjacent lines (coalesced rows of 512 bytes)
// and the W wavefronts of a block take W consecutive segments of them; the
// chain of carries runs through LDS.
// The segmentation depends only on the line length: W = ceil(len / SEG)
// segments of sl = ceil(len / W) values, so a block of more wavefronts than W
// (the batched form sizes blocks for its longest line) computes the same
// values; its spare wavefronts carry identity maps through the chains.
// A segment of ns values sits at the end of the SEG register slots; the
// off = SEG - ns slots before it are padding steps with a = -1, m = 0 in the
// forward sweep (y stays y, here 0) and c = -1 with y = 0 in the backward
// sweep (x stays x), both exact, so the sweeps run without per-value
// branches.  Lane j holds the factors of slot j and the sweeps broadcast
// them with readlane, so no scalar load sits on the recurrence.
constexpr int kPartWaves = 8;  // segments (wavefronts) per block at most
template <int AXIS, int SEG>
__device__ __forceinline__ void thomas_part_body(double* __restrict__ x, int64_t n0, int64_t n1,
                                                 int64_t n2, const double* __restrict__ ta,
                                                 const double* __restrict__ tm,
                                                 const double* __restrict__ tc,
                                                 const double* __restrict__ sub, int64_t blk) {
  static_assert(SEG <= 64, "one factor slot per lane");
  __shared__ double cy[kPartWaves][64], cx[kPartWaves][64];
  __shared__ double ca[kPartWaves], cb[kPartWaves];
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int W = (int)(blockDim.x >> 6);
  int64_t lines, len, stride;
  if (AXIS == 1) {
    lines = n0 * n2;
    len = n1;
    stride = n2;
  } else {
    lines = n1 * n2;
    len = n0;
    stride = n1 * n2;
  }
  // segment geometry in scalar registers (wavefront-uniform)
  const int len32 = (int)len;
  const int nseg = (len32 + SEG - 1) / SEG;
  const int sl = __builtin_amdgcn_readfirstlane((len32 + nseg - 1) / nseg);
  const int s = w * sl;
  const int ns = __builtin_amdgcn_readfirstlane(max(min(sl, len32 - s), 0));
  const int off = SEG - ns;
  // the lane's line as a byte offset from the block's first line (below 2^32
  // for every grid the library accepts: at most the grid's 8-byte values), so
  // each row access is a uniform address plus a 32-bit lane offset
  const int64_t tf = blk * 64;
  const int64_t t0 = tf + lane;
  const bool live = t0 < lines;
  const int64_t t = live ? t0 : lines - 1;
  int64_t bf, bt;
  if (AXIS == 1) {
    bf = (tf / n2) * n1 * n2 + tf % n2;
    bt = (t / n2) * n1 * n2 + t % n2;
  } else {
    bf = tf;
    bt = t;
  }
  const uint32_t lb = (uint32_t)(bt - bf) * 8u;  // bytes
  double* const xb = x + bf;
  // row i of the segment's lines: uniform row address plus the lane's bytes
  const auto at = [&](double* base, int64_t i) -> double& {
    return *reinterpret_cast<double*>(reinterpret_cast<char*>(base + i * stride) + lb);
  };
  double fa = -1.0, fm = 0.0, fc = -1.0;
  if (lane >= off && lane < SEG) {
    const int i = s + lane - off;
    fa = ta[i];
    fm = tm[i];
    fc = tc[i];
  }
  double v[SEG];
  if (ns > 0) {
#pragma unroll
    for (int k = 0; k < SEG; ++k) {
      v[k] = at(xb, max(s + k - off, s));  // padding slots reload the first value
    }
  } else {
#pragma unroll
    for (int k = 0; k < SEG; ++k) v[k] = 0.0;
  }
  // forward sweep of the segment from a zero start
  double prev = 0.0, A = 1.0;
#pragma unroll
  for (int k = 0; k < SEG; ++k) {
    const double a = readlane_d(fa, k);
    prev = thomas_fwd(v[k], a, readlane_d(fm, k), prev);
    v[k] = prev;
    A *= -a;
  }
  cy[w][lane] = prev;
  if (lane == 0) ca[w] = A;
  __syncthreads();
  if (w > 0) {
    double yin = 0.0;
    for (int j = 0; j < w; ++j) yin = fma(ca[j], yin, cy[j][lane]);
    double al = 1.0;
#pragma unroll
    for (int k = 0; k < SEG; ++k) {
      al *= -readlane_d(fa, k);
      if (k >= off) v[k] = fma(al, yin, v[k]);  // padding slots stay 0
    }
  }
  // backward sweep of the segment from a zero end
  double nxt = 0.0, B = 1.0;
#pragma unroll
  for (int k = SEG - 1; k >= 0; --k) {
    const double c = readlane_d(fc, k);
    nxt = thomas_bwd(v[k], c, nxt);
    v[k] = nxt;
    B *= -c;
  }
  cx[w][lane] = nxt;
  if (lane == 0) cb[w] = B;
  __syncthreads();
  if (w < W - 1) {
    double xin = 0.0;
    for (int j = W - 1; j > w; --j) xin = fma(cb[j], xin, cx[j][lane]);
    double be = 1.0;
#pragma unroll
    for (int k = SEG - 1; k >= 0; --k) {
      be *= -readlane_d(fc, k);
      v[k] = fma(be, xin, v[k]);
    }
  }
  if (!live) return;
  if (sub) {
    double* const qb = const_cast<double*>(sub) + bf;
#pragma unroll
    for (int k = 0; k < SEG; ++k)
      if (k >= off) at(xb, s + k - off) = at(qb, s + k - off) - v[k];
  } else {
#pragma unroll
    for (int k = 0; k < SEG; ++k)
      if (k >= off) at(xb, s + k - off) = v[k];
  }
}

template <int AXIS, int SEG>
__global__ __launch_bounds__(64 * kPartWaves) void k_thomas_part(
    double* __restrict__ x, int64_t n0, int64_t n1, int64_t n2, const double* __restrict__ ta,
    const double* __restrict__ tm, const double* __restrict__ tc,
    const double* __restrict__ sub, uint32_t nblk) {
  // Consecutive line windows share their edge cache lines (rows are not
  // line-aligned), so each XCD takes a contiguous range of windows.
  const uint32_t b = xcd_tile(blockIdx.x, gridDim.x);
  if (b >= nblk) return;
  thomas_part_body<AXIS, SEG>(x, n0, n1, n2, ta, tm, tc, sub, b);
}

// Contiguous axis: one wavefront per row at a time, lane l holding the row's
// values l*sl .. l*sl+sl-1 (sl = ceil(n / 64)).  Rows move between HBM and
// registers through LDS with coalesced loads and stores; the chains of
// carries are wavefront scans of the segments' affine maps (composition of
// y -> B + A y is associative).  Each lane keeps its factors in registers
// for every row it solves.
__device__ __forceinline__ double shfl_up_d(double v, int o) { return __shfl_up(v, o, 64); }
__device__ __forceinline__ double shfl_down_d(double v, int o) { return __shfl_down(v, o, 64); }

constexpr int kRowScanWaves = 4;
// (rows blk * 4 + wavefront, then every nblk * 4 rows)
template <int K>
__device__ __forceinline__ void thomas_rowscan_body(double* __restrict__ x, int64_t nrows,
                                                    int64_t n, const double* __restrict__ ta,
                                                    const double* __restrict__ tm,
                                                    const double* __restrict__ tc,
                                                    const double* __restrict__ sub, int64_t blk,
                                                    int64_t nblk) {
  __shared__ double buf[kRowScanWaves][64 * K];
  const int lane = threadIdx.x & 63;
  const int wv = (int)(threadIdx.x >> 6);
  double* b = buf[wv];
  const int sl = (int)((n + 63) / 64);
  const int s = lane * sl;
  const int ns = (int)max<int64_t>(min<int64_t>(sl, n - s), 0);
  double fa[K], fm[K], fc[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int64_t i = min<int64_t>(s + k, n - 1);
    fa[k] = ta[i];
    fm[k] = tm[i];
    fc[k] = tc[i];
  }
  const int64_t step = nblk * kRowScanWaves;
  // Row r's values (g) and the values it is subtracted from (q) are loaded
  // one row ahead: the next row's loads are in flight while this row is
  // solved, and its q loads while the next row is.
  int64_t r = blk * kRowScanWaves + wv;
  double g[K], q[K];
  if (r < nrows) {
#pragma unroll
    for (int k = 0; k < K; ++k) g[k] = x[r * n + min<int64_t>(lane + 64 * k, n - 1)];
    if (sub) {
#pragma unroll
      for (int k = 0; k < K; ++k) q[k] = sub[r * n + min<int64_t>(lane + 64 * k, n - 1)];
    }
  }
  for (; r < nrows; r += step) {
    double* row = x + r * n;
    const int64_t rn = r + step;
#pragma unroll
    for (int k = 0; k < K; ++k)
      if (lane + 64 * k < n) b[lane + 64 * k] = g[k];
    if (rn < nrows) {
#pragma unroll
      for (int k = 0; k < K; ++k) g[k] = x[rn * n + min<int64_t>(lane + 64 * k, n - 1)];
    }
    wave_fence();
    double v[K];
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = b[min<int64_t>(s + k, n - 1)];
    // forward sweep of the lane's segment from a zero start, then the scan
    // of the segments' maps y_end = B + A y_start
    double B = 0.0, A = 1.0;
#pragma unroll
    for (int k = 0; k < K; ++k)
      if (k < ns) {
        B = thomas_fwd(v[k], fa[k], fm[k], B);
        v[k] = B;
        A *= -fa[k];
      }
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const double Ao = shfl_up_d(A, o), Bo = shfl_up_d(B, o);
      if (lane >= o) {
        B = fma(A, Bo, B);
        A *= Ao;
      }
    }
    double yin = shfl_up_d(B, 1);
    if (lane == 0) yin = 0.0;
    {
      double al = 1.0;
#pragma unroll
      for (int k = 0; k < K; ++k)
        if (k < ns) {
          al *= -fa[k];
          v[k] = fma(al, yin, v[k]);
        }
    }
    // backward sweep from a zero end, then the scan of the maps
    // x_start = X + C x_end from the last lane down
    double X = 0.0, C = 1.0;
#pragma unroll
    for (int k = K - 1; k >= 0; --k)
      if (k < ns) {
        X = thomas_bwd(v[k], fc[k], X);
        v[k] = X;
        C *= -fc[k];
      }
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const double Co = shfl_down_d(C, o), Xo = shfl_down_d(X, o);
      if (lane + o < 64) {
        X = fma(C, Xo, X);
        C *= Co;
      }
    }
    double xin = shfl_down_d(X, 1);
    if (lane == 63) xin = 0.0;
    {
      double be = 1.0;
#pragma unroll
      for (int k = K - 1; k >= 0; --k)
        if (k < ns) {
          be *= -fc[k];
          v[k] = fma(be, xin, v[k]);
        }
    }
    wave_fence();
#pragma unroll
    for (int k = 0; k < K; ++k)
      if (k < ns) b[s + k] = v[k];
    wave_fence();
    if (sub) {
#pragma unroll
      for (int k = 0; k < K; ++k)
        if (lane + 64 * k < n) row[lane + 64 * k] = q[k] - b[lane + 64 * k];
      if (rn < nrows) {
#pragma unroll
        for (int k = 0; k < K; ++k) q[k] = sub[rn * n + min<int64_t>(lane + 64 * k, n - 1)];
      }
    } else {
#pragma unroll
      for (int k = 0; k < K; ++k)
        if (lane + 64 * k < n) row[lane + 64 * k] = b[lane + 64 * k];
    }
    wave_fence();
  }
}

template <int K>
__global__ __launch_bounds__(64 * kRowScanWaves) void k_thomas_rowscan(
    double* __restrict__ x, int64_t nrows, int64_t n, const double* __restrict__ ta,
    const double* __restrict__ tm, const double* __restrict__ tc,
    const double* __restrict__ sub) {
  thomas_rowscan_body<K>(x, nrows, n, ta, tm, tc, sub, blockIdx.x, gridDim.x);
}

// Whole lines in LDS, one tile per wavefront.  Each wavefront holds 16
// lines of the axis in its own part of LDS: lines adjacent along the
// contiguous axis for the strided axes (the 16 values at one position are
// 128 contiguous bytes), 16 consecutive rows for the contiguous axis (one
// contiguous block).  It loads the tile with sixteen loads per lane in
// flight, runs the forward and backward sweeps in LDS (one lane per line,
// values and factors through registers in batches) and writes the tile back:
// each value is read and written once per axis, where the segment-staged
// sweeps read and write the forward pass's values a second time.  The
// wavefronts of a block share only the factor tables, so one can sweep
// while the others load or store.
constexpr int kTileLines = 16;
constexpr int kThomasTile4MaxL = 280;  // four tiles per block
constexpr int kThomasTile2MaxL = 540;  // two tiles per block

__host__ __device__ constexpr size_t thomas_tile_lds(int64_t L, int tiles) {
  return ((size_t)L * ((size_t)tiles * (kTileLines + 1) + 3) + (size_t)tiles * kTileLines) *
         sizeof(double);
}

template <int TILES, int AXIS>
__global__ __launch_bounds__(64 * TILES) void k_thomas_tile(double* __restrict__ x, int64_t n0,
                                                             int64_t n1, int64_t n2,
                                                             const double* __restrict__ ta,
                                                             const double* __restrict__ tm,
                                                             const double* __restrict__ tc,
                                                             const double* __restrict__ sub) {
  constexpr int W = kTileLines, NB = 32;
  extern __shared__ double tsm[];
  const int L = (int)(AXIS == 0 ? n0 : (AXIS == 1 ? n1 : n2));
  // strided axes: [position][line] with pitch W + 1; rows: [line][position]
  // with pitch L + 1; room for either
  const int tile_sz = L * (W + 1) + W;
  double* fa = tsm;
  double* fm = fa + L;
  double* fc = fm + L;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  double* T = fc + L + wave * tile_sz;
  for (int i = tid; i < L; i += 64 * TILES) {
    fa[i] = ta[i];
    fm[i] = tm[i];
    fc[i] = tc[i];
  }
  const int64_t tile = (int64_t)blockIdx.x * TILES + wave;
  // first value of the tile, lines in it, distance between positions
  int64_t base0, estride;
  int nl;
  bool live = true;
  if (AXIS == 2) {
    const int64_t r0 = tile * W, rows = n0 * n1;
    live = r0 < rows;
    nl = live ? (int)min<int64_t>(W, rows - r0) : 0;
    base0 = live ? r0 * n2 : 0;
    estride = 1;
  } else if (AXIS == 1) {
    const int64_t gpp = (n2 + W - 1) / W;
    const int64_t i0 = tile / gpp, x0 = (tile - i0 * gpp) * W;
    live = i0 < n0;
    nl = live ? (int)min<int64_t>(W, n2 - x0) : 0;
    base0 = live ? i0 * n1 * n2 + x0 : 0;
    estride = n2;
  } else {
    const int64_t t0 = tile * W, m = n1 * n2;
    live = t0 < m;
    nl = live ? (int)min<int64_t>(W, m - t0) : 0;
    base0 = live ? t0 : 0;
    estride = m;
  }
  __syncthreads();  // factor tables
  if (!live) return;
  const int total = L * nl;  // values in the tile
  // lane's k-th value: global address and LDS slot
  //   rows: value e = lane + 64k of the contiguous block, line e / L
  //   strided: line lane % 16, position lane / 16 + 4k
  const uint64_t mL = div_magic((uint32_t)L);
  const int jl = lane & (W - 1), il = lane >> 4;
  const bool lane_ok = AXIS == 2 || jl < nl;
  double* gp = x + base0 + (AXIS == 2 ? 0 : (int64_t)min(jl, nl - 1) + (int64_t)il * estride);
  const int n_k = AXIS == 2 ? (total + 63) / 64 : (L + 3) / 4;
  auto slot = [&](int k, int& dst) -> int64_t {  // returns the global offset from gp
    if (AXIS == 2) {
      const int e = min(lane + 64 * k, total - 1);
      const int j = (int)div_small((uint32_t)e, mL);
      dst = lane + 64 * k < total ? e + j : -1;  // j * (L + 1) + (e - j * L)
      return e;
    } else {
      const int i = min(il + 4 * k, L - 1);
      dst = lane_ok && il + 4 * k < L ? i * (W + 1) + jl : -1;
      return (int64_t)(i - il) * estride;
    }
  };
  for (int k0 = 0; k0 < n_k; k0 += NB) {
    double v[NB];
    int dst[NB];
#pragma unroll
    for (int u = 0; u < NB; ++u) v[u] = gp[slot(k0 + u, dst[u])];
#pragma unroll
    for (int u = 0; u < NB; ++u)
      if (dst[u] >= 0) T[dst[u]] = v[u];
  }
  wave_fence();
  if (lane < nl) {
    // one line per lane; values and factors move through registers in
    // batches of U, the next batch's LDS reads issued before the current
    // batch's recurrence
    constexpr int U = 8;
    const int pitch = AXIS == 2 ? 1 : W + 1;
    double* c = AXIS == 2 ? T + lane * (L + 1) : T + lane;
    double v[U], a[U], m[U], nv[U], na[U], nm[U];
    auto fwd_load = [&](int i0, double (&pv)[U], double (&pa)[U], double (&pm)[U]) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int i = min(i0 + u, L - 1);
        pv[u] = c[i * pitch];
        pa[u] = fa[i];
        pm[u] = fm[i];
      }
    };
    double prev = 0.0;
    fwd_load(0, v, a, m);
    for (int i0 = 0; i0 < L; i0 += U) {
      if (i0 + U < L) fwd_load(i0 + U, nv, na, nm);
#pragma unroll
      // past the line's end the factors are clamped and the values unused
      for (int u = 0; u < U; ++u) {
        v[u] = thomas_fwd(v[u], a[u], m[u], prev);
        prev = v[u];
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (i0 + u < L) c[(i0 + u) * pitch] = v[u];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        v[u] = nv[u];
        a[u] = na[u];
        m[u] = nm[u];
      }
    }
    auto bwd_load = [&](int hi, double (&pv)[U], double (&pc)[U]) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int i = max(hi - u, 0);
        pv[u] = c[i * pitch];
        pc[u] = fc[i];
      }
    };
    double nxt = 0.0;
    bwd_load(L - 1, v, a);
    for (int hi = L - 1; hi >= 0; hi -= U) {
      if (hi - U >= 0) bwd_load(hi - U, nv, na);
#pragma unroll
      for (int u = 0; u < U; ++u) {
        v[u] = thomas_bwd(v[u], a[u], nxt);
        nxt = v[u];
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (hi - u >= 0) c[(hi - u) * pitch] = v[u];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        v[u] = nv[u];
        a[u] = na[u];
      }
    }
  }
  wave_fence();
  double* gq = gp;
  const double* sp = sub ? sub + (gp - x) : nullptr;
  for (int k0 = 0; k0 < n_k; k0 += NB) {
    double sv[NB];
    int64_t off[NB];
    int src[NB];
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      off[u] = slot(k0 + u, src[u]);
      sv[u] = sp ? sp[off[u]] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < NB; ++u)
      if (src[u] >= 0) gq[off[u]] = sp ? sv[u] - T[src[u]] : T[src[u]];
  }
}

// A coarse grid that fits in LDS: the three sweeps (axis 2, then 1, then 0,
// the order of the per-axis launches) in one workgroup, one thread per line,
// with the same arithmetic; sub - x is formed on the way out, as the last
// per-axis sweep would.  Saves two launches (and their latency) per level on
// the small levels.
constexpr int kThomasGridMax = 16384;  // points (128 KiB of FP64)
constexpr int kThomasGridMaxLine = 128;

struct Thomas3Args {
  const double* ta[3];
  const double* tm[3];
  const double* tc[3];
  int active[3];
};

// Forward and backward sweep of one line held in LDS (L values, stride
// apart), four LDS loads issued ahead of each group of four dependent steps.
__device__ __forceinline__ void lds_line_sweep(double* line, int L, int stride,
                                               const double* __restrict__ ta,
                                               const double* __restrict__ tm,
                                               const double* __restrict__ tc) {
  double prev = 0.0;
  for (int i0 = 0; i0 < L; i0 += 4) {
    double v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = line[min(i0 + u, L - 1) * stride];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int i = min(i0 + u, L - 1);
      v[u] = thomas_fwd(v[u], ta[i], tm[i], prev);
      if (i0 + u < L) prev = v[u];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (i0 + u < L) line[(i0 + u) * stride] = v[u];
  }
  double nxt = 0.0;
  for (int i0 = L - 1; i0 >= 0; i0 -= 4) {
    double v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = line[max(i0 - u, 0) * stride];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int i = max(i0 - u, 0);
      v[u] = thomas_bwd(v[u], tc[i], nxt);
      if (i0 - u >= 0) nxt = v[u];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (i0 - u >= 0) line[(i0 - u) * stride] = v[u];
  }
}

// n contiguous values from global memory into LDS (eight loads per thread in
// flight), and back with sub - value formed on the way out when sub is set.
template <int NT>
__device__ __forceinline__ void block_load_lds(const double* __restrict__ src, double* dst, int n) {
  constexpr int NB = 8;
  for (int i0 = threadIdx.x; i0 < n; i0 += NB * NT) {
    double v[NB];
#pragma unroll
    for (int u = 0; u < NB; ++u) v[u] = src[min(i0 + u * NT, n - 1)];
#pragma unroll
    for (int u = 0; u < NB; ++u)
      if (i0 + u * NT < n) dst[i0 + u * NT] = v[u];
  }
}
template <int NT>
__device__ __forceinline__ void block_store_lds(double* __restrict__ dst, const double* src, int n,
                                                const double* __restrict__ sub) {
  constexpr int NB = 8;
  for (int i0 = threadIdx.x; i0 < n; i0 += NB * NT) {
    double sv[NB];
#pragma unroll
    for (int u = 0; u < NB; ++u) sv[u] = sub ? sub[min(i0 + u * NT, n - 1)] : 0.0;
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int i = i0 + u * NT;
      if (i < n) dst[i] = sub ? sv[u] - src[i] : src[i];
    }
  }
}

constexpr int kThomasGridThreads = 1024;

__global__ __launch_bounds__(kThomasGridThreads) void k_thomas_grid(
    double* __restrict__ x, int64_t n0, int64_t n1, int64_t n2, const Thomas3Args a,
    const double* __restrict__ sub) {
  constexpr int NT = kThomasGridThreads;
  constexpr int ML = kThomasGridMaxLine;
  extern __shared__ double gsm[];
  // the factors of every active axis go to LDS with the grid, so that the
  // sweeps' steps wait on LDS only
  __shared__ double tab[3][3][ML];
  const int n = (int)(n0 * n1 * n2);
  const int64_t nn[3] = {n0, n1, n2};
  for (int i = threadIdx.x; i < 9 * ML; i += NT) {
    const int axis = i / (3 * ML), k = (i / ML) % 3, j = i % ML;
    if (a.active[axis] && j < (int)nn[axis]) {
      const double* src = k == 0 ? a.ta[axis] : (k == 1 ? a.tm[axis] : a.tc[axis]);
      tab[axis][k][j] = src[j];
    }
  }
  block_load_lds<NT>(x, gsm, n);
  __syncthreads();
  for (int axis = 2; axis >= 0; --axis) {
    if (!a.active[axis]) continue;
    const int L = (int)nn[axis];
    const int lines = n / L;
    const int stride = axis == 2 ? 1 : (axis == 1 ? (int)n2 : (int)(n1 * n2));
    for (int t = threadIdx.x; t < lines; t += NT) {
      int base;
      if (axis == 2) base = t * (int)n2;
      else if (axis == 1) base = (t / (int)n2) * (int)(n1 * n2) + t % (int)n2;
      else base = t;
      lds_line_sweep(gsm + base, L, stride, tab[axis][0], tab[axis][1], tab[axis][2]);
    }
    __syncthreads();
  }
  block_store_lds<NT>(x, gsm, n, sub);
}

// ------------------------------------------------ the smallest levels, one block
// The last levels of a hierarchy (fine grids of at most kTailMax points) run
// in one workgroup with every grid in LDS: per level the cells (interpolation
// and quantisation, or recomposition's interpolation plus coefficients), the
// separable restriction (x, then y, then z) and the coarse solves (axes 2,
// 1, 0), with block barriers where the level loop has launches.  Each value
// is formed by the same operations in the same order as in the tiled level
// kernels and the LDS-resident solve (k_thomas_grid), so the results agree
// bit for bit.  The levels' operator tables are one contiguous range of the
// plan's table block (level by level, axis by axis: wl, wr, W, ta, tm, tc and
// the adjoint's tables), copied to LDS with the first grid and the levels'
// geometry, so the kernel waits on memory once before its first level.
constexpr int kTailMax = 4913;     // fine points of the largest level taken (17^3)
constexpr int kTailCoarse = 2464;  // coarse points (and nf0 nc1 nc2) of that level at most
constexpr int kTailLine = 128;     // longest active coarse line (one thread per line)
constexpr int kTailTab = 2048;     // doubles of the table range
constexpr int kTailThreads = 512;

// Pointers into the LDS table copy for one level and axis.
struct TailAxis {
  const double *wl, *wr, *W, *ta;
};
__device__ __forceinline__ TailAxis tail_axis(const double* tab, const TailTabArgs& ta,
                                              const LevelGeom& g, int l, int k) {
  const double* b = tab + ta.wl[l][k];
  const int nf = (int)g.nf[k], nc = (int)g.nc[k];
  return TailAxis{b, b + nf, b + 2 * nf, b + 2 * nf + 5 * nc};
}

// Copies the table range and the geometry of levels 1..top (all loads of a
// thread issued before its stores).  No barrier.
__device__ __forceinline__ void tail_fetch(const TailTabArgs& ta, double* tab,
                                           const LevelGeom* __restrict__ geo, int top,
                                           LevelGeom* sgeo) {
  const int tid = threadIdx.x;
  if (tid >= 1 && tid <= top) sgeo[tid] = geo[tid];
  for (uint32_t i0 = tid; i0 < ta.n; i0 += 8 * kTailThreads) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = ta.src[min(i0 + u * kTailThreads, ta.n - 1)];
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (i0 + u * kTailThreads < ta.n) tab[i0 + u * kTailThreads] = v[u];
  }
}

// The separable restriction (x, then y, then z; taps clamped to the grid,
// where out-of-grid taps have weight zero) of the fine grid F (dims nf) to
// the coarse grid C (dims nc); A and B scratch (B may alias F).
__device__ void tail_restrict(const double* F, double* A, double* B, double* C,
                              const LevelGeom& g, const double* W0, const double* W1,
                              const double* W2) {
  const int tid = threadIdx.x;
  const int nf0 = (int)g.nf[0], nf1 = (int)g.nf[1], nf2 = (int)g.nf[2];
  const int nc0 = (int)g.nc[0], nc1 = (int)g.nc[1], nc2 = (int)g.nc[2];
  const int nA = nf0 * nf1 * nc2;
  for (int e = tid; e < nA; e += kTailThreads) {
    const int cx = e % nc2, row = e / nc2;
    const int p = (int)cpos32((uint32_t)cx, (uint32_t)nf2);
    const double* r = F + row * nf2;
    double acc = 0.0;
#pragma unroll
    for (int d = 0; d < 5; ++d) acc = fma(W2[5 * cx + d], r[min(max(p + d - 2, 0), nf2 - 1)], acc);
    A[e] = acc;
  }
  __syncthreads();
  const int nB = nf0 * nc1 * nc2;
  for (int e = tid; e < nB; e += kTailThreads) {
    const int cx = e % nc2, rest = e / nc2, cy = rest % nc1, z = rest / nc1;
    const int p = (int)cpos32((uint32_t)cy, (uint32_t)nf1);
    double acc = 0.0;
#pragma unroll
    for (int d = 0; d < 5; ++d)
      acc = fma(W1[5 * cy + d], A[(z * nf1 + min(max(p + d - 2, 0), nf1 - 1)) * nc2 + cx], acc);
    B[e] = acc;
  }
  __syncthreads();
  const int nC = nc0 * nc1 * nc2;
  for (int e = tid; e < nC; e += kTailThreads) {
    const int cyx = e % (nc1 * nc2), cz = e / (nc1 * nc2);
    const int p = (int)cpos32((uint32_t)cz, (uint32_t)nf0);
    double acc = 0.0;
#pragma unroll
    for (int d = 0; d < 5; ++d)
      acc = fma(W0[5 * cz + d], B[min(max(p + d - 2, 0), nf0 - 1) * (nc1 * nc2) + cyx], acc);
    C[e] = acc;
  }
  __syncthreads();
}

// The solves of the coarse grid C (dims nc) along its active axes, 2, then
// 1, then 0, one thread per line (as k_thomas_grid).
__device__ void tail_solve(double* C, const LevelGeom& g, const TailAxis (&ax)[3]) {
  const int n0 = (int)g.nc[0], n1 = (int)g.nc[1], n2 = (int)g.nc[2];
  const int n = n0 * n1 * n2;
  const int nn[3] = {n0, n1, n2};
  for (int axis = 2; axis >= 0; --axis) {
    if (g.bit[axis] < 0) continue;
    const int L = nn[axis];
    const int lines = n / L;
    const int stride = axis == 2 ? 1 : (axis == 1 ? n2 : n1 * n2);
    const double* ta = ax[axis].ta;
    for (int t = threadIdx.x; t < lines; t += kTailThreads) {
      int base;
      if (axis == 2) base = t * n2;
      else if (axis == 1) base = (t / n2) * (n1 * n2) + t % n2;
      else base = t;
      lds_line_sweep(C + base, L, stride, ta, ta + L, ta + 2 * L);
    }
    __syncthreads();
  }
}

struct DecTailSmem {
  double X[kTailMax];     // fine grid of the level (or, alternately, its coarse grid)
  double Y[kTailCoarse];  // coarse grid (or, alternately, the fine grid)
  double A[kTailMax];     // restriction along x
  double tab[kTailTab];
  LevelGeom geo[kTailLevels];
  double r[kTailLevels];  // reciprocal bins
  unsigned n_esc;
};

// Decomposition of levels top..1 and level 0: G holds level top's grid.
// The launch is the only writer of the outlier records while it runs (the
// compression's kernels run in stream order), so its escaped values take
// the records after the count it finds, numbered by an LDS counter, and the
// count is advanced once at the end.
template <typename Tin, bool QUANT>
__global__ __launch_bounds__(kTailThreads) void k_dec_tail(
    const Tin* __restrict__ G, const LevelGeom* __restrict__ geo, const int top,
    const TailTabArgs tt, uint16_t* __restrict__ sym, double* __restrict__ raw,
    const double* __restrict__ rdev, const OutlierBuf ob, unsigned* __restrict__ status,
    const unsigned* __restrict__ gate) {
  if (gate_closed(gate)) return;
  __shared__ DecTailSmem sm;
  const int tid = threadIdx.x;
  if (tid == 0) sm.n_esc = 0;
  if (QUANT && tid <= top) sm.r[tid] = rdev[tid];
  const unsigned long long ebase =
      QUANT ? __hip_atomic_load(ob.count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0ull;
  {
    // the grid's first loads in flight across the table copy
    const int n = (int)(geo[top].nf[0] * geo[top].nf[1] * geo[top].nf[2]);
    for (int i0 = tid, first = 1; i0 < n || first; i0 += 8 * kTailThreads, first = 0) {
      Tin v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = G[min(i0 + u * kTailThreads, n - 1)];
      if (first) tail_fetch(tt, sm.tab, geo, top, sm.geo);
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (i0 + u * kTailThreads < n) sm.X[i0 + u * kTailThreads] = (double)v[u];
    }
  }
  __syncthreads();
  // Quantises up to seven values of a lane (emit_q's symbol and escape); the
  // wavefront reserves its escapes' records with one LDS add.
  auto emit_cell = [&](const uint32_t (&pos)[8], const double (&v)[8], const bool (&ok)[8],
                       double r) {
    if (!QUANT) {
#pragma unroll
      for (int k = 1; k < 8; ++k)
        if (ok[k]) raw[pos[k]] = v[k];
      return;
    }
    double t[8];
    bool esc[8];
    unsigned ne = 0;
#pragma unroll
    for (int k = 1; k < 8; ++k) {
      t[k] = rint(v[k] * r);
      esc[k] = ok[k] && !(fabs(t[k]) < 32768.0);
      if (ok[k]) sym[pos[k]] = (uint16_t)(int)((esc[k] ? -32768.0 : t[k]) + 32768.0);
      ne += esc[k] ? 1u : 0u;
    }
    if (__ballot(ne != 0) == 0) return;
    // exclusive prefix of ne (< 8) over the lanes, from its three bits
    const uint64_t lt = (1ull << __lane_id()) - 1;
    unsigned excl = 0, tot = 0;
#pragma unroll
    for (int bit = 0; bit < 3; ++bit) {
      const uint64_t bm = __ballot((ne >> bit) & 1u);
      excl += (unsigned)__popcll(bm & lt) << bit;
      tot += (unsigned)__popcll(bm) << bit;
    }
    unsigned base = 0;
    if (__lane_id() == 0) base = atomicAdd(&sm.n_esc, tot);
    base = (unsigned)__shfl((int)base, 0, 64);
    unsigned long long j = ebase + base + excl;
#pragma unroll
    for (int k = 1; k < 8; ++k) {
      if (!esc[k]) continue;
      int64_t kv = 0;
      if (fabs(t[k]) < 4611686018427387904.0) kv = (int64_t)t[k];
      else atomicOr(status, ST_RANGE);
      if (j < ob.cap) {
        ob.pos[j] = pos[k];
        ob.val[j] = kv;
      }
      ++j;
    }
  };
  double* F = sm.X;  // fine grid of the level
  double* C = sm.Y;  // its coarse grid
  for (int l = top; l >= 1; --l) {
    const LevelGeom& g = sm.geo[l];
    const TailAxis ax[3] = {tail_axis(sm.tab, tt, g, l, 0), tail_axis(sm.tab, tt, g, l, 1),
                            tail_axis(sm.tab, tt, g, l, 2)};
    const double r = QUANT ? sm.r[l] : 0.0;
    const uint32_t nf0 = (uint32_t)g.nf[0], nf1 = (uint32_t)g.nf[1], nf2 = (uint32_t)g.nf[2];
    const uint32_t nc0 = (uint32_t)g.nc[0], nc1 = (uint32_t)g.nc[1], nc2 = (uint32_t)g.nc[2];
    const uint32_t e1c = nc1, e1n = nf1 - nc1, e2c = nc2, e2n = nf2 - nc2;
    const uint32_t lvl = (uint32_t)g.level_off;
    const int m0 = g.bit[0] >= 0 ? 1 << g.bit[0] : 0, m1 = g.bit[1] >= 0 ? 1 << g.bit[1] : 0,
              m2 = g.bit[2] >= 0 ? 1 << g.bit[2] : 0;
    uint32_t so[8];
    subband_offsets(g, so);
    auto T = [&](uint32_t z, uint32_t y, uint32_t x) { return F[(z * nf1 + y) * nf2 + x]; };
    // cells: the new nodes' coefficients (the forms of lerp_cells); every
    // lane of a wavefront takes part in each round (for the reservation)
    const uint32_t ncell = nc0 * nc1 * nc2;
    for (uint32_t e0 = 0; e0 < ncell; e0 += kTailThreads) {
      const uint32_t e = min(e0 + tid, ncell - 1);
      const bool live = e0 + tid < ncell;
      const uint32_t J2 = e % nc2, rest = e / nc2, J1 = rest % nc1, J0 = rest / nc1;
      const bool h0 = 2 * J0 + 1 < nf0 - 1, h1 = 2 * J1 + 1 < nf1 - 1, h2 = 2 * J2 + 1 < nf2 - 1;
      const uint32_t p0 = cpos32(J0, nf0), p1 = cpos32(J1, nf1), p2 = cpos32(J2, nf2);
      const uint32_t s0 = h0 ? p0 + 2 : p0, s1 = h1 ? p1 + 2 : p1, s2 = h2 ? p2 + 2 : p2;
      const uint32_t q0 = h0 ? p0 + 1 : p0, q1 = h1 ? p1 + 1 : p1, q2 = h2 ? p2 + 1 : p2;
      const double wz0 = ax[0].wl[q0], wz1 = ax[0].wr[q0];
      const double wy0 = ax[1].wl[q1], wy1 = ax[1].wr[q1];
      const double wx0 = ax[2].wl[q2], wx1 = ax[2].wr[q2];
      const double c000 = T(p0, p1, p2), c001 = T(p0, p1, s2), c010 = T(p0, s1, p2),
                   c011 = T(p0, s1, s2), c100 = T(s0, p1, p2), c101 = T(s0, p1, s2),
                   c110 = T(s0, s1, p2), c111 = T(s0, s1, s2);
      const double ix00 = lin2(wx0, c000, wx1, c001), ix01 = lin2(wx0, c010, wx1, c011);
      const double ix10 = lin2(wx0, c100, wx1, c101), ix11 = lin2(wx0, c110, wx1, c111);
      const uint32_t base_cc = (J0 * e1c + J1) * e2c + J2, base_cn = (J0 * e1c + J1) * e2n + J2;
      const uint32_t base_nc = (J0 * e1n + J1) * e2c + J2, base_nn = (J0 * e1n + J1) * e2n + J2;
      uint32_t pos[8];
      double v[8];
      bool ok[8];
      pos[0] = 0;
      v[0] = 0.0;
      ok[0] = false;
      pos[1] = lvl + sel8(so, m2) + base_cn;
      v[1] = T(p0, p1, q2) - ix00;
      ok[1] = live && h2;
      pos[2] = lvl + sel8(so, m1) + base_nc;
      v[2] = T(p0, q1, p2) - (lin2(wy0, c000, wy1, c010));
      ok[2] = live && h1;
      pos[3] = lvl + sel8(so, m1 | m2) + base_nn;
      v[3] = T(p0, q1, q2) - (lin2(wy0, ix00, wy1, ix01));
      ok[3] = live && h1 && h2;
      pos[4] = lvl + sel8(so, m0) + base_cc;
      v[4] = T(q0, p1, p2) - (lin2(wz0, c000, wz1, c100));
      ok[4] = live && h0;
      pos[5] = lvl + sel8(so, m0 | m2) + base_cn;
      v[5] = T(q0, p1, q2) - (lin2(wz0, ix00, wz1, ix10));
      ok[5] = live && h0 && h2;
      pos[6] = lvl + sel8(so, m0 | m1) + base_nc;
      v[6] = T(q0, q1, p2) -
             (lin2(wz0, lin2(wy0, c000, wy1, c010), wz1, lin2(wy0, c100, wy1, c110)));
      ok[6] = live && h0 && h1;
      pos[7] = lvl + sel8(so, m0 | m1 | m2) + base_nn;
      v[7] = T(q0, q1, q2) -
             (lin2(wz0, lin2(wy0, ix00, wy1, ix01), wz1, lin2(wy0, ix10, wy1, ix11)));
      ok[7] = live && h0 && h1 && h2;
      emit_cell(pos, v, ok, r);
    }
    // (the restriction's first pass only reads F, as the cells do)
    tail_restrict(F, sm.A, F, C, g, ax[0].W, ax[1].W, ax[2].W);
    tail_solve(C, g, ax);
    double* t = F;
    F = C;
    C = t;
  }
  // level 0: the coarsest grid's values at stream positions 0..
  const LevelGeom& g1 = sm.geo[1];
  const int n0 = (int)(g1.nc[0] * g1.nc[1] * g1.nc[2]);
  const double r0 = QUANT ? sm.r[0] : 0.0;
  for (int i0 = 0; i0 < n0; i0 += kTailThreads) {
    const int i = min(i0 + tid, n0 - 1);
    uint32_t pos[8] = {0, (uint32_t)i, 0, 0, 0, 0, 0, 0};
    double v[8] = {0.0, F[i], 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    bool ok[8] = {false, i0 + tid < n0, false, false, false, false, false, false};
    emit_cell(pos, v, ok, r0);
  }
  if (QUANT) {
    __syncthreads();
    if (tid == 0 && sm.n_esc) atomicAdd(ob.count, (unsigned long long)sm.n_esc);
  }
}

struct TailQ {
  double q[kTailLevels];
};

struct RecTailSmem {
  double X[kTailMax];      // the level's coefficients on its fine grid
  double Y[kTailCoarse];   // coarse grid
  double A[kTailMax];      // restriction along x
  double B[kTailCoarse];   // restriction along y
  double Gp[kTailCoarse];  // the previous level's values (the coarse grid's)
  double tab[kTailTab];
  LevelGeom geo[kTailLevels];
};

// Recomposition of level 0 and levels 1..top: out receives level top's grid.
// Coefficients of levels <= coarse_top come from `coarse` (FP64), the others
// from src.
template <typename Tout>
__global__ __launch_bounds__(kTailThreads) void k_rec_tail(
    const CoeffSrc src, const CoeffSrc coarse, const int coarse_top, const TailQ tq,
    const LevelGeom* __restrict__ geo, const int top, const TailTabArgs tt,
    Tout* __restrict__ out) {
  __shared__ RecTailSmem sm;
  const int tid = threadIdx.x;
  auto coef = [&](int l, uint32_t pos) -> double {
    const CoeffSrc& s = l <= coarse_top ? coarse : src;
    if (s.raw) return s.raw[pos];
    return dequant(s, s.sym[pos], pos, tq.q[l]);
  };
  {
    // level 0 (as k_rec_level0), with the tables and geometry
    const int n0 = (int)(geo[1].nc[0] * geo[1].nc[1] * geo[1].nc[2]);
    for (int i0 = tid, first = 1; i0 < n0 || first; i0 += 8 * kTailThreads, first = 0) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = coef(0, (uint32_t)min(i0 + u * kTailThreads, n0 - 1));
      if (first) tail_fetch(tt, sm.tab, geo, top, sm.geo);
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (i0 + u * kTailThreads < n0) sm.Gp[i0 + u * kTailThreads] = v[u];
    }
  }
  __syncthreads();
  for (int l = 1; l <= top; ++l) {
    const LevelGeom& g = sm.geo[l];
    const TailAxis ax[3] = {tail_axis(sm.tab, tt, g, l, 0), tail_axis(sm.tab, tt, g, l, 1),
                            tail_axis(sm.tab, tt, g, l, 2)};
    const uint32_t nf0 = (uint32_t)g.nf[0], nf1 = (uint32_t)g.nf[1], nf2 = (uint32_t)g.nf[2];
    const uint32_t nc0 = (uint32_t)g.nc[0], nc1 = (uint32_t)g.nc[1], nc2 = (uint32_t)g.nc[2];
    const uint32_t e1c = nc1, e1n = nf1 - nc1, e2c = nc2, e2n = nf2 - nc2;
    const uint32_t lvl = (uint32_t)g.level_off;
    const int m0 = g.bit[0] >= 0 ? 1 << g.bit[0] : 0, m1 = g.bit[1] >= 0 ? 1 << g.bit[1] : 0,
              m2 = g.bit[2] >= 0 ? 1 << g.bit[2] : 0;
    uint32_t so[8];
    subband_offsets(g, so);
    const uint32_t nfine = nf0 * nf1 * nf2, ncell = nc0 * nc1 * nc2;
    auto fidx = [&](uint32_t i0, uint32_t i1, uint32_t i2) { return (i0 * nf1 + i1) * nf2 + i2; };
    // 1. the coefficients on the fine grid (zero at the coarse nodes)
    for (uint32_t i = tid; i < nfine; i += kTailThreads) sm.X[i] = 0.0;
    __syncthreads();
    for (uint32_t e = tid; e < ncell; e += kTailThreads) {
      const uint32_t J2 = e % nc2, rest = e / nc2, J1 = rest % nc1, J0 = rest / nc1;
      const bool h0 = 2 * J0 + 1 < nf0 - 1, h1 = 2 * J1 + 1 < nf1 - 1, h2 = 2 * J2 + 1 < nf2 - 1;
      const uint32_t P0 = cpos32(J0, nf0), P1 = cpos32(J1, nf1), P2 = cpos32(J2, nf2);
      const uint32_t bcc = (J0 * e1c + J1) * e2c + J2, bcn = (J0 * e1c + J1) * e2n + J2;
      const uint32_t bnc = (J0 * e1n + J1) * e2c + J2, bnn = (J0 * e1n + J1) * e2n + J2;
      double v[8];
#pragma unroll
      for (int k = 1; k < 8; ++k) {
        const bool nx = k & 1, ny = k & 2, nz = k & 4;
        const bool ok = (!nx || h2) && (!ny || h1) && (!nz || h0);
        const int m = (nz ? m0 : 0) | (ny ? m1 : 0) | (nx ? m2 : 0);
        const uint32_t bse = ny ? (nx ? bnn : bnc) : (nx ? bcn : bcc);
        v[k] = ok ? coef(l, lvl + sel8(so, m) + bse) : 0.0;
      }
#pragma unroll
      for (int k = 1; k < 8; ++k) {
        const bool nx = k & 1, ny = k & 2, nz = k & 4;
        if ((!nx || h2) && (!ny || h1) && (!nz || h0))
          sm.X[fidx(P0 + (nz ? 1 : 0), P1 + (ny ? 1 : 0), P2 + (nx ? 1 : 0))] = v[k];
      }
    }
    __syncthreads();
    // 2. restriction, solves, and sub - x with the previous level's values
    tail_restrict(sm.X, sm.A, sm.B, sm.Y, g, ax[0].W, ax[1].W, ax[2].W);
    tail_solve(sm.Y, g, ax);
    for (uint32_t i = tid; i < ncell; i += kTailThreads) sm.Y[i] = sm.Gp[i] - sm.Y[i];
    __syncthreads();
    // 3. the level's values (the forms of rec_interp_body; the coefficients
    //    from step 1)
    auto Gc = [&](uint32_t a, uint32_t b, uint32_t c) { return sm.Y[(a * nc1 + b) * nc2 + c]; };
    const bool last = l == top;
    for (uint32_t e = tid; e < ncell; e += kTailThreads) {
      const uint32_t J2 = e % nc2, rest = e / nc2, J1 = rest % nc1, J0 = rest / nc1;
      const bool h0 = 2 * J0 + 1 < nf0 - 1, h1 = 2 * J1 + 1 < nf1 - 1, h2 = 2 * J2 + 1 < nf2 - 1;
      const uint32_t P0 = cpos32(J0, nf0), P1 = cpos32(J1, nf1), P2 = cpos32(J2, nf2);
      const uint32_t r0 = P0 + (h0 ? 1 : 0), r1 = P1 + (h1 ? 1 : 0), r2 = P2 + (h2 ? 1 : 0);
      const double wz0 = ax[0].wl[r0], wz1 = ax[0].wr[r0], wy0 = ax[1].wl[r1], wy1 = ax[1].wr[r1];
      const double wx0 = ax[2].wl[r2], wx1 = ax[2].wr[r2];
      const uint32_t a1 = h0 ? J0 + 1 : J0, b1 = h1 ? J1 + 1 : J1, c1 = h2 ? J2 + 1 : J2;
      const double c000 = Gc(J0, J1, J2), c001 = Gc(J0, J1, c1), c010 = Gc(J0, b1, J2),
                   c011 = Gc(J0, b1, c1), c100 = Gc(a1, J1, J2), c101 = Gc(a1, J1, c1),
                   c110 = Gc(a1, b1, J2), c111 = Gc(a1, b1, c1);
      const double ix00 = lin2(wx0, c000, wx1, c001), ix01 = lin2(wx0, c010, wx1, c011);
      const double ix10 = lin2(wx0, c100, wx1, c101), ix11 = lin2(wx0, c110, wx1, c111);
      auto cf = [&](uint32_t i0, uint32_t i1, uint32_t i2) { return sm.X[fidx(i0, i1, i2)]; };
      auto put = [&](uint32_t i0, uint32_t i1, uint32_t i2, double v) {
        const uint32_t o = fidx(i0, i1, i2);
        if (last) out[o] = (Tout)v;
        else sm.Gp[o] = v;
      };
      put(P0, P1, P2, c000);
      if (h2) put(P0, P1, P2 + 1, ix00 + cf(P0, P1, P2 + 1));
      if (h1) put(P0, P1 + 1, P2, (lin2(wy0, c000, wy1, c010)) + cf(P0, P1 + 1, P2));
      if (h1 && h2) put(P0, P1 + 1, P2 + 1, (lin2(wy0, ix00, wy1, ix01)) + cf(P0, P1 + 1, P2 + 1));
      if (h0) put(P0 + 1, P1, P2, (lin2(wz0, c000, wz1, c100)) + cf(P0 + 1, P1, P2));
      if (h0 && h2) put(P0 + 1, P1, P2 + 1, (lin2(wz0, ix00, wz1, ix10)) + cf(P0 + 1, P1, P2 + 1));
      if (h0 && h1)
        put(P0 + 1, P1 + 1, P2,
            (lin2(wz0, lin2(wy0, c000, wy1, c010), wz1, lin2(wy0, c100, wy1, c110))) +
                cf(P0 + 1, P1 + 1, P2));
      if (h0 && h1 && h2)
        put(P0 + 1, P1 + 1, P2 + 1,
            (lin2(wz0, lin2(wy0, ix00, wy1, ix01), wz1, lin2(wy0, ix10, wy1, ix11))) +
                cf(P0 + 1, P1 + 1, P2 + 1));
    }
    __syncthreads();
  }
}

template <typename Tin, bool QUANT>
__device__ __forceinline__ void level0_body(const Tin* __restrict__ G0, int64_t m0,
                                            uint16_t* __restrict__ sym, double* __restrict__ raw,
                                            double r, const OutlierBuf& ob, unsigned* status,
                                            uint32_t blk, uint32_t nblk) {
  const int64_t stride = (int64_t)nblk * 256;
  for (int64_t i = (int64_t)blk * 256 + threadIdx.x; i < m0; i += stride) {
    const double c = (double)G0[i];
    if (QUANT) emit_q(i, c, r, sym, ob, status);
    else raw[i] = c;
  }
}

template <typename Tin, bool QUANT>
__global__ __launch_bounds__(256) void k_level0(const Tin* __restrict__ G0, int64_t m0,
                                                 uint16_t* __restrict__ sym,
                                                 double* __restrict__ raw,
                                                 const double* __restrict__ rp,
                                                 const OutlierBuf ob, unsigned* status,
                                                 const unsigned* __restrict__ gate) {
  if (gate_closed(gate)) return;
  level0_body<Tin, QUANT>(G0, m0, sym, raw, rp ? *rp : 0.0, ob, status, blockIdx.x, gridDim.x);
}

template <typename Tout, bool RAW>
__global__ __launch_bounds__(256) void k_rec_level0(const CoeffSrc src, int64_t m0, double q,
                                                     Tout* __restrict__ out) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m0; i += stride)
    out[i] = (Tout)coeff_at<RAW>(src, i, q);
}

// Coarse levels of a decompression dequantised ahead of the level loop: the
// coarse levels hold most escaped values, and a binary search through the
// outlier list per escaped coefficient (a chain of dependent loads) would
// make their small launches latency-bound.  The first kernel writes k q_l
// for every symbol of stream positions [0, m) (0 for the escape symbol), the
// second the escaped values there; the level kernels then read FP64 values.
// Same products as the symbol path, so the results are identical.
__device__ __forceinline__ int level_of(const LevelBins& lb, int64_t pos) {
  int lo = 0, hi = lb.n - 1;  // largest l with off[l] <= pos
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (lb.off[mid] <= pos) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

__global__ __launch_bounds__(256) void k_dequant_prefix(const uint16_t* __restrict__ sym,
                                                         int64_t m, const LevelBins lb,
                                                         double* __restrict__ raw) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += stride) {
    const uint16_t v = sym[i];
    raw[i] = v != 0 ? (double)((int64_t)v - 32768) * lb.q[level_of(lb, i)] : 0.0;
  }
}

__global__ __launch_bounds__(256) void k_dequant_escapes(const uint64_t* __restrict__ opos,
                                                          const int64_t* __restrict__ oval,
                                                          int64_t n_out, int64_t m,
                                                          const LevelBins lb,
                                                          double* __restrict__ raw) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_out; i += stride) {
    const uint64_t p = opos[i];
    if (p < (uint64_t)m) raw[p] = (double)oval[i] * lb.q[level_of(lb, (int64_t)p)];
  }
}

// Small device-to-host transfers: one block copies n bytes into mapped
// pinned host memory (cheaper than a runtime copy for a few hundred bytes).
__global__ __launch_bounds__(256) void k_copy_bytes(uint8_t* __restrict__ dst,
                                                     const uint8_t* __restrict__ src, int n) {
  for (int i = threadIdx.x; i < n; i += 256) dst[i] = src[i];
}

// Up to four word ranges set to zero in one launch (the per-call counters
// and tables a compression starts from).
struct ZeroRanges {
  uint32_t* p[4];
  uint32_t n[4];
};
__global__ __launch_bounds__(256) void k_zero_ranges(const ZeroRanges z) {
  const uint32_t stride = gridDim.x * 256;
  for (int r = 0; r < 4; ++r)
    for (uint32_t i = blockIdx.x * 256 + threadIdx.x; i < z.n[r]; i += stride) z.p[r][i] = 0u;
}

template <typename Tout>
__global__ __launch_bounds__(256) void k_fill(Tout* __restrict__ out, int64_t N, double v) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += stride)
    out[i] = (Tout)v;
}

// ------------------------------------------------------------ batched form
// Each batched kernel finds its array through the launch's block map (or its
// block index, for one block per array), reads the array's pointers and level
// geometry from the job table, and runs the same body as the plain kernel.
// Arrays whose range pass flagged them (constant, empty, non-finite, no
// budget) are skipped.  Step s of the level loop works on level L - s of each
// array; level outputs alternate between the gA (even steps) and gB buffers.
__device__ __forceinline__ bool job_skipped(const Job& J) { return (*J.status & ST_SKIP) != 0; }

__global__ __launch_bounds__(256) void kb_zero(const Job* __restrict__ jobs) {
  const Job& J = jobs[blockIdx.y];
  const uint32_t b = blockIdx.x;
  if (b < 16) {
    for (uint32_t i = threadIdx.x; i < 4096; i += 256) J.hist[b * 4096 + i] = 0;
    return;
  }
  if (threadIdx.x < 4) J.status[threadIdx.x] = 0;
  if (threadIdx.x == 4) *J.n_out = 0;
  unsigned* lw = reinterpret_cast<unsigned*>(J.lay);
  for (uint32_t i = threadIdx.x; i < sizeof(Layout) / 4; i += 256) lw[i] = 0;
}

template <typename T>
__global__ __launch_bounds__(256) void kb_range(const Job* __restrict__ jobs,
                                                 const JobBlock* __restrict__ map, uint32_t nb) {
  if (blockIdx.x >= nb) return;
  const JobBlock jb = map[blockIdx.x];
  const Job& J = jobs[jb.job];
  const T* u = static_cast<const T*>(J.in);
  if ((reinterpret_cast<uintptr_t>(u) & 15) == 0)
    range_partial_body<T, true>(u, J.N, J.part + 4 * jb.local, jb.local, jb.count);
  else
    range_partial_body<T, false>(u, J.N, J.part + 4 * jb.local, jb.local, jb.count);
}

__global__ __launch_bounds__(256) void kb_budget(const Job* __restrict__ jobs) {
  const Job& J = jobs[blockIdx.x];
  if (J.N == 0) {
    if (threadIdx.x == 0) atomicOr(J.status, ST_EMPTY);
    return;
  }
  double r4[4];
  range_final_body(J.part, (int)range_blocks(J.N), J.bud, r4);
  if (threadIdx.x == 0) budget_from_range(J.bi, r4, J.bud, J.status);
}

template <typename Tin, int TZ, int TY, int TX>
__global__ __launch_bounds__(256) void kb_dec_level(const Job* __restrict__ jobs,
                                                     const JobBlock* __restrict__ map,
                                                     uint32_t nb, int step) {
  const uint32_t b = xcd_tile(blockIdx.x, gridDim.x);
  if (b >= nb) return;
  const JobBlock jb = map[b];
  const Job& J = jobs[jb.job];
  if (job_skipped(J)) return;
  const int l = J.L - step;
  const Tin* G = step == 0 ? static_cast<const Tin*>(J.in)
                           : reinterpret_cast<const Tin*>((step & 1) ? J.gA : J.gB);
  double* F = (step & 1) ? J.gB : J.gA;
  const OutlierBuf ob{J.opos, J.oval, J.n_out, J.cap};
  dec_level_body<Tin, TZ, TY, TX, 0>(G, J.geo[l], F, J.sym, nullptr, J.bud[bud_r(J.L, l)], ob,
                                     J.status, jb.local);
}

template <int SEG>
__global__ __launch_bounds__(64) void kb_thomas_rows(const Job* __restrict__ jobs,
                                                      const JobBlock* __restrict__ map,
                                                      uint32_t nb, int step) {
  if (blockIdx.x >= nb) return;
  const JobBlock jb = map[blockIdx.x];
  const Job& J = jobs[jb.job];
  if (job_skipped(J)) return;
  const LevelGeom& g = J.geo[J.L - step];
  const AxisTab& t = g.ax[2];
  thomas_rows_body<SEG>((step & 1) ? J.gB : J.gA, g.nc[0] * g.nc[1], g.nc[2], t.ta, t.tm, t.tc,
                        nullptr, jb.local);
}

template <int AXIS, int U>
__global__ __launch_bounds__(256) void kb_thomas_strided(const Job* __restrict__ jobs,
                                                          const JobBlock* __restrict__ map,
                                                          uint32_t nb, int step) {
  if (blockIdx.x >= nb) return;
  const JobBlock jb = map[blockIdx.x];
  const Job& J = jobs[jb.job];
  if (job_skipped(J)) return;
  const LevelGeom& g = J.geo[J.L - step];
  const AxisTab& t = g.ax[AXIS];
  thomas_strided_body<AXIS, U>((step & 1) ? J.gB : J.gA, g.nc[0], g.nc[1], g.nc[2], t.ta, t.tm,
                               t.tc, nullptr, (int64_t)jb.local * 256 + threadIdx.x);
}

template <int AXIS, int SEG>
__global__ __launch_bounds__(64 * kPartWaves) void kb_thomas_part(const Job* __restrict__ jobs,
                                                                   const JobBlock* __restrict__ map,
                                                                   uint32_t nb, int step) {
  if (blockIdx.x >= nb) return;
  const JobBlock jb = map[blockIdx.x];
  const Job& J = jobs[jb.job];
  if (job_skipped(J)) return;
  const LevelGeom& g = J.geo[J.L - step];
  const AxisTab& t = g.ax[AXIS];
  thomas_part_body<AXIS, SEG>((step & 1) ? J.gB : J.gA, g.nc[0], g.nc[1], g.nc[2], t.ta, t.tm,
                              t.tc, nullptr, jb.local);
}

template <int K>
__global__ __launch_bounds__(64 * kRowScanWaves) void kb_thomas_rowscan(
    const Job* __restrict__ jobs, const JobBlock* __restrict__ map, uint32_t nb, int step) {
  if (blockIdx.x >= nb) return;
  const JobBlock jb = map[blockIdx.x];
  const Job& J = jobs[jb.job];
  if (job_skipped(J)) return;
  const LevelGeom& g = J.geo[J.L - step];
  const AxisTab& t = g.ax[2];
  thomas_rowscan_body<K>((step & 1) ? J.gB : J.gA, g.nc[0] * g.nc[1], g.nc[2], t.ta, t.tm, t.tc,
                         nullptr, jb.local, jb.count);
}

template <typename Tin>
__global__ __launch_bounds__(256) void kb_level0(const Job* __restrict__ jobs,
                                                  const JobBlock* __restrict__ map, uint32_t nb) {
  if (blockIdx.x >= nb) return;
  const JobBlock jb = map[blockIdx.x];
  const Job& J = jobs[jb.job];
  if (job_skipped(J)) return;
  const Tin* G0 = J.L == 0 ? static_cast<const Tin*>(J.in)
                           : reinterpret_cast<const Tin*>(((J.L - 1) & 1) ? J.gB : J.gA);
  const LevelGeom& g = J.geo[0];
  const OutlierBuf ob{J.opos, J.oval, J.n_out, J.cap};
  level0_body<Tin, true>(G0, g.nf[0] * g.nf[1] * g.nf[2], J.sym, nullptr,
                         J.bud[bud_r(J.L, 0)], ob, J.status, jb.local, jb.count);
}

inline unsigned grid_for(int64_t n, int block = 256, int64_t cap = 65536) {
  int64_t b = (n + block - 1) / block;
  if (b < 1) b = 1;
  return (unsigned)(b < cap ? b : cap);
}

struct TileGrid {
  uint32_t n_tiles, tiles_x, tiles_y;
  unsigned grid;
};

TileGrid tile_grid(const LevelGeom& g, int tz, int ty, int tx) {
  TileGrid t;
  t.tiles_x = (uint32_t)((g.nc[2] + tx - 1) / tx);
  t.tiles_y = (uint32_t)((g.nc[1] + ty - 1) / ty);
  const uint32_t tiles_z = (uint32_t)((g.nc[0] + tz - 1) / tz);
  t.n_tiles = t.tiles_x * t.tiles_y * tiles_z;
  t.grid = (t.n_tiles + 7) & ~7u;
  return t;
}

// Blocks of the z-streamed level kernels: (y, x) columns times z segments,
// at most one block per resident slot (four per CU) so that every block runs
// in the same pass; a segment is at least 8 coarse planes long (its 3-plane
// halo then costs at most 3/16 of the planes).
struct StreamGrid {
  int seg;
  uint32_t n_blocks;
  unsigned grid;
};

StreamGrid stream_grid(const LevelGeom& g) {
  const int64_t tiles_x = (g.nc[2] + kStreamSX - 1) / kStreamSX;
  const int64_t tiles_y = (g.nc[1] + kStreamSY - 1) / kStreamSY;
  const int64_t cols = tiles_x * tiles_y;
  const int64_t want = std::max<int64_t>(1, std::min<int64_t>(g.nc[0], 1024 / cols));
  StreamGrid sg;
  sg.seg = (int)std::min<int64_t>(g.nc[0], std::max<int64_t>(8, (g.nc[0] + want - 1) / want));
  const int64_t segs = (g.nc[0] + sg.seg - 1) / sg.seg;
  sg.n_blocks = (uint32_t)(cols * segs);
  sg.grid = (sg.n_blocks + 7) & ~7u;
  return sg;
}

int active_axes(const LevelGeom& g) {
  return (g.bit[0] >= 0) + (g.bit[1] >= 0) + (g.bit[2] >= 0);
}

template <typename Tin, int MODE, int C>
void dec_3(const Tin* Gp, const LevelGeom& g, double* fout, uint16_t* sym, double* raw,
           const double* rp, const OutlierBuf& ob, unsigned* status, const unsigned* gate,
           hipStream_t s) {
  constexpr TileShape ts = sizeof(Tin) == 4 ? kDecTiles3F32[C] : kDecTiles3F64[C];
  const TileGrid t = tile_grid(g, ts.z, ts.y, ts.x);
  hipLaunchKernelGGL((k_dec_level<Tin, ts.z, ts.y, ts.x, MODE>), dim3(t.grid), dim3(256), 0, s,
                     Gp, g, fout, sym, raw, rp, ob, status, gate, t.n_tiles);
}

template <typename Tin, int MODE>
void dec_dispatch(const void* G, const LevelGeom& g, double* fout, uint16_t* sym, double* raw,
                  const double* rp, const OutlierBuf& ob, unsigned* status,
                  const unsigned* gate, hipStream_t s, int cand = 0) {
  const Tin* Gp = static_cast<const Tin*>(G);
  const int D = active_axes(g);
  if (D == 3 && MODE != 2 && cand == 0 && g.nf[0] * g.nf[1] * g.nf[2] >= kStreamMinPoints) {
    const StreamGrid sg = stream_grid(g);
    hipLaunchKernelGGL((k_dec_stream<Tin, MODE == 0>), dim3(sg.grid), dim3(256), 0, s, Gp, g, fout,
                       sym, raw, rp, ob, status, gate, sg.seg, sg.n_blocks);
    return;
  }
  if (D == 3) {
    if (MODE == 2) cand = 0;
    switch (cand) {
      case 1: dec_3<Tin, MODE, 1>(Gp, g, fout, sym, raw, rp, ob, status, gate, s); break;
      case 2: dec_3<Tin, MODE, 2>(Gp, g, fout, sym, raw, rp, ob, status, gate, s); break;
      case 3: dec_3<Tin, MODE, 3>(Gp, g, fout, sym, raw, rp, ob, status, gate, s); break;
      default: dec_3<Tin, MODE, 0>(Gp, g, fout, sym, raw, rp, ob, status, gate, s);
    }
  } else if (D == 2) {
    constexpr TileShape ts = sizeof(Tin) == 4 ? kDecTile2F32 : kDecTile2F64;
    const TileGrid t = tile_grid(g, ts.z, ts.y, ts.x);
    hipLaunchKernelGGL((k_dec_level<Tin, ts.z, ts.y, ts.x, MODE>), dim3(t.grid), dim3(256), 0, s,
                       Gp, g, fout, sym, raw, rp, ob, status, gate, t.n_tiles);
  } else {
    constexpr TileShape ts = kDecTile1;
    const TileGrid t = tile_grid(g, ts.z, ts.y, ts.x);
    hipLaunchKernelGGL((k_dec_level<Tin, ts.z, ts.y, ts.x, MODE>), dim3(t.grid), dim3(256), 0, s,
                       Gp, g, fout, sym, raw, rp, ob, status, gate, t.n_tiles);
  }
}

template <bool RAW>
void rec_restrict_dispatch(const LevelGeom& g, const CoeffSrc& src, double q, double* fout,
                           hipStream_t s) {
  const int D = active_axes(g);
  if (D == 3 && g.nf[0] * g.nf[1] * g.nf[2] >= kRecStreamMinPoints) {
    const StreamGrid sg = stream_grid(g);
    hipLaunchKernelGGL((k_rec_stream<RAW>), dim3(sg.grid), dim3(256), 0, s, g, src, q, fout,
                       sg.seg, sg.n_blocks);
    return;
  }
  if (D == 3) {
    const TileGrid t = tile_grid(g, 4, 8, 8);
    hipLaunchKernelGGL((k_rec_restrict<4, 8, 8, RAW>), dim3(t.grid), dim3(256), 0, s, g, src, q,
                       fout, t.n_tiles);
  } else if (D == 2) {
    const TileGrid t = tile_grid(g, 1, 8, 32);
    hipLaunchKernelGGL((k_rec_restrict<1, 8, 32, RAW>), dim3(t.grid), dim3(256), 0, s, g, src, q,
                       fout, t.n_tiles);
  } else {
    const TileGrid t = tile_grid(g, 1, 1, 256);
    hipLaunchKernelGGL((k_rec_restrict<1, 1, 256, RAW>), dim3(t.grid), dim3(256), 0, s, g, src,
                       q, fout, t.n_tiles);
  }
}

template <typename Tout, int SRC>
void rec_interp_dispatch(const double* Gc, const LevelGeom& g, const CoeffSrc& src, double q,
                         Tout* out, hipStream_t s) {
  const int D = active_axes(g);
  if (D == 3) {
    const TileGrid t = tile_grid(g, 4, 8, 16);
    hipLaunchKernelGGL((k_rec_interp<Tout, 4, 8, 16, SRC>), dim3(t.grid), dim3(256), 0, s, Gc, g,
                       src, q, out, t.n_tiles);
  } else if (D == 2) {
    const TileGrid t = tile_grid(g, 1, 16, 32);
    hipLaunchKernelGGL((k_rec_interp<Tout, 1, 16, 32, SRC>), dim3(t.grid), dim3(256), 0, s, Gc, g,
                       src, q, out, t.n_tiles);
  } else {
    const TileGrid t = tile_grid(g, 1, 1, 256);
    hipLaunchKernelGGL((k_rec_interp<Tout, 1, 1, 256, SRC>), dim3(t.grid), dim3(256), 0, s, Gc,
                       g, src, q, out, t.n_tiles);
  }
}

}  // namespace

void launch_range(const void* u, mgc_dtype dt, int64_t N, double* part, const BudgetIn& b,
                  double* bud, unsigned* status, hipStream_t s) {
  const bool vec = (reinterpret_cast<uintptr_t>(u) & 15) == 0;
  const unsigned nb = range_blocks(N);
  if (dt == MGC_F32) {
    if (vec) hipLaunchKernelGGL((k_range_partial<float, true>), dim3(nb), dim3(256), 0, s,
                                static_cast<const float*>(u), N, part);
    else hipLaunchKernelGGL((k_range_partial<float, false>), dim3(nb), dim3(256), 0, s,
                            static_cast<const float*>(u), N, part);
  } else {
    if (vec) hipLaunchKernelGGL((k_range_partial<double, true>), dim3(nb), dim3(256), 0, s,
                                static_cast<const double*>(u), N, part);
    else hipLaunchKernelGGL((k_range_partial<double, false>), dim3(nb), dim3(256), 0, s,
                            static_cast<const double*>(u), N, part);
  }
  hipLaunchKernelGGL(k_budget, dim3(1), dim3(256), 0, s, part, (int)nb, b, bud, status);
}

void launch_dec_level(const void* G, bool g_is_f32, const LevelGeom& g, double* fout,
                      uint16_t* sym, double* raw, const double* rp, const OutlierBuf& ob,
                      unsigned* status, const unsigned* gate, hipStream_t s, int cand) {
  if (sym) {
    if (g_is_f32) dec_dispatch<float, 0>(G, g, fout, sym, raw, rp, ob, status, gate, s, cand);
    else dec_dispatch<double, 0>(G, g, fout, sym, raw, rp, ob, status, gate, s, cand);
  } else {
    if (g_is_f32) dec_dispatch<float, 1>(G, g, fout, sym, raw, rp, ob, status, gate, s, cand);
    else dec_dispatch<double, 1>(G, g, fout, sym, raw, rp, ob, status, gate, s, cand);
  }
}

namespace {
template <int C>
void thomas_c(int axis, double* x, const int64_t nc[3], const AxisTab& t, const double* sub,
              hipStream_t s) {
  if (axis == 2) {
    const int64_t rows = nc[0] * nc[1];
    hipLaunchKernelGGL(k_thomas_rows<kThomasSeg[C]>, dim3((unsigned)((rows + 63) / 64)), dim3(64),
                       0, s, x, rows, nc[2], t.ta, t.tm, t.tc, sub);
    return;
  }
  const int64_t lines = axis == 1 ? nc[0] * nc[2] : nc[1] * nc[2];
  const unsigned blocks = (unsigned)((lines + 255) / 256);
  if (axis == 1)
    hipLaunchKernelGGL((k_thomas_strided<1, kThomasU[C]>), dim3(blocks), dim3(256), 0, s, x,
                       nc[0], nc[1], nc[2], t.ta, t.tm, t.tc, sub);
  else
    hipLaunchKernelGGL((k_thomas_strided<0, kThomasU[C]>), dim3(blocks), dim3(256), 0, s, x,
                       nc[0], nc[1], nc[2], t.ta, t.tm, t.tc, sub);
}
}  // namespace

namespace {
template <int TILES, int AXIS>
void thomas_tiles_axis(double* x, const int64_t nc[3], const AxisTab& t, const double* sub,
                       hipStream_t s) {
  static bool attr = false;
  if (!attr) {
    MGC_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(k_thomas_tile<TILES, AXIS>),
                                hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)thomas_tile_lds(TILES == 4 ? kThomasTile4MaxL
                                                                : kThomasTile2MaxL, TILES)));
    attr = true;
  }
  int64_t tiles;
  if (AXIS == 2) tiles = (nc[0] * nc[1] + kTileLines - 1) / kTileLines;
  else if (AXIS == 1) tiles = nc[0] * ((nc[2] + kTileLines - 1) / kTileLines);
  else tiles = (nc[1] * nc[2] + kTileLines - 1) / kTileLines;
  const int64_t blocks = (tiles + TILES - 1) / TILES;
  hipLaunchKernelGGL((k_thomas_tile<TILES, AXIS>), dim3((unsigned)blocks), dim3(64 * TILES),
                     thomas_tile_lds(nc[AXIS], TILES), s, x, nc[0], nc[1], nc[2], t.ta, t.tm, t.tc,
                     sub);
}
template <int TILES>
void thomas_tiles(int axis, double* x, const int64_t nc[3], const AxisTab& t, const double* sub,
                  hipStream_t s) {
  if (axis == 2) thomas_tiles_axis<TILES, 2>(x, nc, t, sub, s);
  else if (axis == 1) thomas_tiles_axis<TILES, 1>(x, nc, t, sub, s);
  else thomas_tiles_axis<TILES, 0>(x, nc, t, sub, s);
}
}  // namespace

namespace {
template <int K>
void thomas_rowscan(double* x, const int64_t nc[3], const AxisTab& t, const double* sub,
                    hipStream_t s) {
  const int64_t rows = nc[0] * nc[1];
  const int64_t blocks = std::min<int64_t>((rows + kRowScanWaves - 1) / kRowScanWaves, 4096);
  hipLaunchKernelGGL(k_thomas_rowscan<K>, dim3((unsigned)blocks), dim3(64 * kRowScanWaves), 0, s,
                     x, rows, nc[2], t.ta, t.tm, t.tc, sub);
}
template <int AXIS, int SEG>
void thomas_part_axis(double* x, const int64_t nc[3], const AxisTab& t, const double* sub,
                      hipStream_t s) {
  const int64_t w = (nc[AXIS] + SEG - 1) / SEG;
  const int64_t lines = AXIS == 1 ? nc[0] * nc[2] : nc[1] * nc[2];
  const uint32_t nblk = (uint32_t)((lines + 63) / 64);
  hipLaunchKernelGGL((k_thomas_part<AXIS, SEG>), dim3((nblk + 7u) & ~7u), dim3((unsigned)(64 * w)),
                     0, s, x, nc[0], nc[1], nc[2], t.ta, t.tm, t.tc, sub, nblk);
}
// Partitioned sweeps of class c (thomas_part_class).
void thomas_part(int axis, int c, double* x, const int64_t nc[3], const AxisTab& t,
                 const double* sub, hipStream_t s) {
  if (axis == 2) {
    const int64_t len = nc[2];
    if (len <= 128) thomas_rowscan<2>(x, nc, t, sub, s);
    else if (len <= 256) thomas_rowscan<4>(x, nc, t, sub, s);
    else if (len <= 320) thomas_rowscan<5>(x, nc, t, sub, s);
    else if (len <= 512) thomas_rowscan<8>(x, nc, t, sub, s);
    else thomas_rowscan<16>(x, nc, t, sub, s);
    return;
  }
  if (axis == 1) {
    if (c == kPart40) thomas_part_axis<1, 40>(x, nc, t, sub, s);
    else thomas_part_axis<1, 64>(x, nc, t, sub, s);
  } else {
    if (c == kPart40) thomas_part_axis<0, 40>(x, nc, t, sub, s);
    else thomas_part_axis<0, 64>(x, nc, t, sub, s);
  }
}
}  // namespace

int thomas_part_class(int axis, int64_t len) {
  if (axis == 2) return len <= 1024 ? kPartScan : kPartNone;
  if (len <= 40 * kPartWaves) return kPart40;
  if (len <= 64 * kPartWaves) return kPart64;
  return kPartNone;
}

void launch_thomas(int axis, double* x, const int64_t nc[3], const AxisTab& t,
                   const double* sub, hipStream_t s, int cand) {
  const int64_t L = nc[axis];
  if (cand == 0) {
    const int c = thomas_part_class(axis, L);
    if (c != kPartNone) {
      thomas_part(axis, c, x, nc, t, sub, s);
      return;
    }
  }
  if (cand == 0 && L <= kThomasTile2MaxL && nc[0] * nc[1] * nc[2] <= kThomasTilePoints) {
    if (L <= kThomasTile4MaxL) thomas_tiles<4>(axis, x, nc, t, sub, s);
    else thomas_tiles<2>(axis, x, nc, t, sub, s);
    return;
  }
  switch (cand) {
    case 1: thomas_c<1>(axis, x, nc, t, sub, s); break;
    case 2: thomas_c<2>(axis, x, nc, t, sub, s); break;
    default: thomas_c<0>(axis, x, nc, t, sub, s);
  }
}

bool thomas_grid_fits(const LevelGeom& g) {
  if (g.nc[0] * g.nc[1] * g.nc[2] > kThomasGridMax) return false;
  // One thread per line: long lines would serialise the whole launch.
  for (int k = 0; k < 3; ++k)
    if (g.bit[k] >= 0 && g.nc[k] > kThomasGridMaxLine) return false;
  return true;
}

void launch_thomas_grid(double* x, const LevelGeom& g, const double* sub, hipStream_t s) {
  const int64_t n = g.nc[0] * g.nc[1] * g.nc[2];
  if (n > kThomasGridMax) throw std::logic_error("launch_thomas_grid: grid exceeds LDS");
  static bool attr = false;
  if (!attr) {
    MGC_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(k_thomas_grid),
                                hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)(kThomasGridMax * sizeof(double))));
    attr = true;
  }
  Thomas3Args a;
  for (int k = 0; k < 3; ++k) {
    a.ta[k] = g.ax[k].ta;
    a.tm[k] = g.ax[k].tm;
    a.tc[k] = g.ax[k].tc;
    a.active[k] = g.bit[k] >= 0;
  }
  hipLaunchKernelGGL(k_thomas_grid, dim3(1), dim3(kThomasGridThreads), (size_t)n * sizeof(double),
                     s, x, g.nc[0], g.nc[1], g.nc[2], a, sub);
}

void launch_level0(const void* G0, bool g_is_f32, int64_t m0, uint16_t* sym, double* raw,
                   const double* rp, const OutlierBuf& ob, unsigned* status,
                   const unsigned* gate, hipStream_t s) {
  const unsigned b = grid_for(m0);
  if (g_is_f32) {
    if (sym) hipLaunchKernelGGL((k_level0<float, true>), dim3(b), dim3(256), 0, s,
                                static_cast<const float*>(G0), m0, sym, raw, rp, ob, status, gate);
    else hipLaunchKernelGGL((k_level0<float, false>), dim3(b), dim3(256), 0, s,
                            static_cast<const float*>(G0), m0, sym, raw, rp, ob, status, gate);
  } else {
    if (sym) hipLaunchKernelGGL((k_level0<double, true>), dim3(b), dim3(256), 0, s,
                                static_cast<const double*>(G0), m0, sym, raw, rp, ob, status, gate);
    else hipLaunchKernelGGL((k_level0<double, false>), dim3(b), dim3(256), 0, s,
                            static_cast<const double*>(G0), m0, sym, raw, rp, ob, status, gate);
  }
}

void launch_rec_restrict(const LevelGeom& g, const CoeffSrc& src, double q, double* fout,
                         hipStream_t s) {
  if (src.raw) rec_restrict_dispatch<true>(g, src, q, fout, s);
  else rec_restrict_dispatch<false>(g, src, q, fout, s);
}

void launch_rec_interp(const double* Gc, const LevelGeom& g, const CoeffSrc& src, double q,
                       void* out, bool out_f32, hipStream_t s) {
  if (out_f32) {
    if (src.raw) rec_interp_dispatch<float, 1>(Gc, g, src, q, static_cast<float*>(out), s);
    else rec_interp_dispatch<float, 0>(Gc, g, src, q, static_cast<float*>(out), s);
  } else {
    if (src.raw) rec_interp_dispatch<double, 1>(Gc, g, src, q, static_cast<double*>(out), s);
    else rec_interp_dispatch<double, 0>(Gc, g, src, q, static_cast<double*>(out), s);
  }
}

void launch_adj_restrict(const double* gl, const LevelGeom& g, double* Gc, double* Gc_copy,
                         hipStream_t s) {
  dec_dispatch<double, 2>(gl, g, Gc, nullptr, Gc_copy, nullptr,
                          OutlierBuf{nullptr, nullptr, nullptr, 0}, nullptr, nullptr, s);
}

void launch_prolong(const double* v, const LevelGeom& g, double* out, hipStream_t s) {
  const CoeffSrc none{nullptr, nullptr, nullptr, nullptr, 0};
  rec_interp_dispatch<double, 2>(v, g, none, 0.0, out, s);
}

void launch_adj_mass(const double* Pv, const double* gl, const LevelGeom& g, double* cbar,
                     hipStream_t s) {
  const int64_t rows = g.nf[0] * g.nf[1];
  const dim3 grid((unsigned)((g.nf[2] + 255) / 256), (unsigned)(rows < 65535 ? rows : 65535));
  hipLaunchKernelGGL(k_adj_mass, grid, dim3(256), 0, s, Pv, gl, g, cbar);
}

void launch_dequant_prefix(const CoeffSrc& src, int64_t m, const LevelBins& lb, double* raw,
                           hipStream_t s) {
  if (m <= 0) return;
  const unsigned b = (unsigned)std::min<int64_t>((m + 255) / 256, 4096);
  hipLaunchKernelGGL(k_dequant_prefix, dim3(b), dim3(256), 0, s, src.sym, m, lb, raw);
  if (src.n_out > 0) {
    const unsigned bo = (unsigned)std::min<int64_t>((src.n_out + 255) / 256, 2048);
    hipLaunchKernelGGL(k_dequant_escapes, dim3(bo), dim3(256), 0, s, src.opos, src.oval,
                       src.n_out, m, lb, raw);
  }
}

bool tail_level_fits(const LevelGeom& g) {
  const int64_t nf = g.nf[0] * g.nf[1] * g.nf[2], nc = g.nc[0] * g.nc[1] * g.nc[2];
  if (nf > kTailMax || nc > kTailCoarse || g.nf[0] * g.nc[1] * g.nc[2] > kTailCoarse) return false;
  for (int k = 0; k < 3; ++k)
    if (g.bit[k] >= 0 && g.nc[k] > kTailLine) return false;
  return true;
}
size_t tail_max_table() { return kTailTab; }

void launch_dec_tail(const void* G, bool g_is_f32, const LevelGeom* d_geo, int top,
                     const TailTabArgs& tt, uint16_t* sym, double* raw, const double* rdev,
                     const OutlierBuf& ob, unsigned* status, const unsigned* gate, hipStream_t s) {
  if (top < 1 || top >= kTailLevels || tt.n > (uint32_t)kTailTab)
    throw std::logic_error("launch_dec_tail: levels exceed the LDS tables");
  const dim3 b(1), t(kTailThreads);
  if (g_is_f32) {
    if (sym) hipLaunchKernelGGL((k_dec_tail<float, true>), b, t, 0, s, static_cast<const float*>(G),
                                d_geo, top, tt, sym, raw, rdev, ob, status, gate);
    else hipLaunchKernelGGL((k_dec_tail<float, false>), b, t, 0, s, static_cast<const float*>(G),
                            d_geo, top, tt, sym, raw, rdev, ob, status, gate);
  } else {
    if (sym) hipLaunchKernelGGL((k_dec_tail<double, true>), b, t, 0, s,
                                static_cast<const double*>(G), d_geo, top, tt, sym, raw, rdev, ob,
                                status, gate);
    else hipLaunchKernelGGL((k_dec_tail<double, false>), b, t, 0, s,
                            static_cast<const double*>(G), d_geo, top, tt, sym, raw, rdev, ob,
                            status, gate);
  }
}

void launch_rec_tail(const CoeffSrc& src, const CoeffSrc& coarse, int coarse_top,
                     const double* q, const LevelGeom* d_geo, int top, const TailTabArgs& tt,
                     void* out, bool out_f32, hipStream_t s) {
  if (top < 1 || top >= kTailLevels || tt.n > (uint32_t)kTailTab)
    throw std::logic_error("launch_rec_tail: levels exceed the LDS tables");
  TailQ tq{};
  for (int l = 0; l <= top; ++l) tq.q[l] = q[l];
  const dim3 b(1), t(kTailThreads);
  if (out_f32)
    hipLaunchKernelGGL((k_rec_tail<float>), b, t, 0, s, src, coarse, coarse_top, tq, d_geo, top,
                       tt, static_cast<float*>(out));
  else
    hipLaunchKernelGGL((k_rec_tail<double>), b, t, 0, s, src, coarse, coarse_top, tq, d_geo, top,
                       tt, static_cast<double*>(out));
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

// ---- batched launchers
void launch_b_zero(const Job* jobs, int n, hipStream_t s) {
  hipLaunchKernelGGL(kb_zero, dim3(17, (unsigned)n), dim3(256), 0, s, jobs);
}

void launch_b_range(const Job* jobs, const JobBlock* map, uint32_t nb, bool f32, hipStream_t s) {
  if (f32) hipLaunchKernelGGL(kb_range<float>, dim3(nb), dim3(256), 0, s, jobs, map, nb);
  else hipLaunchKernelGGL(kb_range<double>, dim3(nb), dim3(256), 0, s, jobs, map, nb);
}

void launch_b_budget(const Job* jobs, int n, hipStream_t s) {
  hipLaunchKernelGGL(kb_budget, dim3((unsigned)n), dim3(256), 0, s, jobs);
}

namespace {
template <typename Tin, int TZ, int TY, int TX>
void b_dec(const Job* jobs, const JobBlock* map, uint32_t nb, int step, hipStream_t s) {
  const unsigned grid = (nb + 7) & ~7u;
  hipLaunchKernelGGL((kb_dec_level<Tin, TZ, TY, TX>), dim3(grid), dim3(256), 0, s, jobs, map, nb,
                     step);
}
template <typename Tin, int C>
void b_dec_3(const Job* jobs, const JobBlock* map, uint32_t nb, int step, hipStream_t s) {
  constexpr TileShape t = sizeof(Tin) == 4 ? kDecTiles3F32[C] : kDecTiles3F64[C];
  b_dec<Tin, t.z, t.y, t.x>(jobs, map, nb, step, s);
}
template <typename Tin>
void b_dec_cand(const Job* jobs, const JobBlock* map, uint32_t nb, int step, int D, int cand,
                hipStream_t s) {
  if (D == 3) {
    switch (cand) {
      case 1: b_dec_3<Tin, 1>(jobs, map, nb, step, s); break;
      case 2: b_dec_3<Tin, 2>(jobs, map, nb, step, s); break;
      case 3: b_dec_3<Tin, 3>(jobs, map, nb, step, s); break;
      default: b_dec_3<Tin, 0>(jobs, map, nb, step, s);
    }
  } else if (D == 2) {
    constexpr TileShape t = sizeof(Tin) == 4 ? kDecTile2F32 : kDecTile2F64;
    b_dec<Tin, t.z, t.y, t.x>(jobs, map, nb, step, s);
  } else {
    b_dec<Tin, kDecTile1.z, kDecTile1.y, kDecTile1.x>(jobs, map, nb, step, s);
  }
}
}  // namespace

void launch_b_dec_level(const Job* jobs, const JobBlock* map, uint32_t nb, int step, int D,
                        bool f32, int cand, hipStream_t s) {
  if (f32) b_dec_cand<float>(jobs, map, nb, step, D, cand, s);
  else b_dec_cand<double>(jobs, map, nb, step, D, cand, s);
}

namespace {
template <int C>
void b_thomas(int axis, const Job* jobs, const JobBlock* map, uint32_t nb, int step,
              hipStream_t s) {
  if (axis == 2)
    hipLaunchKernelGGL(kb_thomas_rows<kThomasSeg[C]>, dim3(nb), dim3(64), 0, s, jobs, map, nb,
                       step);
  else if (axis == 1)
    hipLaunchKernelGGL((kb_thomas_strided<1, kThomasU[C]>), dim3(nb), dim3(256), 0, s, jobs, map,
                       nb, step);
  else
    hipLaunchKernelGGL((kb_thomas_strided<0, kThomasU[C]>), dim3(nb), dim3(256), 0, s, jobs, map,
                       nb, step);
}
}  // namespace

void launch_b_thomas(int axis, const Job* jobs, const JobBlock* map, uint32_t nb, int step,
                     int cand, hipStream_t s) {
  switch (cand) {
    case 1: b_thomas<1>(axis, jobs, map, nb, step, s); break;
    case 2: b_thomas<2>(axis, jobs, map, nb, step, s); break;
    default: b_thomas<0>(axis, jobs, map, nb, step, s);
  }
}

void launch_b_thomas_part(int axis, int c, int waves, const Job* jobs, const JobBlock* map,
                          uint32_t nb, int step, hipStream_t s) {
  if (waves < 1 || waves > kPartWaves) throw std::logic_error("launch_b_thomas_part: waves");
  const dim3 blk((unsigned)(64 * waves));
  if (axis == 2) {
    if (c == kPartScanLong)
      hipLaunchKernelGGL(kb_thomas_rowscan<16>, dim3(nb), dim3(64 * kRowScanWaves), 0, s, jobs,
                         map, nb, step);
    else
      hipLaunchKernelGGL(kb_thomas_rowscan<4>, dim3(nb), dim3(64 * kRowScanWaves), 0, s, jobs,
                         map, nb, step);
  } else if (axis == 1) {
    if (c == kPart40)
      hipLaunchKernelGGL((kb_thomas_part<1, 40>), dim3(nb), blk, 0, s, jobs, map, nb, step);
    else hipLaunchKernelGGL((kb_thomas_part<1, 64>), dim3(nb), blk, 0, s, jobs, map, nb, step);
  } else {
    if (c == kPart40)
      hipLaunchKernelGGL((kb_thomas_part<0, 40>), dim3(nb), blk, 0, s, jobs, map, nb, step);
    else hipLaunchKernelGGL((kb_thomas_part<0, 64>), dim3(nb), blk, 0, s, jobs, map, nb, step);
  }
}

void launch_b_level0(const Job* jobs, const JobBlock* map, uint32_t nb, bool f32,
                     hipStream_t s) {
  if (f32) hipLaunchKernelGGL(kb_level0<float>, dim3(nb), dim3(256), 0, s, jobs, map, nb);
  else hipLaunchKernelGGL(kb_level0<double>, dim3(nb), dim3(256), 0, s, jobs, map, nb);
}

void launch_copy_bytes(void* dst, const void* src, size_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_copy_bytes, dim3(1), dim3(256), 0, s, static_cast<uint8_t*>(dst),
                     static_cast<const uint8_t*>(src), (int)n);
}

void launch_zero_words(void* const* ptrs, const size_t* bytes, int n, hipStream_t s) {
  if (n < 1 || n > 4) throw std::logic_error("launch_zero_words: one to four ranges");
  ZeroRanges z{};
  uint32_t most = 0;
  for (int r = 0; r < n; ++r) {
    if (bytes[r] % 4 != 0 || bytes[r] / 4 > 0xFFFFFFFFull ||
        (reinterpret_cast<uintptr_t>(ptrs[r]) & 3) != 0)
      throw std::logic_error("launch_zero_words: ranges of whole aligned words");
    z.p[r] = static_cast<uint32_t*>(ptrs[r]);
    z.n[r] = (uint32_t)(bytes[r] / 4);
    most = std::max(most, z.n[r]);
  }
  const unsigned blocks = std::max(1u, std::min(64u, (most + 1023) / 1024));
  hipLaunchKernelGGL(k_zero_ranges, dim3(blocks), dim3(256), 0, s, z);
}

void launch_fill(void* out, bool out_f32, int64_t N, double v, hipStream_t s) {
  if (N <= 0) return;
  const unsigned b = grid_for(N);
  if (out_f32) hipLaunchKernelGGL(k_fill<float>, dim3(b), dim3(256), 0, s, static_cast<float*>(out), N, v);
  else hipLaunchKernelGGL(k_fill<double>, dim3(b), dim3(256), 0, s, static_cast<double*>(out), N, v);
}

}  // namespace mgc
