// C-ABI entry points and host orchestration of the kernels.
//
// compress runs Algorithm 1 of the paper end to end on one stream: a range
// pre-pass (min, max, sum of squares) whose last block turns the relative
// bound into the per-level bins on the device, then for each level from the
// finest the fused lerp/quantise/mass_trans kernel and the tridiagonal
// sweeps, the coarsest block, and the Huffman stage of Algorithm 2, ending
// with a header kernel that writes the stream length and status to device
// memory.  Nothing is read back to the host, so the call is asynchronous and
// can be captured into a graph; inputs the range pass flags (constant,
// NaN/Inf, no budget) close the gate of every later kernel.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <vector>

#include "host.hpp"

#pragma clang fp contract(off)

namespace mgc {

thread_local std::string g_err;
void set_error(const std::string& msg) { g_err = msg; }
void fail(mgc_status st, const std::string& msg) {
  g_err = msg;
  throw Fail{st};
}

StageScope::StageScope(Profiler* prof, const char* name, hipStream_t stream)
    : p(prof && prof->enabled ? prof : nullptr), slot(-1), s(stream), a(nullptr) {
  if (!p) return;
  slot = p->slot(name);
  a = p->get();
  MGC_HIP(hipEventRecord(a, s));
}
StageScope::~StageScope() {
  if (!p) return;
  hipEvent_t b = p->get();
  if (hipEventRecord(b, s) == hipSuccess) p->pending.push_back({slot, a, b});
}

uint64_t default_outlier_cap(int64_t N) {
  return std::max<uint64_t>(65536, (uint64_t)N / 16);
}

int key_bits(int64_t N) {
  if (N <= 1) return 1;
  uint64_t v = (uint64_t)(N - 1);
  int b = 0;
  while (v) {
    ++b;
    v >>= 1;
  }
  return b;
}

Header make_header(const Plan& p, int ndim, const uint64_t* shape, mgc_dtype dtype,
                   double bound, mgc_norm norm, mgc_mode mode) {
  Header h{};
  h.magic = kMagic;
  h.version = kVersion;
  h.dtype = (uint8_t)dtype;
  h.norm = (uint8_t)norm;
  h.mode = (uint8_t)mode;
  h.ndim = (uint8_t)ndim;
  h.D = (uint8_t)p.D;
  h.L = (uint32_t)p.L;
  for (int d = 0; d < ndim; ++d) h.shape[d] = shape[d];
  h.bound = bound;
  h.S = kDict;
  h.C = kChunk;
  h.N = (uint64_t)p.N;
  h.n_chunks = (p.N + kChunk - 1) / kChunk;
  if (p.N == 0) {
    h.flags = FLAG_EMPTY;
    h.n_chunks = 0;
    h.D = 0;  // number of axes longer than 1, as given
    for (int d = 0; d < ndim; ++d) h.D += shape[d] > 1;
  }
  return h;
}

CompressWs carve_compress(Carver& c, const Plan& p, uint64_t cap) {
  CompressWs w;
  const int64_t n_coarse = p.L >= 1 ? p.points(p.L - 1) : 1;
  const int64_t n_chunks = (p.N + kChunk - 1) / kChunk;
  w.sym = c.take<uint16_t>(std::max<int64_t>(p.N, 1));
  w.gA = c.take<double>(n_coarse);
  w.gB = c.take<double>(n_coarse);
  w.part = c.take<double>(4 * kRangeBlocks);
  w.bud = c.take<double>(kBudDoubles);
  w.status = c.take<unsigned>(4);
  w.n_out = c.take<unsigned long long>(1);
  w.lay = c.take<Layout>(1);
  w.hist = c.take<unsigned>(kDict);
  w.code = c.take<uint32_t>(kDict);
  w.clen = c.take<uint8_t>(kDict);
  w.cbs = c.take<uint8_t>(codebook_scratch_bytes());
  w.cw = c.take<uint32_t>(chunk_words_len(n_chunks));
  w.opos = c.take<uint32_t>(cap);
  w.oval = c.take<int64_t>(cap);
  w.okA = c.take<uint32_t>(cap);
  w.ovA = c.take<uint32_t>(cap);
  w.okB = c.take<uint32_t>(cap);
  w.ovB = c.take<uint32_t>(cap);
  w.info = c.take<unsigned long long>(4);
  w.zc = c.take<uint32_t>(std::max<int64_t>(n_chunks, 1));
  w.zpre = c.take<uint32_t>(std::max<int64_t>(n_chunks, 1));
  w.zsums = c.take<uint32_t>(kEscSumsMax);
  w.zl = c.take<uint32_t>(64 * std::max<int64_t>(n_chunks, 1));
  return w;
}

size_t max_stream_bytes(const Plan& p, uint64_t cap) {
  const uint64_t n_chunks = (p.N + kChunk - 1) / kChunk;
  return kHeaderBytes + 8 * (p.L + 1) + pad8(3 * kDict) + 8 * (n_chunks + 1) + 16 * cap +
         4 * ((uint64_t)p.N + n_chunks) + 8;
}

struct DecompressWs {
  uint16_t* sym;
  double *gA, *gB;
  double* coarse;  // dequantised coefficients of levels 0 .. L-2
  void* tables;
  unsigned* status;
};

DecompressWs carve_decompress(Carver& c, const Plan& p) {
  DecompressWs w;
  const int64_t n_coarse = p.L >= 1 ? p.points(p.L - 1) : 1;
  w.sym = c.take<uint16_t>(std::max<int64_t>(p.N, 1));
  w.gA = c.take<double>(n_coarse);
  w.gB = c.take<double>(n_coarse);
  w.tables = c.take<uint8_t>(decode_tables_bytes());
  w.status = c.take<unsigned>(4);
  w.coarse = p.L >= 2 ? c.take<double>(p.points(p.L - 2)) : nullptr;
  return w;
}

size_t decompress_ws_bytes(const Plan& p) {
  Carver c(nullptr);
  carve_decompress(c, p);
  return c.off;
}

size_t dtype_size(mgc_dtype d) { return d == MGC_F32 ? 4 : 8; }

// Parses and validates a stream header held in host memory.
void parse_header(const uint8_t* b, size_t n, Header* h, std::vector<double>* q) {
  if (n < (size_t)kHeaderBytes) fail(MGC_EFORMAT, "stream shorter than its header");
  std::memcpy(h, b, kHeaderBytes);
  if (h->magic != kMagic || h->version != kVersion) fail(MGC_EFORMAT, "bad magic or version");
  if (h->dtype > 1 || h->norm > 1 || h->mode > 1 || h->ndim < 1 || h->ndim > 3 ||
      h->L > (uint32_t)kMaxLevels || (h->flags & ~3u))
    fail(MGC_EFORMAT, "bad header field");
  if (n < (size_t)kHeaderBytes + 8 * (h->L + 1)) fail(MGC_EFORMAT, "truncated bins");
  q->resize(h->L + 1);
  std::memcpy(q->data(), b + kHeaderBytes, 8 * (h->L + 1));
}

}  // namespace mgc

using namespace mgc;

namespace mgc {
void check_ctx(mgc_ctx ctx) {
  if (!ctx) fail(MGC_EINVAL, "null context");
  MGC_HIP(hipSetDevice(ctx->device));
}

const Plan& get_plan(mgc_ctx ctx, int ndim, const uint64_t* shape) {
  if (ndim < 1) fail(MGC_EINVAL, "ndim must be at least 1");
  if (ndim > 3) fail(MGC_EUNSUPPORTED, "ndim above 3 is not supported");
  std::vector<uint64_t> key(shape, shape + ndim);
  key.insert(key.begin(), (uint64_t)ndim);
  auto it = ctx->plans.find(key);
  if (it != ctx->plans.end()) return it->second;
  Plan p = build_plan(ndim, shape);
  upload_plan(p);
  return ctx->plans.emplace(key, std::move(p)).first->second;
}
}  // namespace mgc

namespace {

hipStream_t as_stream(void* s) { return static_cast<hipStream_t>(s); }

// Candidate of a tuning kind for plain calls: the caller's forced choice, else
// the default (entry 0).
int tuned(mgc_ctx ctx, int kind) {
  const int c = ctx->forced_tuning[kind];
  return c >= 0 ? c : 0;
}

// stage names of the finest level's sweeps, per internal axis
const char* const kThomasFinest[3] = {"thomas_ax0[finest]", "thomas_ax1[finest]",
                                      "thomas_ax2[finest]"};

// Reads n bytes of device memory into ctx->pinned (n <= 4 KiB): a one-block
// copy into the mapped staging buffer, then a stream synchronisation.
void sync_read(mgc_ctx ctx, void* host, const void* dev, size_t n, hipStream_t s) {
  if (host != ctx->pinned || n > 4096) fail(MGC_EINVAL, "staging read too large");
  launch_copy_bytes(ctx->pinned_dev, dev, n, s);
  MGC_HIP(hipGetLastError());
  MGC_HIP(hipStreamSynchronize(s));
}

// The solves on one level's coarse grid x: axis 2, then 1, then 0 (the
// active ones); with sub (recomposition) axis 0, then 1, then 2, and sub - x
// formed by the last, so the subtraction rides on the contiguous-axis sweep,
// which loads its rows one ahead.  The axes' solves commute (the mass matrix
// is a Kronecker product of per-axis factors).  One launch when the grid fits
// in LDS (serial sweeps), else one per axis: partitioned sweeps where the
// lines fit, serial ones otherwise or when a tuning candidate forces them
// (the caller's forced candidates when use_tuning is set).
void solve_coarse(mgc_ctx ctx, const LevelGeom& g, double* x, const double* sub, bool fin,
                  bool use_tuning, hipStream_t s) {
  if (thomas_grid_fits(g)) {
    StageScope sc(&ctx->prof, fin ? "thomas[finest]" : "thomas", s);
    launch_thomas_grid(x, g, sub, s);
    return;
  }
  auto cand = [&](int axis) {
    return use_tuning ? tuned(ctx, axis == 2 ? MGC_TUNE_THOMAS_ROWS : MGC_TUNE_THOMAS_STRIDED)
                      : 0;
  };
  int order[3] = {2, 1, 0};
  if (sub) order[0] = 0, order[2] = 2;
  int last = -1;  // the axis swept last
  for (int i = 0; i < 3; ++i)
    if (g.bit[order[i]] >= 0) last = order[i];
  for (int i = 0; i < 3; ++i) {
    const int axis = order[i];
    if (g.bit[axis] < 0) continue;
    StageScope sc(&ctx->prof, fin ? kThomasFinest[axis] : "thomas", s);
    launch_thomas(axis, x, g.nc, g.ax[axis], axis == last ? sub : nullptr, s, cand(axis));
  }
}

// The levels 1..top that run in one workgroup with their grids in LDS (0:
// none): the largest top whose levels all fit, their tables within the LDS
// copy; *tt receives the copy's range and offsets.
int tail_top(const Plan& p, TailTabArgs* tt) {
  int top = 0;
  const size_t t0 = p.lv.size() > 1 ? p.lv[1].t_wl[0] : 0;
  for (int l = 1; l <= p.L && l < kTailLevels; ++l) {
    const PlanLevel& v = p.lv[l];
    const size_t end = v.t_Mt[2] + 3 * (size_t)v.nf[2];
    if (!tail_level_fits(p.geom(l)) || end - t0 > tail_max_table()) break;
    top = l;
    tt->n = (uint32_t)(end - t0);
    for (int k = 0; k < 3; ++k) tt->wl[l][k] = (uint32_t)(v.t_wl[k] - t0);
  }
  tt->src = p.d_tab + t0;
  return top;
}

// rdev: device reciprocal bins r_0..r_L (quantising runs, sym != nullptr);
// gate: the compression's status word (null: ungated).
void run_levels_decompose(mgc_ctx ctx, const Plan& p, const void* d_in, bool in_f32,
                          double* gA, double* gB, uint16_t* sym, double* raw,
                          const double* rdev, const OutlierBuf& ob, unsigned* status,
                          const unsigned* gate, hipStream_t s) {
  const void* Gcur = d_in;
  bool cur_f32 = in_f32;
  TailTabArgs tt{};
  const int top = tail_top(p, &tt);
  for (int l = p.L; l > top; --l) {
    double* Gnext = ((p.L - l) % 2 == 0) ? gA : gB;
    const LevelGeom g = p.geom(l);
    {
      StageScope sc(&ctx->prof, l == p.L ? "dec_level[finest]" : "dec_level", s);
      launch_dec_level(Gcur, cur_f32, g, Gnext, sym, raw, sym ? rdev + l : nullptr, ob, status,
                       gate, s, tuned(ctx, cur_f32 ? MGC_TUNE_DEC_F32 : MGC_TUNE_DEC_F64));
    }
    solve_coarse(ctx, g, Gnext, nullptr, l == p.L, true, s);
    Gcur = Gnext;
    cur_f32 = false;
  }
  if (top >= 1) {
    StageScope sc(&ctx->prof, "dec_tail", s);
    launch_dec_tail(Gcur, cur_f32, p.d_geo, top, tt, sym, raw, sym ? rdev : nullptr, ob, status,
                    gate, s);
    return;
  }
  StageScope sc(&ctx->prof, "level0", s);
  launch_level0(Gcur, cur_f32, p.points(0), sym, raw, sym ? rdev : nullptr, ob, status, gate,
                s);
}

// levels (optional) receives G_0 .. G_{L-1}, level after level.
// coarse (optional): FP64 coefficients read for levels 0 .. coarse_top
// instead of src.
void run_levels_recompose(mgc_ctx ctx, const Plan& p, const CoeffSrc& src,
                          const std::vector<double>& q, double* gA, double* gB, void* d_out,
                          bool out_f32, hipStream_t s, double* levels = nullptr,
                          const CoeffSrc* coarse = nullptr, int coarse_top = -1) {
  auto src_of = [&](int l) -> const CoeffSrc& {
    return coarse && l <= coarse_top ? *coarse : src;
  };
  if (p.L == 0) {
    StageScope sc(&ctx->prof, "rec_level0", s);
    launch_rec_level0(src_of(0), p.points(0), q[0], d_out, out_f32, s);
    return;
  }
  std::vector<double*> slot(p.L + 1, gA);
  if (levels) {
    size_t off = 0;
    for (int l = 0; l < p.L; ++l) {
      slot[l] = levels + off;
      off += (size_t)p.points(l);
    }
  }
  // (with levels requested every level's grid goes to memory: no tail)
  TailTabArgs tt{};
  const int top = levels ? 0 : tail_top(p, &tt);
  if (top >= 1) {
    StageScope sc(&ctx->prof, "rec_tail", s);
    launch_rec_tail(src, coarse ? *coarse : src, coarse ? coarse_top : -1, q.data(), p.d_geo, top,
                    tt, top == p.L ? d_out : (void*)slot[0], top == p.L && out_f32, s);
    if (top == p.L) return;
  } else {
    StageScope sc(&ctx->prof, "rec_level0", s);
    launch_rec_level0(src_of(0), p.points(0), q[0], slot[0], false, s);
  }
  double* Gprev = slot[0];
  double* F = gB;
  for (int l = top + 1; l <= p.L; ++l) {
    const LevelGeom g = p.geom(l);
    const bool fin = l == p.L;
    {
      StageScope sc(&ctx->prof, fin ? "rec_restrict[finest]" : "rec_restrict", s);
      launch_rec_restrict(g, src_of(l), q[l], F, s);
    }
    solve_coarse(ctx, g, F, Gprev, fin, true, s);
    {
      StageScope sc(&ctx->prof, fin ? "rec_interp[finest]" : "rec_interp", s);
      double* dst = levels ? slot[l] : Gprev;
      launch_rec_interp(F, g, src_of(l), q[l], fin ? d_out : (void*)dst, fin && out_f32, s);
      if (!fin) Gprev = dst;
    }
  }
}


// ------------------------------------------------ allocation-free compression
// Device scratch of mgc_compress_noalloc: the plan tables and every work
// buffer of one compression, so that call allocates no device memory.  Each
// device holds its own copy until the process ends.  In host code the
// array's name is not a device address: the address of a device's copy comes
// from hipGetSymbolAddress, taken once per device at context creation, and
// only that pointer reaches kernels and copies.
static __device__ __align__(256) uint8_t scratch[MGC_NOALLOC_SCRATCH_BYTES];

struct ScratchState {
  uint8_t* ptr = nullptr;          // this device's copy of the scratch array
  std::vector<uint64_t> resident;  // shape whose plan tables the copy holds
};
struct NoAllocPlan {
  Plan plan;                       // device pointers into the device's scratch
  std::vector<uint8_t> image;      // the tables as uploaded (kept alive)
};
std::mutex g_scratch_mu;
std::map<int, ScratchState> g_scratch;  // by device ordinal
std::map<std::pair<int, std::vector<uint64_t>>, NoAllocPlan> g_noalloc_plans;

// Called with `device` current.
void scratch_setup(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  ScratchState& st = g_scratch[device];
  if (st.ptr) return;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || p == nullptr)
    fail(MGC_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
  st.ptr = static_cast<uint8_t*>(p);
}

// Stage timing is off for the duration of a call (its events are created on
// demand).
struct ProfilerPause {
  Profiler& p;
  bool was;
  explicit ProfilerPause(Profiler& prof) : p(prof), was(prof.enabled) { p.enabled = false; }
  ~ProfilerPause() { p.enabled = was; }
};

// Work buffers of the Huffman stage on its own (Algorithm 2 alone).
struct HuffWs {
  unsigned* hist;
  uint32_t* code;
  uint8_t* clen;
  CodebookScratch cbsc;
  uint32_t* cw;
  Layout* lay;
};
HuffWs carve_huff(Carver& c, uint64_t n_chunks) {
  HuffWs w;
  w.hist = c.take<unsigned>(kDict);
  w.code = c.take<uint32_t>(kDict);
  w.clen = c.take<uint8_t>(kDict);
  void* cbs = c.take<uint8_t>(codebook_scratch_bytes());
  w.cbsc = c.base ? carve_codebook_scratch(cbs) : CodebookScratch{};
  w.cw = c.take<uint32_t>(chunk_words_len((int64_t)n_chunks));
  w.lay = c.take<Layout>(1);
  return w;
}
uint64_t huff_max_bytes(uint64_t n, uint32_t C) {
  const uint64_t n_chunks = (n + C - 1) / C;
  return kHuffHeaderBytes + pad8(3 * kDict) + 8 * (n_chunks + 1) + 4 * (n + n_chunks) + 8;
}
// Histogram, codebook, chunk sizes, layout scan and encode of n > 0 keys into
// the Huffman-only stream at out (its 48-byte header is written separately).
void huff_encode_enqueue(mgc_ctx ctx, const uint16_t* sym, uint64_t n, uint32_t C,
                         uint8_t* out, const HuffWs& w, hipStream_t s,
                         uint32_t win_lo = kHistWinLo, uint32_t hot = 0) {
  const uint64_t n_chunks = (n + C - 1) / C;
  {
    StageScope st(&ctx->prof, "histogram", s);
    launch_histogram(sym, (int64_t)n, w.hist, s, nullptr, win_lo, hot);
  }
  {
    StageScope st(&ctx->prof, "codebook", s);
    launch_codebook(w.hist, w.cbsc, w.code, w.clen, out, kHuffHeaderBytes, w.lay, s);
  }
  {
    StageScope st(&ctx->prof, "chunk_words", s);
    launch_chunk_words(sym, (int64_t)n, (int)C, w.clen, w.cw, w.lay, s);
  }
  {
    StageScope st(&ctx->prof, "layout_scan", s);
    launch_layout_scan(w.cw, (int64_t)n_chunks, out, kHuffHeaderBytes, w.lay, nullptr, 0, true, s);
  }
  {
    StageScope st(&ctx->prof, "encode", s);
    launch_encode(sym, (int64_t)n, (int)C, w.code, w.clen, w.cbsc.pk, out, w.lay, s);
  }
}
// Checks a Huffman-only stream header against the values it must describe;
// returns the byte offsets of its chunk offsets and words sections.
void check_huff_header(const HuffHeader& h, uint64_t n, uint64_t avail, uint64_t* off,
                       uint64_t* words) {
  if (h.magic != kHuffMagic || h.N != n || h.C < 1 || h.C > (1u << 20) ||
      h.n_chunks != (h.N + h.C - 1) / h.C || h.n_codes > kDict || (n > 0 && h.n_codes < 1))
    fail(MGC_EFORMAT, "bad huffman header");
  *off = pad8(kHuffHeaderBytes + 3 * h.n_codes);
  *words = *off + 8 * (h.n_chunks + 1);
  const uint64_t end = pad8(*words + 4 * h.n_words);
  if (end != h.total || h.total > avail) fail(MGC_EFORMAT, "truncated huffman stream");
  if (n > 0 && h.n_words < 1) fail(MGC_EFORMAT, "huffman stream without coded words");
}

// Huffman-X value types: width, whether values can escape, and the key
// window [lo, hi] of a dictionary and base (validated).
uint32_t hx_width(int type) { return type == MGC_HX_U8 ? 1 : type == MGC_HX_U16 ? 2 : type == MGC_HX_I32 ? 4 : 8; }
bool hx_escapes(int type) { return type == MGC_HX_I32 || type == MGC_HX_I64; }
void hx_window(int type, uint32_t dict, int64_t base, int64_t* lo, int64_t* hi) {
  if (type < MGC_HX_U8 || type > MGC_HX_I64) fail(MGC_EINVAL, "unknown Huffman-X value type");
  if (!hx_escapes(type)) {
    if (dict != (type == MGC_HX_U8 ? 256u : 65536u) || base != 0)
      fail(MGC_EINVAL, "u8 and u16 streams take their full range as the dictionary, base 0");
    *lo = 0;
    *hi = (int64_t)dict - 1;
    return;
  }
  if (dict < 2 || dict > 65536) fail(MGC_EINVAL, "dictionary size must be in [2, 65536]");
  const int64_t tmax = type == MGC_HX_I32 ? INT32_MAX : INT64_MAX;
  const int64_t tmin = type == MGC_HX_I32 ? INT32_MIN : INT64_MIN;
  if (base < tmin || base > tmax) fail(MGC_EINVAL, "base outside the value type");
  *lo = base;
  *hi = base > tmax - (int64_t)(dict - 2) ? tmax : base + (int64_t)(dict - 2);
}

struct HxWs {
  uint16_t* key;  // null for u16 (the values are the keys)
  HuffWs huff;
  unsigned long long* info;
  uint32_t *zc, *zpre, *sums;
  DecodeTables* tables;
  unsigned* status;
  Layout* lay0;  // a clear layout for the decoder's chunk prefix
};
HxWs carve_hx(Carver& c, uint64_t n, int type, uint32_t C) {
  HxWs w;
  const uint64_t n_chunks = (n + C - 1) / C, n1024 = (n + 1023) / 1024;
  w.key = type == MGC_HX_U16 ? nullptr : c.take<uint16_t>(std::max<uint64_t>(n, 1));
  w.huff = carve_huff(c, n_chunks);
  w.info = c.take<unsigned long long>(4);
  w.zc = c.take<uint32_t>(std::max<uint64_t>(n1024, 1));
  w.zpre = c.take<uint32_t>(std::max<uint64_t>(n1024, 1));
  w.sums = c.take<uint32_t>(kEscSumsMax);
  w.tables = reinterpret_cast<DecodeTables*>(c.take<uint8_t>(decode_tables_bytes()));
  w.status = c.take<unsigned>(4);
  w.lay0 = c.take<Layout>(1);
  return w;
}
}  // namespace

namespace mgc {
// Decompression launches on stream s for a stream whose first head_bytes
// (header and bins) the host already holds; returns the device status word
// the decoder sets (ST_FORMAT on corrupt data), or null when nothing was
// decoded (empty or constant arrays).
const unsigned* decompress_enqueue(mgc_ctx ctx, const uint8_t* head, size_t head_bytes,
                                   const void* d_in, size_t in_bytes, void* d_out,
                                   size_t out_cap, void* d_ws, size_t ws_bytes, hipStream_t s) {
  Header h;
  std::vector<double> q;
  parse_header(head, head_bytes, &h, &q);
  const Plan& p = get_plan(ctx, h.ndim, h.shape);
  const mgc_dtype dt = (mgc_dtype)h.dtype;
  if ((uint64_t)p.N != h.N) fail(MGC_EFORMAT, "header size inconsistent with its shape");
  if (h.total > in_bytes) fail(MGC_EFORMAT, "truncated stream");
  if (out_cap < (size_t)p.N * dtype_size(dt)) fail(MGC_ENOSPC, "output capacity too small");
  if (h.flags & FLAG_EMPTY) return nullptr;
  if (h.flags & FLAG_CONSTANT) {
    launch_fill(d_out, dt == MGC_F32, p.N, h.const_value, s);
    MGC_HIP(hipGetLastError());
    return nullptr;
  }
  if (h.L != (uint32_t)p.L || h.S != kDict || h.C < 1 || h.C > (1u << 20) ||
      h.n_chunks != (h.N + h.C - 1) / h.C || h.n_codes > kDict || h.n_codes < 1 ||
      h.n_outliers > h.N || h.n_words < 1)
    fail(MGC_EFORMAT, "inconsistent header counts");
  const uint64_t cb = kHeaderBytes + 8 * (h.L + 1);
  const uint64_t off = pad8(cb + 3 * h.n_codes);
  const uint64_t opos = off + 8 * (h.n_chunks + 1);
  const uint64_t oval = opos + 8 * h.n_outliers;
  const uint64_t words = oval + 8 * h.n_outliers;
  const uint64_t end = pad8(words + 4 * h.n_words);
  if (end != h.total) fail(MGC_EFORMAT, "section sizes disagree with the stream length");
  Carver meas(nullptr);
  carve_decompress(meas, p);
  if (ws_bytes < meas.off) fail(MGC_ENOSPC, "workspace too small");
  Carver c(d_ws);
  DecompressWs w = carve_decompress(c, p);
  const uint8_t* in = static_cast<const uint8_t*>(d_in);
  {
    // (the table build clears the status words first)
    StageScope st(&ctx->prof, "decode_tables", s);
    launch_decode_tables(in + cb, h.n_codes, static_cast<DecodeTables*>(w.tables), w.status, s);
  }
  {
    StageScope st(&ctx->prof, "decode", s);
    ctx->dec_last = launch_decode(in, off, words, h.n_chunks, h.n_words, (int)h.C, p.N,
                                  h.n_codes, static_cast<const DecodeTables*>(w.tables),
                                  w.sym, w.status, s, ctx->dec_force);
  }
  CoeffSrc src{w.sym, nullptr, reinterpret_cast<const uint64_t*>(in + opos),
               reinterpret_cast<const int64_t*>(in + oval), (int64_t)h.n_outliers};
  if (p.L >= 2) {
    // levels 0 .. L-2 dequantised ahead (escaped values resolved once)
    LevelBins lb{};
    lb.n = p.L - 1;
    for (int l = 0; l < lb.n; ++l) {
      lb.off[l] = p.lv[l].off;
      lb.q[l] = q[l];
    }
    const int64_t m = p.points(p.L - 2);
    {
      StageScope st(&ctx->prof, "dequant_coarse", s);
      launch_dequant_prefix(src, m, lb, w.coarse, s);
    }
    const CoeffSrc coarse{nullptr, w.coarse, nullptr, nullptr, 0};
    run_levels_recompose(ctx, p, src, q, w.gA, w.gB, d_out, dt == MGC_F32, s, nullptr,
                         &coarse, p.L - 2);
  } else {
    run_levels_recompose(ctx, p, src, q, w.gA, w.gB, d_out, dt == MGC_F32, s);
  }
  MGC_HIP(hipGetLastError());
  return w.status;
}
}  // namespace mgc

extern "C" {

int mgc_version(void) { return 1; }

const char* mgc_last_error(void) { return g_err.c_str(); }

mgc_status mgc_create(int device, mgc_ctx* out) {
  return guard([&] {
    if (!out) fail(MGC_EINVAL, "null output");
    int n = 0;
    MGC_HIP(hipGetDeviceCount(&n));
    if (device < 0 || device >= n) fail(MGC_EINVAL, "device ordinal out of range");
    MGC_HIP(hipSetDevice(device));
    scratch_setup(device);
    auto* c = new mgc_ctx_s;
    c->device = device;
    if (hipHostMalloc((void**)&c->pinned, 4096, hipHostMallocDefault) != hipSuccess) {
      delete c;
      fail(MGC_EDEVICE, "hipHostMalloc failed");
    }
    if (hipHostGetDevicePointer((void**)&c->pinned_dev, c->pinned, 0) != hipSuccess) {
      (void)hipHostFree(c->pinned);
      delete c;
      fail(MGC_EDEVICE, "hipHostGetDevicePointer failed");
    }
    *out = c;
  });
}

mgc_status mgc_destroy(mgc_ctx ctx) {
  return guard([&] {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    for (auto& kv : ctx->batches) free_batch_plan(kv.second);
    if (ctx->capture_stream) (void)hipStreamDestroy(ctx->capture_stream);
    for (auto& kv : ctx->plans) free_plan(kv.second);
    if (ctx->pinned) (void)hipHostFree(ctx->pinned);
    delete ctx;
  });
}

mgc_status mgc_compress_query(int ndim, const uint64_t* shape, mgc_dtype dtype,
                              uint64_t outlier_cap, size_t* ws_bytes, size_t* max_out_bytes) {
  return guard([&] {
    if (dtype != MGC_F32 && dtype != MGC_F64) fail(MGC_EINVAL, "dtype must be f32 or f64");
    Plan p = build_plan(ndim, shape);
    const uint64_t cap = outlier_cap ? outlier_cap : default_outlier_cap(p.N);
    Carver c(nullptr);
    carve_compress(c, p, cap);
    if (ws_bytes) *ws_bytes = c.off;
    if (max_out_bytes) *max_out_bytes = max_stream_bytes(p, cap);
  });
}

namespace {
// Enqueues a whole compression on s (no host synchronisation).  res: two
// device words receiving the mgc_status and the stream length (or, with
// MGC_ENOSPC, the escaped values needed).  ws must hold carve_compress's
// layout for the outlier capacity cap.
void compress_enqueue(mgc_ctx ctx, const Plan& p, const void* d_in, int ndim,
                      const uint64_t* shape, mgc_dtype dtype, double error_bound,
                      mgc_norm norm, mgc_mode mode, uint64_t cap, void* d_out, void* d_ws,
                      unsigned long long* res, hipStream_t s) {
  Carver c(d_ws);
  CompressWs w = carve_compress(c, p, cap);
  uint8_t* out = static_cast<uint8_t*>(d_out);
  const Header h = make_header(p, ndim, shape, dtype, error_bound, norm, mode);
  if (p.N == 0) {
    launch_header(out, h, nullptr, nullptr, nullptr, true, res, s);
    return;
  }
  {
    void* const zp[4] = {w.status, w.n_out, w.lay, w.hist};
    const size_t zb[4] = {4 * sizeof(unsigned), sizeof(unsigned long long), sizeof(Layout),
                          kDict * sizeof(unsigned)};
    launch_zero_words(zp, zb, 4, s);
  }
  {
    StageScope sc(&ctx->prof, "range", s);
    const BudgetIn bi{(int)dtype, (int)norm, (int)mode, p.L, error_bound, p.N,
                      p.d_K[norm == MGC_LINF ? 0 : 1]};
    launch_range(d_in, dtype, p.N, w.part, bi, w.bud, w.status, s);
  }
  const unsigned* gate = w.status;
  OutlierBuf ob{w.opos, w.oval, w.n_out, cap};
  run_levels_decompose(ctx, p, d_in, dtype == MGC_F32, w.gA, w.gB, w.sym, nullptr,
                       w.bud + bud_r(p.L, 0), ob, w.status, gate, s);
  const uint64_t cb_off = kHeaderBytes + 8 * (p.L + 1);
  const CodebookScratch sc = carve_codebook_scratch(w.cbs);
  {
    StageScope st(&ctx->prof, "histogram", s);
    launch_histogram(w.sym, p.N, w.hist, s, gate);
  }
  {
    StageScope st(&ctx->prof, "codebook", s);
    launch_codebook(w.hist, sc, w.code, w.clen, out, cb_off, w.lay, s, gate);
  }
  {
    StageScope st(&ctx->prof, "chunk_words", s);
    launch_chunk_words(w.sym, p.N, kChunk, w.clen, w.cw, w.lay, s, gate, w.zc, w.zl);
  }
  {
    StageScope st(&ctx->prof, "layout_scan", s);
    launch_layout_scan(w.cw, (int64_t)h.n_chunks, out, cb_off, w.lay, w.n_out, cap, false, s,
                       gate);
  }
  {
    StageScope st(&ctx->prof, "outlier_order", s);
    launch_escape_order(ob, w.zc, w.zl, w.zpre, w.zsums, (int64_t)h.n_chunks, out, w.lay,
                        w.status, s, gate);
  }
  {
    StageScope st(&ctx->prof, "encode", s);
    launch_encode(w.sym, p.N, kChunk, w.code, w.clen, sc.pk, out, w.lay, s, gate);
  }
  {
    StageScope st(&ctx->prof, "header", s);
    launch_header(out, h, w.bud, w.lay, w.status, false, res, s);
  }
  MGC_HIP(hipGetLastError());
}

// Argument checks shared by the compression entry points; returns the plan.
extern "C++" {
static const Plan& compress_checks(mgc_ctx ctx, const void* d_in, int ndim, const uint64_t* shape,
                            mgc_dtype dtype, double error_bound, mgc_norm norm, mgc_mode mode,
                            uint64_t* cap, const void* d_out, size_t out_cap, const void* d_ws,
                            size_t ws_bytes) {
  check_ctx(ctx);
  if (dtype != MGC_F32 && dtype != MGC_F64) fail(MGC_EINVAL, "dtype must be f32 or f64");
  if (norm != MGC_LINF && norm != MGC_L2) fail(MGC_EINVAL, "norm must be L-inf or L2");
  if (mode != MGC_REL && mode != MGC_ABS) fail(MGC_EINVAL, "mode must be rel or abs");
  if (!(error_bound > 0.0) || !std::isfinite(error_bound))
    fail(MGC_EINVAL, "error bound must be positive and finite");
  const Plan& p = get_plan(ctx, ndim, shape);
  *cap = *cap ? *cap : default_outlier_cap(p.N);
  Carver meas(nullptr);
  carve_compress(meas, p, *cap);
  if (ws_bytes < meas.off) fail(MGC_ENOSPC, "workspace too small");
  if (out_cap < max_stream_bytes(p, *cap)) fail(MGC_ENOSPC, "output capacity too small");
  if (!d_out) fail(MGC_EINVAL, "null output pointer");
  if (p.N > 0 && (!d_in || !d_ws)) fail(MGC_EINVAL, "null device pointer");
  return p;
}
}  // extern "C++"
}  // namespace

mgc_status mgc_compress(mgc_ctx ctx, const void* d_in, int ndim, const uint64_t* shape,
                        mgc_dtype dtype, double error_bound, mgc_norm norm, mgc_mode mode,
                        uint64_t outlier_cap, void* d_out, size_t out_cap, void* d_ws,
                        size_t ws_bytes, uint64_t* d_result, void* stream) {
  return guard([&] {
    uint64_t cap = outlier_cap;
    const Plan& p = compress_checks(ctx, d_in, ndim, shape, dtype, error_bound, norm, mode, &cap,
                                    d_out, out_cap, d_ws, ws_bytes);
    if (!d_result) fail(MGC_EINVAL, "null result pointer");
    compress_enqueue(ctx, p, d_in, ndim, shape, dtype, error_bound, norm, mode, cap, d_out, d_ws,
                     reinterpret_cast<unsigned long long*>(d_result), as_stream(stream));
  });
}

mgc_status mgc_compress_blocking(mgc_ctx ctx, const void* d_in, int ndim, const uint64_t* shape,
                                 mgc_dtype dtype, double error_bound, mgc_norm norm,
                                 mgc_mode mode, uint64_t outlier_cap, void* d_out,
                                 size_t out_cap, void* d_ws, size_t ws_bytes, void* stream,
                                 uint64_t* h_out_size) {
  return guard([&] {
    if (!h_out_size) fail(MGC_EINVAL, "null size output");
    uint64_t cap = outlier_cap;
    const Plan& p = compress_checks(ctx, d_in, ndim, shape, dtype, error_bound, norm, mode, &cap,
                                    d_out, out_cap, d_ws, ws_bytes);
    hipStream_t s = as_stream(stream);
    unsigned long long* res = nullptr;
    if (p.N > 0) {
      Carver c(d_ws);
      res = carve_compress(c, p, cap).info;
    } else {
      res = reinterpret_cast<unsigned long long*>(ctx->pinned_dev + 2048);
    }
    compress_enqueue(ctx, p, d_in, ndim, shape, dtype, error_bound, norm, mode, cap, d_out, d_ws,
                     res, s);
    unsigned long long r[2];
    sync_read(ctx, ctx->pinned, res, sizeof(r), s);
    std::memcpy(r, ctx->pinned, sizeof(r));
    *h_out_size = r[1];
    switch ((int)r[0]) {
      case MGC_OK: return;
      case MGC_ENOSPC:
        fail(MGC_ENOSPC, "more escaped values than the outlier capacity; retry with capacity " +
                             std::to_string(r[1]));
      case MGC_EINVAL: fail(MGC_EINVAL, "input holds NaN or Inf");
      case MGC_ERANGE:
        fail(MGC_ERANGE, "error bound below the resolution of the data or the output type");
      default: fail(MGC_EDEVICE, "device status " + std::to_string(r[0]));
    }
  });
}

mgc_status mgc_compress_noalloc(mgc_ctx ctx, const void* d_in, int ndim, const uint64_t* shape,
                                mgc_dtype dtype, double error_bound, mgc_norm norm, mgc_mode mode,
                                uint64_t outlier_cap, void* d_out, size_t out_cap,
                                uint64_t* d_result, void* stream) {
  return guard([&] {
    check_ctx(ctx);
    if (dtype != MGC_F32 && dtype != MGC_F64) fail(MGC_EINVAL, "dtype must be f32 or f64");
    if (norm != MGC_LINF && norm != MGC_L2) fail(MGC_EINVAL, "norm must be L-inf or L2");
    if (mode != MGC_REL && mode != MGC_ABS) fail(MGC_EINVAL, "mode must be rel or abs");
    if (!(error_bound > 0.0) || !std::isfinite(error_bound))
      fail(MGC_EINVAL, "error bound must be positive and finite");
    if (ndim < 1) fail(MGC_EINVAL, "ndim must be at least 1");
    if (ndim > 3) fail(MGC_EUNSUPPORTED, "ndim above 3 is not supported");
    if (!shape) fail(MGC_EINVAL, "null shape");
    if (!d_out || !d_result) fail(MGC_EINVAL, "null output pointer");
    MGC_HIP(hipSetDevice(ctx->device));
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    ScratchState& st = g_scratch[ctx->device];
    if (!st.ptr) fail(MGC_EDEVICE, "scratch of the device not set up");
    std::vector<uint64_t> key(shape, shape + ndim);
    key.insert(key.begin(), (uint64_t)ndim);
    auto it = g_noalloc_plans.find({ctx->device, key});
    if (it == g_noalloc_plans.end()) {
      NoAllocPlan np;
      np.plan = build_plan(ndim, shape);
      np.image = plan_device_image(np.plan, st.ptr);
      it = g_noalloc_plans.emplace(std::make_pair(ctx->device, key), std::move(np)).first;
    }
    const Plan& p = it->second.plan;
    const uint64_t cap = outlier_cap ? outlier_cap : default_outlier_cap(p.N);
    const size_t tab_bytes = (it->second.image.size() + 255) & ~size_t(255);
    Carver meas(nullptr);
    carve_compress(meas, p, cap);
    const size_t need = tab_bytes + meas.off;
    if (need > (size_t)MGC_NOALLOC_SCRATCH_BYTES)
      fail(MGC_ENOSPC, "the allocation-free compression needs " + std::to_string(need) +
                           " bytes of device scratch for this shape and outlier capacity; its "
                           "scratch holds " + std::to_string((size_t)MGC_NOALLOC_SCRATCH_BYTES));
    if (out_cap < max_stream_bytes(p, cap)) fail(MGC_ENOSPC, "output capacity too small");
    if (p.N > 0 && !d_in) fail(MGC_EINVAL, "null device pointer");
    hipStream_t s = as_stream(stream);
    if (st.resident != key) {
      MGC_HIP(hipMemcpyAsync(st.ptr, it->second.image.data(), it->second.image.size(),
                             hipMemcpyHostToDevice, s));
      st.resident = key;
    }
    ProfilerPause pause(ctx->prof);
    compress_enqueue(ctx, p, d_in, ndim, shape, dtype, error_bound, norm, mode, cap, d_out,
                     st.ptr + tab_bytes, reinterpret_cast<unsigned long long*>(d_result), s);
  });
}

mgc_status mgc_header_info(const void* h_prefix, size_t n, int* ndim, uint64_t* shape3,
                           mgc_dtype* dtype, uint64_t* stream_bytes, size_t* ws_bytes) {
  return guard([&] {
    if (!h_prefix) fail(MGC_EINVAL, "null prefix");
    Header h;
    std::vector<double> q;
    parse_header(static_cast<const uint8_t*>(h_prefix), n, &h, &q);
    if (ndim) *ndim = h.ndim;
    if (shape3)
      for (int d = 0; d < 3; ++d) shape3[d] = d < h.ndim ? h.shape[d] : 0;
    if (dtype) *dtype = (mgc_dtype)h.dtype;
    if (stream_bytes) *stream_bytes = h.total;
    if (ws_bytes) {
      Plan p = build_plan(h.ndim, h.shape);
      Carver c(nullptr);
      carve_decompress(c, p);
      *ws_bytes = c.off;
    }
  });
}

mgc_status mgc_decompress(mgc_ctx ctx, const void* d_in, size_t in_bytes, void* d_out,
                          size_t out_cap, void* d_ws, size_t ws_bytes, void* stream) {
  return guard([&] {
    check_ctx(ctx);
    if (!d_in) fail(MGC_EINVAL, "null input");
    hipStream_t s = as_stream(stream);
    const size_t pre = std::min<size_t>(in_bytes, kHeaderBytes + 8 * (kMaxLevels + 1));
    if (pre < (size_t)kHeaderBytes) fail(MGC_EFORMAT, "stream shorter than its header");
    sync_read(ctx, ctx->pinned, d_in, pre, s);
    std::vector<uint8_t> head(ctx->pinned, ctx->pinned + pre);
    const unsigned* status =
        decompress_enqueue(ctx, head.data(), pre, d_in, in_bytes, d_out, out_cap, d_ws, ws_bytes, s);
    if (!status) return;
    unsigned st = 0;
    sync_read(ctx, ctx->pinned, status, sizeof(unsigned), s);
    std::memcpy(&st, ctx->pinned, sizeof(unsigned));
    if (st & ST_FORMAT) fail(MGC_EFORMAT, "corrupt coded data");
  });
}

mgc_status mgc_transform_query(int ndim, const uint64_t* shape, size_t* ws_bytes) {
  return guard([&] {
    Plan p = build_plan(ndim, shape);
    const int64_t n_coarse = p.L >= 1 ? p.points(p.L - 1) : 1;
    Carver c(nullptr);
    c.take<double>(n_coarse);
    c.take<double>(n_coarse);
    c.take<unsigned>(4);
    if (ws_bytes) *ws_bytes = c.off;
  });
}

mgc_status mgc_decompose(mgc_ctx ctx, const void* d_in, int ndim, const uint64_t* shape,
                         mgc_dtype dtype, double* d_coeffs, void* d_ws, size_t ws_bytes,
                         void* stream) {
  return guard([&] {
    check_ctx(ctx);
    if (dtype != MGC_F32 && dtype != MGC_F64) fail(MGC_EINVAL, "dtype must be f32 or f64");
    const Plan& p = get_plan(ctx, ndim, shape);
    if (p.N == 0) return;
    const int64_t n_coarse = p.L >= 1 ? p.points(p.L - 1) : 1;
    Carver c(d_ws);
    double* gA = c.take<double>(n_coarse);
    double* gB = c.take<double>(n_coarse);
    unsigned* status = c.take<unsigned>(4);
    if (ws_bytes < c.off) fail(MGC_ENOSPC, "workspace too small");
    hipStream_t s = as_stream(stream);
    OutlierBuf ob{nullptr, nullptr, nullptr, 0};
    run_levels_decompose(ctx, p, d_in, dtype == MGC_F32, gA, gB, nullptr, d_coeffs, nullptr, ob,
                         status, nullptr, s);
    MGC_HIP(hipGetLastError());
  });
}

mgc_status mgc_recompose(mgc_ctx ctx, const double* d_coeffs, int ndim, const uint64_t* shape,
                         mgc_dtype out_dtype, void* d_out, void* d_ws, size_t ws_bytes,
                         void* stream) {
  return guard([&] {
    check_ctx(ctx);
    if (out_dtype != MGC_F32 && out_dtype != MGC_F64) fail(MGC_EINVAL, "dtype must be f32 or f64");
    const Plan& p = get_plan(ctx, ndim, shape);
    if (p.N == 0) return;
    const int64_t n_coarse = p.L >= 1 ? p.points(p.L - 1) : 1;
    Carver c(d_ws);
    double* gA = c.take<double>(n_coarse);
    double* gB = c.take<double>(n_coarse);
    c.take<unsigned>(4);
    if (ws_bytes < c.off) fail(MGC_ENOSPC, "workspace too small");
    hipStream_t s = as_stream(stream);
    CoeffSrc src{nullptr, d_coeffs, nullptr, nullptr, 0};
    run_levels_recompose(ctx, p, src, std::vector<double>(p.L + 1, 1.0), gA, gB, d_out,
                         out_dtype == MGC_F32, s);
    MGC_HIP(hipGetLastError());
  });
}

namespace {
struct AdjointWs {
  double *gA, *gB, *Y, *T;
};
AdjointWs carve_adjoint(Carver& c, const Plan& p) {
  const int64_t n_coarse = p.L >= 1 ? p.points(p.L - 1) : 1;
  AdjointWs w;
  w.gA = c.take<double>(n_coarse);
  w.gB = c.take<double>(n_coarse);
  w.Y = c.take<double>(n_coarse);
  w.T = c.take<double>(std::max<int64_t>(p.N, 1));
  return w;
}
size_t levels_bytes_of(const Plan& p) {
  size_t n = 0;
  for (int l = 0; l < p.L; ++l) n += (size_t)p.points(l);
  return 8 * std::max<size_t>(n, 1);
}
}  // namespace

mgc_status mgc_adjoint_query(int ndim, const uint64_t* shape, size_t* ws_bytes) {
  return guard([&] {
    Plan p = build_plan(ndim, shape);
    Carver c(nullptr);
    carve_adjoint(c, p);
    if (ws_bytes) *ws_bytes = c.off;
  });
}

mgc_status mgc_recompose_adjoint(mgc_ctx ctx, const double* d_grad_u, int ndim,
                                 const uint64_t* shape, double* d_grad_coeffs, void* d_ws,
                                 size_t ws_bytes, void* stream) {
  return guard([&] {
    check_ctx(ctx);
    const Plan& p = get_plan(ctx, ndim, shape);
    if (p.N == 0) return;
    if (!d_grad_u || !d_grad_coeffs || !d_ws) fail(MGC_EINVAL, "null device pointer");
    Carver meas(nullptr);
    carve_adjoint(meas, p);
    if (ws_bytes < meas.off) fail(MGC_ENOSPC, "workspace too small");
    Carver c(d_ws);
    AdjointWs w = carve_adjoint(c, p);
    hipStream_t s = as_stream(stream);
    const double* g = d_grad_u;
    for (int l = p.L; l >= 1; --l) {
      const LevelGeom geom = p.geom(l);
      double* Gc = (g == w.gA) ? w.gB : w.gA;
      {
        StageScope sc(&ctx->prof, "adj_restrict", s);
        launch_adj_restrict(g, geom, Gc, w.Y, s);
      }
      solve_coarse(ctx, geom, w.Y, nullptr, false, false, s);
      {
        StageScope sc(&ctx->prof, "adj_prolong", s);
        launch_prolong(w.Y, geom, w.T, s);
      }
      {
        StageScope sc(&ctx->prof, "adj_mass", s);
        launch_adj_mass(w.T, g, geom, d_grad_coeffs, s);
      }
      g = Gc;
    }
    OutlierBuf ob{nullptr, nullptr, nullptr, 0};
    launch_level0(g, false, p.points(0), nullptr, d_grad_coeffs, nullptr, ob, nullptr, nullptr,
                  s);
    MGC_HIP(hipGetLastError());
  });
}

mgc_status mgc_levels_query(int ndim, const uint64_t* shape, size_t* levels_bytes) {
  return guard([&] {
    Plan p = build_plan(ndim, shape);
    if (levels_bytes) *levels_bytes = levels_bytes_of(p);
  });
}

mgc_status mgc_recompose_levels(mgc_ctx ctx, const double* d_coeffs, int ndim,
                                const uint64_t* shape, mgc_dtype out_dtype, void* d_out,
                                double* d_levels, size_t levels_bytes, void* d_ws,
                                size_t ws_bytes, void* stream) {
  return guard([&] {
    check_ctx(ctx);
    if (out_dtype != MGC_F32 && out_dtype != MGC_F64) fail(MGC_EINVAL, "dtype must be f32 or f64");
    const Plan& p = get_plan(ctx, ndim, shape);
    if (p.N == 0) return;
    if (levels_bytes < levels_bytes_of(p)) fail(MGC_ENOSPC, "level buffer too small");
    const int64_t n_coarse = p.L >= 1 ? p.points(p.L - 1) : 1;
    Carver c(d_ws);
    double* gA = c.take<double>(n_coarse);
    double* gB = c.take<double>(n_coarse);
    c.take<unsigned>(4);
    if (ws_bytes < c.off) fail(MGC_ENOSPC, "workspace too small");
    CoeffSrc src{nullptr, d_coeffs, nullptr, nullptr, 0};
    run_levels_recompose(ctx, p, src, std::vector<double>(p.L + 1, 1.0), gA, gB, d_out,
                         out_dtype == MGC_F32, as_stream(stream), d_levels);
    MGC_HIP(hipGetLastError());
  });
}

mgc_status mgc_huffman_query(uint64_t n, uint32_t C, size_t* ws_bytes, size_t* max_out_bytes) {
  return guard([&] {
    if (C < 64 || C > 65536 || C % 64) fail(MGC_EINVAL, "chunk size must be a multiple of 64 in [64, 65536]");
    const uint64_t n_chunks = (n + C - 1) / C;
    Carver c(nullptr);
    carve_huff(c, n_chunks);
    c.take<unsigned long long>(4);
    c.take<uint8_t>(decode_tables_bytes());
    c.take<unsigned>(4);
    if (ws_bytes) *ws_bytes = c.off;
    if (max_out_bytes) *max_out_bytes = huff_max_bytes(n, C);
  });
}

mgc_status mgc_huffman_encode(mgc_ctx ctx, const uint16_t* d_sym, uint64_t n, uint32_t C,
                              void* d_out, size_t out_cap, void* d_ws, size_t ws_bytes,
                              void* stream, uint64_t* h_out_size) {
  return guard([&] {
    check_ctx(ctx);
    size_t need_ws = 0, need_out = 0;
    if (mgc_huffman_query(n, C, &need_ws, &need_out) != MGC_OK) throw Fail{MGC_EINVAL};
    if (ws_bytes < need_ws || out_cap < need_out) fail(MGC_ENOSPC, "workspace or output too small");
    if (n >= (1ull << 32)) fail(MGC_EUNSUPPORTED, "2^32 or more symbols");
    if (!h_out_size) fail(MGC_EINVAL, "null size output");
    hipStream_t s = as_stream(stream);
    const uint64_t n_chunks = (n + C - 1) / C;
    Carver c(d_ws);
    const HuffWs w = carve_huff(c, n_chunks);
    unsigned long long* info = c.take<unsigned long long>(4);
    uint8_t* out = static_cast<uint8_t*>(d_out);
    MGC_HIP(hipMemsetAsync(w.hist, 0, kDict * sizeof(unsigned), s));
    MGC_HIP(hipMemsetAsync(w.lay, 0, sizeof(Layout), s));
    if (n > 0) {
      huff_encode_enqueue(ctx, d_sym, n, C, out, w, s);
    } else {
      StageScope st(&ctx->prof, "codebook", s);
      launch_codebook(w.hist, w.cbsc, w.code, w.clen, out, kHuffHeaderBytes, w.lay, s);
      launch_layout_scan(w.cw, 0, out, kHuffHeaderBytes, w.lay, nullptr, 0, true, s);
    }
    launch_huff_header(out, C, n, n_chunks, w.lay, info, s);
    MGC_HIP(hipGetLastError());
    unsigned long long inf[3];
    sync_read(ctx, ctx->pinned, info, sizeof(inf), s);
    std::memcpy(inf, ctx->pinned, sizeof(inf));
    if (inf[0]) fail(MGC_EDEVICE, "huffman encode failed");
    *h_out_size = inf[2];
  });
}

mgc_status mgc_huffman_decode(mgc_ctx ctx, const void* d_in, size_t in_bytes, uint16_t* d_sym,
                              uint64_t n, void* d_ws, size_t ws_bytes, void* stream) {
  return guard([&] {
    check_ctx(ctx);
    if (in_bytes < (size_t)kHuffHeaderBytes) fail(MGC_EFORMAT, "stream shorter than its header");
    hipStream_t s = as_stream(stream);
    sync_read(ctx, ctx->pinned, d_in, kHuffHeaderBytes, s);
    HuffHeader h;
    std::memcpy(&h, ctx->pinned, kHuffHeaderBytes);
    uint64_t off = 0, words = 0;
    check_huff_header(h, n, in_bytes, &off, &words);
    Carver meas(nullptr);
    meas.take<uint8_t>(decode_tables_bytes());
    meas.take<unsigned>(4);
    if (ws_bytes < meas.off) fail(MGC_ENOSPC, "workspace too small");
    if (n == 0) return;
    Carver c(d_ws);
    void* tables = c.take<uint8_t>(decode_tables_bytes());
    unsigned* status = c.take<unsigned>(4);
    const uint8_t* in = static_cast<const uint8_t*>(d_in);
    MGC_HIP(hipMemsetAsync(status, 0, 4 * sizeof(unsigned), s));
    {
      StageScope st(&ctx->prof, "decode_tables", s);
      launch_decode_tables(in + kHuffHeaderBytes, h.n_codes, static_cast<DecodeTables*>(tables),
                           status, s);
    }
    {
      StageScope st(&ctx->prof, "decode", s);
      ctx->dec_last = launch_decode(in, off, words, h.n_chunks, h.n_words, (int)h.C,
                                    (int64_t)n, h.n_codes,
                                    static_cast<const DecodeTables*>(tables), d_sym, status, s,
                                    ctx->dec_force);
    }
    MGC_HIP(hipGetLastError());
    unsigned st = 0;
    sync_read(ctx, ctx->pinned, status, sizeof(unsigned), s);
    std::memcpy(&st, ctx->pinned, sizeof(unsigned));
    if (st & ST_FORMAT) fail(MGC_EFORMAT, "corrupt coded data");
  });
}

mgc_status mgc_zfp_query(int ndim, const uint64_t* shape, mgc_dtype dtype, double rate,
                         size_t* stream_bytes) {
  return guard([&] {
    if (ndim < 1 || ndim > 3 || !shape) fail(MGC_EINVAL, "ndim must be 1..3");
    if (dtype != MGC_F32 && dtype != MGC_F64) fail(MGC_EINVAL, "bad dtype");
    uint64_t nb = 1;
    for (int d = 0; d < ndim; ++d) {
      if (shape[d] == 0) fail(MGC_EINVAL, "empty arrays are not block-coded");
      nb *= (shape[d] + 3) / 4;
    }
    const int P = dtype == MGC_F64 ? 64 : 32, eb = dtype == MGC_F64 ? 12 : 9;
    const double mbd = std::nearbyint(rate * (double)(1u << (2 * ndim)));
    if (!std::isfinite(rate) || mbd < 2 + eb || rate > 2.0 * P)
      fail(MGC_EINVAL, "rate out of range");
    const uint64_t mb = (uint64_t)mbd;
    if (stream_bytes) *stream_bytes = kZfpHeaderBytes + 8 * ((nb * mb + 63) / 64);
  });
}

mgc_status mgc_zfp_compress(mgc_ctx ctx, const void* d_in, int ndim, const uint64_t* shape,
                            mgc_dtype dtype, double rate, void* d_out, size_t out_cap,
                            uint64_t* d_result, void* stream) {
  return guard([&] {
    check_ctx(ctx);
    size_t need = 0;
    if (mgc_zfp_query(ndim, shape, dtype, rate, &need) != MGC_OK) throw Fail{MGC_EINVAL};
    if (!d_in || !d_out || !d_result) fail(MGC_EINVAL, "null pointer");
    if (reinterpret_cast<uintptr_t>(d_out) % 8 ||
        reinterpret_cast<uintptr_t>(d_in) % (dtype == MGC_F64 ? 8 : 4))
      fail(MGC_EINVAL, "misaligned input or output");
    if (out_cap < need) fail(MGC_ENOSPC, "output too small");
    hipStream_t s = as_stream(stream);
    ZfpHead h{};
    h.magic = kZfpMagic;
    h.dtype = (uint8_t)dtype;
    h.ndim = (uint8_t)ndim;
    h.maxbits = (uint32_t)std::nearbyint(rate * (double)(1u << (2 * ndim)));
    uint64_t nb = 1;
    for (int d = 0; d < ndim; ++d) {
      h.shape[d] = shape[d];
      nb *= (shape[d] + 3) / 4;
    }
    h.rate = rate;
    h.blocks = nb;
    h.total = need;
    uint8_t* out = static_cast<uint8_t*>(d_out);
    // blocks that share words OR their bits into a cleared payload
    if (h.maxbits % 64) MGC_HIP(hipMemsetAsync(out + kZfpHeaderBytes, 0, need - kZfpHeaderBytes, s));
    // d_result[0] serves as the non-finite flag until the header kernel
    // turns it into the outcome
    MGC_HIP(hipMemsetAsync(d_result, 0, 16, s));
    launch_zfp_encode(d_in, dtype == MGC_F64, ndim, shape, nb, h.maxbits, out,
                      reinterpret_cast<unsigned*>(d_result), h,
                      reinterpret_cast<unsigned long long*>(d_result), s);
    MGC_HIP(hipGetLastError());
  });
}

mgc_status mgc_zfp_parse_header(const void* h_header, size_t bytes, int* ndim,
                                uint64_t* shape3, mgc_dtype* dtype, double* rate,
                                uint64_t* stream_bytes) {
  return guard([&] {
    if (!h_header || bytes < (size_t)kZfpHeaderBytes) fail(MGC_EFORMAT, "stream shorter than its header");
    ZfpHead h;
    std::memcpy(&h, h_header, kZfpHeaderBytes);
    if (h.magic != kZfpMagic || h.dtype > 1 || h.ndim < 1 || h.ndim > 3)
      fail(MGC_EFORMAT, "not a fixed-rate block-coded stream");
    if (ndim) *ndim = h.ndim;
    if (shape3)
      for (int d = 0; d < 3; ++d) shape3[d] = d < h.ndim ? h.shape[d] : 0;
    if (dtype) *dtype = (mgc_dtype)h.dtype;
    if (rate) *rate = h.rate;
    if (stream_bytes) *stream_bytes = h.total;
  });
}

mgc_status mgc_zfp_decompress(mgc_ctx ctx, const void* d_in, size_t in_bytes, void* d_out,
                              size_t out_cap, void* stream) {
  return guard([&] {
    check_ctx(ctx);
    if (!d_in || !d_out) fail(MGC_EINVAL, "null pointer");
    if (reinterpret_cast<uintptr_t>(d_in) % 8) fail(MGC_EINVAL, "stream not 8-byte aligned");
    if (in_bytes < (size_t)kZfpHeaderBytes) fail(MGC_EFORMAT, "stream shorter than its header");
    hipStream_t s = as_stream(stream);
    sync_read(ctx, ctx->pinned, d_in, kZfpHeaderBytes, s);
    ZfpHead h;
    std::memcpy(&h, ctx->pinned, kZfpHeaderBytes);
    int nd = 0;
    uint64_t shp[3];
    mgc_dtype dt;
    double rate = 0;
    uint64_t total = 0;
    if (mgc_zfp_parse_header(&h, sizeof(h), &nd, shp, &dt, &rate, &total) != MGC_OK)
      fail(MGC_EFORMAT, "not a fixed-rate block-coded stream");
    size_t need = 0;
    if (mgc_zfp_query(nd, shp, dt, rate, &need) != MGC_OK || need != total ||
        h.maxbits != (uint32_t)std::nearbyint(rate * (double)(1u << (2 * nd))))
      fail(MGC_EFORMAT, "inconsistent header");
    if (total > in_bytes) fail(MGC_EFORMAT, "truncated stream");
    uint64_t n = 1;
    for (int d = 0; d < nd; ++d) n *= shp[d];
    if (reinterpret_cast<uintptr_t>(d_out) % (dt == MGC_F64 ? 8 : 4))
      fail(MGC_EINVAL, "misaligned output");
    if (out_cap < n * (dt == MGC_F64 ? 8 : 4)) fail(MGC_ENOSPC, "output too small");
    launch_zfp_decode(static_cast<const uint8_t*>(d_in), dt == MGC_F64, nd, shp, h.blocks,
                      h.maxbits, d_out, s);
    MGC_HIP(hipGetLastError());
  });
}

mgc_status mgc_hx_query(uint64_t n, mgc_hx_type type, uint32_t C, size_t* ws_bytes,
                        size_t* max_out_bytes) {
  return guard([&] {
    if (C < 64 || C > 65536 || C % 64) fail(MGC_EINVAL, "chunk size must be a multiple of 64 in [64, 65536]");
    if (type < MGC_HX_U8 || type > MGC_HX_I64) fail(MGC_EINVAL, "unknown Huffman-X value type");
    Carver c(nullptr);
    carve_hx(c, n, type, C);
    if (ws_bytes) *ws_bytes = c.off;
    if (max_out_bytes)
      *max_out_bytes = kHxHeaderBytes + huff_max_bytes(n, C) +
                       (hx_escapes(type) ? pad8(n * hx_width(type)) : 0);
  });
}

mgc_status mgc_hx_compress(mgc_ctx ctx, const void* d_in, uint64_t n, mgc_hx_type type,
                           uint32_t dict, int64_t base, uint32_t C, void* d_out, size_t out_cap,
                           void* d_ws, size_t ws_bytes, uint64_t* d_result, void* stream) {
  return guard([&] {
    check_ctx(ctx);
    int64_t lo = 0, hi = 0;
    hx_window(type, dict, base, &lo, &hi);
    size_t need_ws = 0, need_out = 0;
    if (mgc_hx_query(n, type, C, &need_ws, &need_out) != MGC_OK) throw Fail{MGC_EINVAL};
    if (n >= (1ull << 32)) fail(MGC_EUNSUPPORTED, "2^32 or more values");
    if (!d_out || !d_ws || !d_result || (n > 0 && !d_in)) fail(MGC_EINVAL, "null pointer");
    if (reinterpret_cast<uintptr_t>(d_in) % hx_width(type) ||
        reinterpret_cast<uintptr_t>(d_out) % 8)
      fail(MGC_EINVAL, "input not aligned to its value type or output not 8-byte aligned");
    if (ws_bytes < need_ws || out_cap < need_out) fail(MGC_ENOSPC, "workspace or output too small");
    hipStream_t s = as_stream(stream);
    Carver c(d_ws);
    const HxWs w = carve_hx(c, n, type, C);
    uint8_t* out = static_cast<uint8_t*>(d_out);
    uint8_t* sec = out + kHxHeaderBytes;
    const bool esc = hx_escapes(type);
    const uint64_t n_chunks = (n + C - 1) / C;
    if (n > 0) {
      MGC_HIP(hipMemsetAsync(w.huff.hist, 0, kDict * sizeof(unsigned), s));
      MGC_HIP(hipMemsetAsync(w.huff.lay, 0, sizeof(Layout), s));
      const uint16_t* key = static_cast<const uint16_t*>(d_in);
      if (type != MGC_HX_U16) {
        StageScope st(&ctx->prof, "hx_keys", s);
        launch_hx_keys(d_in, n, type, lo, hi, dict - 1, w.key, w.zc, s);
        key = w.key;
      }
      // histogram window: u8 keys from 0; otherwise centred on the key of
      // value 0 (the centre of the range for u16), escapes in the spare slot
      const int64_t k0 = type == MGC_HX_U16 ? (int64_t)kHalf
                         : lo > 0 ? 0 : lo < -(int64_t)kDict ? (int64_t)kDict : -lo;
      const int64_t wl = std::min<int64_t>(std::max<int64_t>(k0 - (int64_t)kHistWindow / 2, 0),
                                           (int64_t)(kDict - kHistWindow));
      huff_encode_enqueue(ctx, key, n, C, sec, w.huff, s,
                          type == MGC_HX_U8 ? 0u : (uint32_t)wl, esc ? dict - 1 : 0u);
      launch_huff_header(sec, C, n, n_chunks, w.huff.lay, w.info, s);
      if (esc) {
        StageScope st(&ctx->prof, "hx_escapes", s);
        launch_chunk_prefix(w.zc, w.zpre, w.sums, (int64_t)((n + 1023) / 1024), w.huff.lay, s);
        launch_hx_place(d_in, n, type, lo, hi, w.zc, w.zpre, sec, w.huff.lay, s);
      }
    }
    launch_hx_header(out, type, dict, C, base, n, (esc && n > 0) ? w.zc : nullptr,
                     (esc && n > 0) ? w.zpre : nullptr, w.huff.lay,
                     reinterpret_cast<unsigned long long*>(d_result), s);
    MGC_HIP(hipGetLastError());
  });
}

mgc_status mgc_hx_parse_header(const void* h_header, size_t bytes, mgc_hx_type* type,
                               uint64_t* n, uint32_t* dict, int64_t* base, uint32_t* C,
                               uint64_t* total) {
  return guard([&] {
    if (!h_header || bytes < (size_t)kHxHeaderBytes) fail(MGC_EFORMAT, "stream shorter than its header");
    const uint8_t* b = static_cast<const uint8_t*>(h_header);
    uint32_t magic, d, c;
    int64_t bs;
    uint64_t nn, tot;
    std::memcpy(&magic, b, 4);
    std::memcpy(&d, b + 8, 4);
    std::memcpy(&c, b + 12, 4);
    std::memcpy(&bs, b + 16, 8);
    std::memcpy(&nn, b + 24, 8);
    std::memcpy(&tot, b + 48, 8);
    if (magic != kHxMagic || b[4] > MGC_HX_I64) fail(MGC_EFORMAT, "not a Huffman-X stream");
    if (type) *type = static_cast<mgc_hx_type>(b[4]);
    if (n) *n = nn;
    if (dict) *dict = d;
    if (base) *base = bs;
    if (C) *C = c;
    if (total) *total = tot;
  });
}

mgc_status mgc_hx_decompress(mgc_ctx ctx, const void* d_in, size_t in_bytes, void* d_out,
                             uint64_t n, mgc_hx_type type, void* d_ws, size_t ws_bytes,
                             void* stream) {
  return guard([&] {
    check_ctx(ctx);
    if (!d_in || (n > 0 && !d_out)) fail(MGC_EINVAL, "null pointer");
    if (reinterpret_cast<uintptr_t>(d_in) % 8 ||
        reinterpret_cast<uintptr_t>(d_out) % hx_width(type))
      fail(MGC_EINVAL, "stream not 8-byte aligned or output not aligned to its value type");
    if (in_bytes < (size_t)kHxHeaderBytes) fail(MGC_EFORMAT, "stream shorter than its header");
    hipStream_t s = as_stream(stream);
    const size_t head = in_bytes >= (size_t)(kHxHeaderBytes + kHuffHeaderBytes)
                            ? kHxHeaderBytes + kHuffHeaderBytes : kHxHeaderBytes;
    sync_read(ctx, ctx->pinned, d_in, head, s);
    uint8_t hb[kHxHeaderBytes + kHuffHeaderBytes] = {};
    std::memcpy(hb, ctx->pinned, head);
    mgc_hx_type t;
    uint64_t hn, total, n_esc, secb;
    uint32_t dict, C;
    int64_t base;
    if (mgc_hx_parse_header(hb, head, &t, &hn, &dict, &base, &C, &total) != MGC_OK)
      fail(MGC_EFORMAT, "not a Huffman-X stream");
    std::memcpy(&n_esc, hb + 32, 8);
    std::memcpy(&secb, hb + 40, 8);
    if (t != type || hn != n) fail(MGC_EINVAL, "value type or count differs from the stream's");
    int64_t lo = 0, hi = 0;
    try {
      hx_window(type, dict, base, &lo, &hi);
    } catch (const Fail&) {
      fail(MGC_EFORMAT, "bad dictionary or base in the stream");
    }
    if (C < 64 || C > 65536 || C % 64) fail(MGC_EFORMAT, "bad chunk size in the stream");
    const bool esc = hx_escapes(type);
    const uint32_t width = hx_width(type);
    if (n_esc > n || (!esc && n_esc) || (n == 0 && secb) || secb % 8 ||
        total != kHxHeaderBytes + secb + pad8(n_esc * width) || total > in_bytes)
      fail(MGC_EFORMAT, "inconsistent Huffman-X stream lengths");
    size_t need_ws = 0;
    if (mgc_hx_query(n, type, C, &need_ws, nullptr) != MGC_OK) throw Fail{MGC_EINVAL};
    if (!d_ws || ws_bytes < need_ws) fail(MGC_ENOSPC, "workspace too small");
    if (n == 0) return;
    if (n >= (1ull << 32)) fail(MGC_EUNSUPPORTED, "2^32 or more values");
    if (head < (size_t)(kHxHeaderBytes + kHuffHeaderBytes)) fail(MGC_EFORMAT, "truncated stream");
    HuffHeader h;
    std::memcpy(&h, hb + kHxHeaderBytes, kHuffHeaderBytes);
    uint64_t off = 0, words = 0;
    check_huff_header(h, n, secb, &off, &words);
    if (h.C != C) fail(MGC_EFORMAT, "chunk sizes of the header and the coded section differ");
    Carver c(d_ws);
    const HxWs w = carve_hx(c, n, type, C);
    const uint8_t* sec = static_cast<const uint8_t*>(d_in) + kHxHeaderBytes;
    uint16_t* key = type == MGC_HX_U16 ? static_cast<uint16_t*>(d_out) : w.key;
    MGC_HIP(hipMemsetAsync(w.status, 0, 4 * sizeof(unsigned), s));
    {
      StageScope st(&ctx->prof, "decode_tables", s);
      launch_decode_tables(sec + kHuffHeaderBytes, h.n_codes, w.tables, w.status, s);
    }
    {
      StageScope st(&ctx->prof, "decode", s);
      ctx->dec_last = launch_decode(sec, off, words, h.n_chunks, h.n_words, (int)C, (int64_t)n,
                                    h.n_codes, w.tables, key, w.status, s, ctx->dec_force);
    }
    if (type != MGC_HX_U16) {
      StageScope st(&ctx->prof, "hx_values", s);
      if (esc) {
        MGC_HIP(hipMemsetAsync(w.lay0, 0, sizeof(Layout), s));
        launch_hx_count(key, n, dict - 1, w.zc, s);
        launch_chunk_prefix(w.zc, w.zpre, w.sums, (int64_t)((n + 1023) / 1024), w.lay0, s);
      }
      launch_hx_values(key, n, type, lo, (uint32_t)(hi - lo), dict - 1, sec + secb, n_esc, w.zc,
                       w.zpre, d_out, w.status, s);
    }
    MGC_HIP(hipGetLastError());
    unsigned st = 0;
    sync_read(ctx, ctx->pinned, w.status, sizeof(unsigned), s);
    std::memcpy(&st, ctx->pinned, sizeof(unsigned));
    if (st & ST_FORMAT) fail(MGC_EFORMAT, "corrupt coded data");
  });
}

mgc_status mgc_set_decoder(mgc_ctx ctx, int ring, int waves) {
  return guard([&] {
    if (!ctx) fail(MGC_EINVAL, "null context");
    if (ring < 0 || ring > 3) fail(MGC_EINVAL, "decoder ring must be 0..3");
    if (waves < 0 || waves > 16) fail(MGC_EINVAL, "decoder wavefronts must be 0..16");
    ctx->dec_force = DecodeShape{ring, waves};
  });
}

mgc_status mgc_decoder_info(mgc_ctx ctx, int* ring, int* waves) {
  return guard([&] {
    if (!ctx) fail(MGC_EINVAL, "null context");
    if (ring) *ring = ctx->dec_last.ring;
    if (waves) *waves = ctx->dec_last.waves;
  });
}

mgc_status mgc_profile_enable(mgc_ctx ctx, int enable) {
  return guard([&] {
    if (!ctx) fail(MGC_EINVAL, "null context");
    ctx->prof.enabled = enable != 0;
  });
}

mgc_status mgc_profile_reset(mgc_ctx ctx) {
  return guard([&] {
    if (!ctx) fail(MGC_EINVAL, "null context");
    MGC_HIP(hipSetDevice(ctx->device));
    ctx->prof.flush();
    std::fill(ctx->prof.ms.begin(), ctx->prof.ms.end(), 0.0);
    std::fill(ctx->prof.counts.begin(), ctx->prof.counts.end(), 0);
  });
}

mgc_status mgc_profile_read(mgc_ctx ctx, char* names, size_t names_cap, uint64_t* counts,
                            double* ms, int cap, int* n_stages) {
  return guard([&] {
    if (!ctx) fail(MGC_EINVAL, "null context");
    MGC_HIP(hipSetDevice(ctx->device));
    ctx->prof.flush();
    const int n = (int)ctx->prof.names.size();
    if (n_stages) *n_stages = n;
    std::string all;
    for (int i = 0; i < n; ++i) {
      if (i) all += '\n';
      all += ctx->prof.names[i];
      if (i < cap) {
        if (counts) counts[i] = ctx->prof.counts[i];
        if (ms) ms[i] = ctx->prof.ms[i];
      }
    }
    if (names && names_cap) {
      const size_t k = std::min(all.size(), names_cap - 1);
      std::memcpy(names, all.data(), k);
      names[k] = 0;
    }
  });
}

}  // extern "C"
