// Host-resident arrays: the host-device pipeline of Section V.
//
// The execution model the paper assumes (one compute engine and two DMA
// engines per GPU) is what an MI355X exposes: kernels on one queue, host to
// device and device to host copies each on their own engine.  A chunk's three
// tasks (copy in, compress, copy out) run in order on one of three HIP
// streams, chunk i on stream i mod 3, so the copy in of chunk i+1 and the
// copy out of chunk i-1 overlap the kernels of chunk i.  Two input and two
// output buffers serve the three streams: chunk i+1's copy in waits for chunk
// i-1's kernels (the input buffer they read), chunk i's kernels wait for
// chunk i-2's copy out (the output buffer it reads); kernels of consecutive
// chunks never overlap (only one reduction at a time, as in the paper).
// The stream length of a chunk is known only when its kernels end: the host
// waits for it (through a one-block copy into mapped host memory, so the
// wait does not queue behind a copy engine), then enqueues the copy out of
// exactly that many bytes and the next chunk's kernels.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "host.hpp"

using namespace mgc;

namespace {

constexpr uint32_t kPipeMagic = 0x5043474Du;  // "MGCP"
constexpr size_t kPipeHead = 64;
constexpr size_t kPipeEntry = 32;
constexpr size_t kPinSlot = 2048;  // results read through ctx->pinned from this offset
constexpr uint64_t kDefaultInit = 64ull << 20;
constexpr uint64_t kDefaultLimit = 1ull << 30;

#pragma pack(push, 1)
struct PipeHead {
  uint32_t magic, n_chunks;
  uint8_t dtype, norm, mode, ndim;
  uint32_t z0;
  uint64_t shape[3];
  double bound, tau;
  uint64_t total;
};
struct PipeEntry {
  uint64_t first, planes, offset, bytes;
};
#pragma pack(pop)
static_assert(sizeof(PipeHead) == kPipeHead, "pipeline header is 64 bytes");
static_assert(sizeof(PipeEntry) == kPipeEntry, "pipeline entry is 32 bytes");

struct DevMem {
  void* p = nullptr;
  size_t n = 0;
  DevMem() = default;
  DevMem(const DevMem&) = delete;
  DevMem& operator=(const DevMem&) = delete;
  ~DevMem() {
    if (p) (void)hipFree(p);
  }
  void need(size_t bytes) {
    if (bytes <= n) return;
    if (p) MGC_HIP(hipFree(p));
    p = nullptr;
    n = 0;
    MGC_HIP(hipMalloc(&p, std::max<size_t>(bytes, 256)));
    n = bytes;
  }
};

struct Queues {
  hipStream_t q[3] = {nullptr, nullptr, nullptr};
  Queues() {
    for (auto& s : q) MGC_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
  }
  ~Queues() {
    for (auto s : q)
      if (s) (void)hipStreamDestroy(s);
  }
};

// Events of the timeline: one pair around each task.
struct Timeline {
  std::vector<hipEvent_t> ev;
  hipEvent_t base = nullptr;
  struct Task {
    int kind;  // 0 copy in, 1 kernels, 2 copy out
    hipEvent_t a, b;
  };
  std::vector<Task> tasks;
  Timeline() { MGC_HIP(hipEventCreate(&base)); }
  ~Timeline() {
    for (auto e : ev) (void)hipEventDestroy(e);
    if (base) (void)hipEventDestroy(base);
  }
  hipEvent_t make() {
    hipEvent_t e;
    MGC_HIP(hipEventCreate(&e));
    ev.push_back(e);
    return e;
  }
  // records a before the task's work on s and returns the pair's index
  size_t begin(int kind, hipStream_t s) {
    Task t{kind, make(), make()};
    MGC_HIP(hipEventRecord(t.a, s));
    tasks.push_back(t);
    return tasks.size() - 1;
  }
  void end(size_t i, hipStream_t s) { MGC_HIP(hipEventRecord(tasks[i].b, s)); }
  hipEvent_t done(size_t i) const { return tasks[i].b; }
  // seconds per kind and the overlap ratio, after everything finished
  void summarise(mgc_pipe_stats* st) const {
    std::vector<std::pair<double, double>> iv[3];
    for (const auto& t : tasks) {
      float a = 0.f, b = 0.f;
      MGC_HIP(hipEventElapsedTime(&a, base, t.a));
      MGC_HIP(hipEventElapsedTime(&b, base, t.b));
      iv[t.kind].push_back({a * 1e-3, b * 1e-3});
    }
    double sum[3] = {0, 0, 0};
    for (int k = 0; k < 3; ++k)
      for (auto& x : iv[k]) sum[k] += x.second - x.first;
    // copy time covered by kernel time (the kernels of one call never overlap)
    double covered = 0.0;
    for (int k : {0, 2})
      for (auto& c : iv[k])
        for (auto& r : iv[1]) {
          const double lo = std::max(c.first, r.first), hi = std::min(c.second, r.second);
          if (hi > lo) covered += hi - lo;
        }
    st->h2d_s = sum[0];
    st->kernel_s = sum[1];
    st->d2h_s = sum[2];
    st->overlap = sum[0] + sum[2] > 0 ? covered / (sum[0] + sum[2]) : 0.0;
  }
};

size_t esize(mgc_dtype dt) { return dt == MGC_F64 ? 8 : 4; }

uint64_t plane_values(int ndim, const uint64_t* shape) {
  uint64_t v = 1;
  for (int d = 1; d < ndim; ++d) v *= shape[d];
  return v;
}

void chunk_shape(int ndim, const uint64_t* shape, uint64_t planes, uint64_t* out) {
  for (int d = 0; d < ndim; ++d) out[d] = shape[d];
  out[0] = planes;
}

mgc_pipe_model resolve(const mgc_pipe_model* m) {
  mgc_pipe_model r{};
  if (m) r = *m;
  if (!r.init_chunk_bytes) r.init_chunk_bytes = kDefaultInit;
  if (!r.limit_chunk_bytes) r.limit_chunk_bytes = kDefaultLimit;
  if (r.limit_chunk_bytes < r.init_chunk_bytes) r.limit_chunk_bytes = r.init_chunk_bytes;
  return r;
}

// Phi(C): compression throughput (bytes/s) of a chunk of C bytes
double phi(const mgc_pipe_model& m, double C) {
  if (C >= (double)m.phi_threshold) return m.phi_gamma;
  return std::max(m.phi_alpha * C + m.phi_beta, 1.0);
}

// Next chunk size in bytes: the bytes the host can copy in while the current
// chunk compresses, never below the current size nor above the limit.
uint64_t next_bytes(const mgc_pipe_model& m, uint64_t cur) {
  if (!(m.phi_gamma > 0.0) || !(m.h2d_bytes_per_s > 0.0)) return cur;
  const double t = (double)cur / phi(m, (double)cur);
  const double c = t * m.h2d_bytes_per_s;
  return (uint64_t)std::min<double>(std::max<double>(c, (double)cur), (double)m.limit_chunk_bytes);
}

uint64_t planes_of(uint64_t bytes, uint64_t plane_bytes) {
  return std::max<uint64_t>(1, bytes / plane_bytes);
}

// Largest container for the array under the model's chunking (the smallest
// chunks are init_chunk_bytes; every chunk adds at most a one-plane
// stream's fixed part on top of its share of the whole array's bound).
size_t max_container(int ndim, const uint64_t* shape, mgc_dtype dt, const mgc_pipe_model& m) {
  const uint64_t pb = plane_values(ndim, shape) * esize(dt);
  const uint64_t init_planes = planes_of(m.init_chunk_bytes, pb);
  const uint64_t K = (shape[0] + init_planes - 1) / init_planes + 1;
  size_t whole = 0, one = 0;
  uint64_t s1[3];
  chunk_shape(ndim, shape, 1, s1);
  if (mgc_compress_query(ndim, shape, dt, 0, nullptr, &whole) != MGC_OK ||
      mgc_compress_query(ndim, s1, dt, 0, nullptr, &one) != MGC_OK)
    fail(MGC_EINVAL, "bad shape or dtype");
  return kPipeHead + whole + (size_t)K * (one + kPipeEntry + 8);
}

void check_request(int ndim, const uint64_t* shape, mgc_dtype dt, double bound, mgc_norm norm,
                   mgc_mode mode) {
  if (ndim < 1 || ndim > 3 || !shape) fail(MGC_EINVAL, "ndim must be 1..3");
  for (int d = 0; d < ndim; ++d)
    if (shape[d] == 0) fail(MGC_EINVAL, "empty arrays are not pipelined");
  if (dt != MGC_F32 && dt != MGC_F64) fail(MGC_EINVAL, "bad dtype");
  if (!(bound > 0.0) || !std::isfinite(bound)) fail(MGC_EINVAL, "error bound must be positive");
  if ((norm != MGC_LINF && norm != MGC_L2) || (mode != MGC_REL && mode != MGC_ABS))
    fail(MGC_EINVAL, "bad norm or mode");
}

// Reads n bytes of device memory through the mapped staging area (a kernel
// copy, so the read does not wait behind a copy engine), then waits.
void read_small(mgc_ctx ctx, void* host, const void* dev, size_t n, hipStream_t s) {
  launch_copy_bytes(ctx->pinned_dev + kPinSlot, dev, n, s);
  MGC_HIP(hipGetLastError());
  MGC_HIP(hipStreamSynchronize(s));
  std::memcpy(host, ctx->pinned + kPinSlot, n);
}

// min, max, sum of squares of the whole array: chunks streamed through the
// range pass on two streams.  With `resident` (a device copy of the whole
// array) the chunks are copied there and stay for the compression.
void range_prepass(mgc_ctx ctx, const uint8_t* h_in, int ndim, const uint64_t* shape,
                   mgc_dtype dt, uint64_t chunk_bytes, Queues& Q, double r[3],
                   uint8_t* resident) {
  const uint64_t pb = plane_values(ndim, shape) * esize(dt);
  const uint64_t cp = planes_of(chunk_bytes, pb);
  DevMem in[2], part, bud, st;
  if (!resident)
    for (auto& b : in) b.need(cp * pb);
  part.need(2 * 8 * 4 * (size_t)kRangeBlocks);
  bud.need(2 * 8 * 128);
  st.need(2 * 16);
  MGC_HIP(hipMemsetAsync(st.p, 0, 32, Q.q[0]));
  std::vector<double> acc;  // per chunk: min, max, sum of squares, bad
  DevMem res;
  const uint64_t nck = (shape[0] + cp - 1) / cp;
  res.need(nck * 32);
  MGC_HIP(hipStreamSynchronize(Q.q[0]));
  for (uint64_t k = 0; k < nck; ++k) {
    hipStream_t s = Q.q[k % 2];
    const uint64_t p0 = k * cp, np = std::min(cp, shape[0] - p0);
    void* dst = resident ? static_cast<void*>(resident + p0 * pb) : in[k % 2].p;
    MGC_HIP(hipMemcpyAsync(dst, h_in + p0 * pb, np * pb, hipMemcpyHostToDevice, s));
    BudgetIn b{};
    b.dtype = dt;
    b.norm = MGC_LINF;
    b.mode = MGC_ABS;
    b.L = -1;  // range only: no bins
    b.bound = 1.0;
    b.N = (int64_t)(np * (pb / esize(dt)));
    double* bd = static_cast<double*>(bud.p) + 128 * (k % 2);
    unsigned* sw = static_cast<unsigned*>(st.p) + 4 * (k % 2);
    // each of the two streams has its own partial sums, budget and status
    double* pt = static_cast<double*>(part.p) + (k % 2) * 4 * (size_t)kRangeBlocks;
    launch_range(dst, dt, b.N, pt, b, bd, sw, s);
    MGC_HIP(hipMemcpyAsync(static_cast<uint8_t*>(res.p) + 32 * k, bd, 32,
                           hipMemcpyDeviceToDevice, s));
  }
  for (auto s : Q.q) MGC_HIP(hipStreamSynchronize(s));
  std::vector<double> h(4 * nck);
  MGC_HIP(hipMemcpy(h.data(), res.p, 32 * nck, hipMemcpyDeviceToHost));
  double mn = h[0], mx = h[1], ss = 0.0, bad = 0.0;
  for (uint64_t k = 0; k < nck; ++k) {
    mn = std::min(mn, h[4 * k]);
    mx = std::max(mx, h[4 * k + 1]);
    ss += h[4 * k + 2];
    bad = std::max(bad, h[4 * k + 3]);
  }
  if (bad != 0.0) fail(MGC_EINVAL, "the data holds NaN or Inf");
  r[0] = mn;
  r[1] = mx;
  r[2] = ss;
}

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // namespace

extern "C" {

mgc_status mgc_pipe_max_bytes(int ndim, const uint64_t* shape, mgc_dtype dtype,
                              const mgc_pipe_model* model, size_t* max_out_bytes) {
  return guard([&] {
    if (ndim < 1 || ndim > 3 || !shape) fail(MGC_EINVAL, "ndim must be 1..3");
    const mgc_pipe_model m = resolve(model);
    const size_t b = max_container(ndim, shape, dtype, m);
    if (max_out_bytes) *max_out_bytes = b;
  });
}

mgc_status mgc_pipe_compress(mgc_ctx ctx, const void* h_in, int ndim, const uint64_t* shape,
                             mgc_dtype dtype, double error_bound, mgc_norm norm, mgc_mode mode,
                             const mgc_pipe_model* model, void* h_out, size_t out_cap,
                             uint64_t* h_out_size, mgc_pipe_stats* stats) {
  return guard([&] {
    check_ctx(ctx);
    check_request(ndim, shape, dtype, error_bound, norm, mode);
    if (!h_in || !h_out || !h_out_size) fail(MGC_EINVAL, "null pointer");
    const double t0 = now_s();
    const mgc_pipe_model m = resolve(model);
    uint64_t N = 1;
    for (int d = 0; d < ndim; ++d) N *= shape[d];
    const uint64_t pv = plane_values(ndim, shape), pb = pv * esize(dtype);
    const uint8_t* src = static_cast<const uint8_t*>(h_in);
    uint8_t* out = static_cast<uint8_t*>(h_out);
    Queues Q;
    mgc_pipe_stats st{};
    // Arrays that fit in a quarter of the free device memory stay resident
    // once copied: the chunks of a relative bound's range pass are then the
    // compression's input, and no chunk waits for an input buffer.
    DevMem Res;
    {
      size_t free_b = 0, total_b = 0;
      MGC_HIP(hipMemGetInfo(&free_b, &total_b));
      if (N * esize(dtype) <= free_b / 4) Res.need(N * esize(dtype));
    }
    const bool resident = Res.p != nullptr;
    // the absolute bound of the whole array
    double tau = error_bound;
    if (mode == MGC_REL) {
      const double a = now_s();
      double r[3];
      range_prepass(ctx, src, ndim, shape, dtype, m.limit_chunk_bytes, Q, r,
                    static_cast<uint8_t*>(Res.p));
      tau = norm == MGC_LINF ? error_bound * (r[1] - r[0]) : error_bound * std::sqrt(r[2]);
      if (r[1] == r[0]) tau = 1.0;  // constant array: every chunk stores its value
      st.prepass_s = now_s() - a;
      if (!(tau > 0.0)) fail(MGC_ERANGE, "the bound vanishes for this data");
    }
    // chunk plan: sizes follow the model as the chunks are issued
    std::vector<PipeEntry> ent;
    {
      uint64_t p0 = 0, cur = m.init_chunk_bytes;
      while (p0 < shape[0]) {
        const uint64_t np = std::min(planes_of(cur, pb), shape[0] - p0);
        ent.push_back({p0, np, 0, 0});
        p0 += np;
        cur = next_bytes(m, cur);
      }
    }
    const size_t K = ent.size();
    if (kPinSlot + 16 > 4096) fail(MGC_EDEVICE, "staging area");
    const size_t table = kPipeHead + K * kPipeEntry;
    if (out_cap < table) fail(MGC_ENOSPC, "output too small");
    // device buffers sized for the largest chunk
    uint64_t maxp = 0;
    for (auto& e : ent) maxp = std::max(maxp, e.planes);
    uint64_t cs[3];
    chunk_shape(ndim, shape, maxp, cs);
    size_t ws_n = 0, so_n = 0;
    if (mgc_compress_query(ndim, cs, dtype, 0, &ws_n, &so_n) != MGC_OK) throw Fail{MGC_EINVAL};
    DevMem I[2], O[2], W, R, OR;
    if (!resident)
      for (auto& b : I) b.need(maxp * pb);
    if (resident) {  // every chunk's stream in its own slot when they fit
      size_t free_b = 0, total_b = 0;
      MGC_HIP(hipMemGetInfo(&free_b, &total_b));
      if ((size_t)K * so_n <= free_b / 4) OR.need((size_t)K * so_n);
    }
    const bool out_resident = OR.p != nullptr;
    auto input_of = [&](size_t i) -> void* {
      return resident ? static_cast<void*>(static_cast<uint8_t*>(Res.p) + ent[i].first * pb)
                      : I[i % 2].p;
    };
    if (!out_resident)
      for (auto& b : O) b.need(so_n);
    W.need(ws_n);
    R.need(2 * 16);
    Timeline tl;
    MGC_HIP(hipDeviceSynchronize());
    MGC_HIP(hipEventRecord(tl.base, Q.q[0]));
    for (auto s : Q.q) MGC_HIP(hipStreamWaitEvent(s, tl.base, 0));
    std::vector<size_t> t_in(K), t_k(K), t_out(K);
    uint64_t off = pad8(table);
    const bool copied = resident && mode == MGC_REL;  // the range pass brought it in
    auto copy_in = [&](size_t i) {
      if (copied) return;
      hipStream_t s = Q.q[i % 3];
      if (i >= 2 && !resident) MGC_HIP(hipStreamWaitEvent(s, tl.done(t_k[i - 2]), 0));
      t_in[i] = tl.begin(0, s);
      MGC_HIP(hipMemcpyAsync(input_of(i), src + ent[i].first * pb, ent[i].planes * pb,
                             hipMemcpyHostToDevice, s));
      tl.end(t_in[i], s);
    };
    copy_in(0);
    for (size_t i = 0; i < K; ++i) {
      hipStream_t s = Q.q[i % 3];
      if (i + 1 < K) copy_in(i + 1);
      if (i >= 2 && !out_resident)
        MGC_HIP(hipStreamWaitEvent(s, tl.done(t_out[i - 2]), 0));  // output buffer free
      DevMem& Ob = O[i % 2];
      uint8_t* obuf = out_resident ? static_cast<uint8_t*>(OR.p) + i * so_n
                                   : static_cast<uint8_t*>(Ob.p);
      size_t ocap = out_resident ? so_n : Ob.n;
      chunk_shape(ndim, shape, ent[i].planes, cs);
      const double tc = norm == MGC_LINF
                            ? tau
                            : tau * std::sqrt((double)(ent[i].planes * pv) / (double)N);
      uint64_t* res = static_cast<uint64_t*>(R.p) + 2 * (i % 2);
      t_k[i] = tl.begin(1, s);
      mgc_status rc = mgc_compress(ctx, input_of(i), ndim, cs, dtype, tc, norm, MGC_ABS, 0,
                                   obuf, ocap, W.p, W.n, res, s);
      if (rc != MGC_OK) throw Fail{rc};
      uint64_t r2[2];
      read_small(ctx, r2, res, 16, s);
      if (r2[0] == MGC_ENOSPC) {
        // more escaped values than the default capacity: this chunk again
        const uint64_t cap = r2[1];
        size_t w2 = 0, o2 = 0;
        if (mgc_compress_query(ndim, cs, dtype, cap, &w2, &o2) != MGC_OK) throw Fail{MGC_EINVAL};
        // (a buffer of its own for this chunk's stream: nothing may still
        // read the one it replaces)
        for (auto q : Q.q) MGC_HIP(hipStreamSynchronize(q));
        Ob.need(o2);
        obuf = static_cast<uint8_t*>(Ob.p);
        ocap = Ob.n;
        W.need(w2);
        rc = mgc_compress(ctx, input_of(i), ndim, cs, dtype, tc, norm, MGC_ABS, cap, obuf, ocap,
                          W.p, W.n, res, s);
        if (rc != MGC_OK) throw Fail{rc};
        read_small(ctx, r2, res, 16, s);
      }
      tl.end(t_k[i], s);
      if (r2[0] != MGC_OK) fail((mgc_status)r2[0], "chunk compression failed");
      ent[i].offset = off;
      ent[i].bytes = r2[1];
      if (off + r2[1] > out_cap) fail(MGC_ENOSPC, "output too small");
      t_out[i] = tl.begin(2, s);
      MGC_HIP(hipMemcpyAsync(out + off, obuf, r2[1], hipMemcpyDeviceToHost, s));
      tl.end(t_out[i], s);
      off = pad8(off + r2[1]);
    }
    for (auto s : Q.q) MGC_HIP(hipStreamSynchronize(s));
    // header, table and the padding between streams
    PipeHead h{};
    h.magic = kPipeMagic;
    h.n_chunks = (uint32_t)K;
    h.dtype = (uint8_t)dtype;
    h.norm = (uint8_t)norm;
    h.mode = (uint8_t)mode;
    h.ndim = (uint8_t)ndim;
    for (int d = 0; d < ndim; ++d) h.shape[d] = shape[d];
    h.bound = error_bound;
    h.tau = tau;
    h.total = off;
    std::memcpy(out, &h, kPipeHead);
    std::memcpy(out + kPipeHead, ent.data(), K * kPipeEntry);
    std::memset(out + table, 0, pad8(table) - table);
    for (size_t i = 0; i < K; ++i) {
      const uint64_t e = ent[i].offset + ent[i].bytes;
      const uint64_t next = i + 1 < K ? ent[i + 1].offset : off;
      std::memset(out + e, 0, next - e);
    }
    *h_out_size = off;
    if (stats) {
      tl.summarise(&st);
      st.chunks = K;
      st.total_s = now_s() - t0;
      *stats = st;
    }
  });
}

mgc_status mgc_pipe_info(const void* h_in, size_t in_bytes, int* ndim, uint64_t* shape3,
                         mgc_dtype* dtype, uint64_t* total, uint64_t* chunks) {
  return guard([&] {
    if (!h_in || in_bytes < kPipeHead) fail(MGC_EFORMAT, "container shorter than its header");
    PipeHead h;
    std::memcpy(&h, h_in, kPipeHead);
    if (h.magic != kPipeMagic || h.ndim < 1 || h.ndim > 3 || h.dtype > 1)
      fail(MGC_EFORMAT, "bad container header");
    if (ndim) *ndim = h.ndim;
    if (shape3)
      for (int d = 0; d < 3; ++d) shape3[d] = d < h.ndim ? h.shape[d] : 0;
    if (dtype) *dtype = (mgc_dtype)h.dtype;
    if (total) *total = h.total;
    if (chunks) *chunks = h.n_chunks;
  });
}

mgc_status mgc_pipe_decompress(mgc_ctx ctx, const void* h_in, size_t in_bytes, void* h_out,
                               size_t out_cap, mgc_pipe_stats* stats) {
  return guard([&] {
    check_ctx(ctx);
    if (!h_in || !h_out) fail(MGC_EINVAL, "null pointer");
    const double t0 = now_s();
    const uint8_t* in = static_cast<const uint8_t*>(h_in);
    if (in_bytes < kPipeHead) fail(MGC_EFORMAT, "container shorter than its header");
    PipeHead h;
    std::memcpy(&h, in, kPipeHead);
    if (h.magic != kPipeMagic || h.ndim < 1 || h.ndim > 3 || h.dtype > 1 || h.n_chunks == 0 ||
        h.total > in_bytes || kPipeHead + (uint64_t)h.n_chunks * kPipeEntry > in_bytes)
      fail(MGC_EFORMAT, "bad container header");
    const int ndim = h.ndim;
    const mgc_dtype dt = (mgc_dtype)h.dtype;
    const uint64_t pv = plane_values(ndim, h.shape), pb = pv * esize(dt);
    const size_t K = h.n_chunks;
    std::vector<PipeEntry> ent(K);
    std::memcpy(ent.data(), in + kPipeHead, K * kPipeEntry);
    uint64_t p0 = 0, maxp = 0, maxs = 0;
    for (auto& e : ent) {
      if (e.first != p0 || e.planes == 0 || e.offset % 8 || e.offset + e.bytes > h.total ||
          e.bytes < (uint64_t)kHeaderBytes)
        fail(MGC_EFORMAT, "bad chunk table");
      p0 += e.planes;
      maxp = std::max(maxp, e.planes);
      maxs = std::max(maxs, e.bytes);
    }
    if (p0 != h.shape[0]) fail(MGC_EFORMAT, "chunks do not cover the array");
    if (out_cap < h.shape[0] * pb) fail(MGC_ENOSPC, "output too small");
    if (K > (4096 - kPinSlot) / 4) fail(MGC_EUNSUPPORTED, "too many chunks");
    size_t ws = 0;
    uint64_t cs[3];
    for (auto& e : ent) {
      chunk_shape(ndim, h.shape, e.planes, cs);
      ws = std::max(ws, decompress_ws_bytes(get_plan(ctx, ndim, cs)));
    }
    // With room (a quarter of the free device memory) the whole container
    // and the whole array live on the device, so no chunk waits for a
    // buffer; otherwise two input and two output buffers rotate.
    DevMem I[2], O[2], W, RI, RO;
    {
      size_t free_b = 0, total_b = 0;
      MGC_HIP(hipMemGetInfo(&free_b, &total_b));
      if (h.total + h.shape[0] * pb <= free_b / 4) {
        RI.need(h.total);
        RO.need(h.shape[0] * pb);
      }
    }
    const bool resident = RI.p != nullptr;
    if (!resident) {
      for (auto& b : I) b.need(maxs);
      for (auto& b : O) b.need(maxp * pb);
    }
    auto in_of = [&](size_t i) -> uint8_t* {
      return resident ? static_cast<uint8_t*>(RI.p) + ent[i].offset
                      : static_cast<uint8_t*>(I[i % 2].p);
    };
    auto out_of = [&](size_t i) -> uint8_t* {
      return resident ? static_cast<uint8_t*>(RO.p) + ent[i].first * pb
                      : static_cast<uint8_t*>(O[i % 2].p);
    };
    W.need(ws);
    uint8_t* out = static_cast<uint8_t*>(h_out);
    Queues Q;
    Timeline tl;
    MGC_HIP(hipDeviceSynchronize());
    MGC_HIP(hipEventRecord(tl.base, Q.q[0]));
    for (auto s : Q.q) MGC_HIP(hipStreamWaitEvent(s, tl.base, 0));
    std::vector<size_t> t_in(K), t_k(K), t_out(K);
    auto copy_in = [&](size_t i) {
      hipStream_t s = Q.q[i % 3];
      if (i >= 2 && !resident) MGC_HIP(hipStreamWaitEvent(s, tl.done(t_k[i - 2]), 0));
      t_in[i] = tl.begin(0, s);
      MGC_HIP(hipMemcpyAsync(in_of(i), in + ent[i].offset, ent[i].bytes,
                             hipMemcpyHostToDevice, s));
      tl.end(t_in[i], s);
    };
    unsigned* flags = reinterpret_cast<unsigned*>(ctx->pinned + kPinSlot);
    std::memset(flags, 0, 4 * K);
    copy_in(0);
    for (size_t i = 0; i < K; ++i) {
      hipStream_t s = Q.q[i % 3];
      if (i + 1 < K) copy_in(i + 1);
      if (i >= 1) MGC_HIP(hipStreamWaitEvent(s, tl.done(t_k[i - 1]), 0));  // one at a time
      if (i >= 2 && !resident) MGC_HIP(hipStreamWaitEvent(s, tl.done(t_out[i - 2]), 0));
      chunk_shape(ndim, h.shape, ent[i].planes, cs);
      Header ch;
      std::memcpy(&ch, in + ent[i].offset, kHeaderBytes);
      if (ch.ndim != ndim || ch.shape[0] != cs[0] || (ndim > 1 && ch.shape[1] != cs[1]) ||
          (ndim > 2 && ch.shape[2] != cs[2]) || ch.dtype != h.dtype)
        fail(MGC_EFORMAT, "chunk shape differs from the table");
      // the chunk's header is parsed from the host copy: no device read
      const size_t head = std::min<size_t>(ent[i].bytes, kHeaderBytes + 8 * (kMaxLevels + 1));
      t_k[i] = tl.begin(1, s);
      const unsigned* sw = decompress_enqueue(ctx, in + ent[i].offset, head, in_of(i),
                                              ent[i].bytes, out_of(i), ent[i].planes * pb, W.p,
                                              W.n, s);
      if (sw) launch_copy_bytes(ctx->pinned_dev + kPinSlot + 4 * i, sw, 4, s);
      tl.end(t_k[i], s);
      t_out[i] = tl.begin(2, s);
      MGC_HIP(hipMemcpyAsync(out + ent[i].first * pb, out_of(i), ent[i].planes * pb,
                             hipMemcpyDeviceToHost, s));
      tl.end(t_out[i], s);
    }
    for (auto s : Q.q) MGC_HIP(hipStreamSynchronize(s));
    for (size_t i = 0; i < K; ++i)
      if (flags[i] & ST_FORMAT) fail(MGC_EFORMAT, "corrupt coded data in a chunk");
    if (stats) {
      mgc_pipe_stats st{};
      tl.summarise(&st);
      st.chunks = K;
      st.total_s = now_s() - t0;
      *stats = st;
    }
  });
}

mgc_status mgc_pipe_profile(mgc_ctx ctx, const void* h_in, int ndim, const uint64_t* shape,
                            mgc_dtype dtype, double error_bound, mgc_norm norm, mgc_mode mode,
                            mgc_pipe_model* model) {
  return guard([&] {
    check_ctx(ctx);
    check_request(ndim, shape, dtype, error_bound, norm, mode);
    if (!h_in || !model) fail(MGC_EINVAL, "null pointer");
    mgc_pipe_model m = resolve(model);
    const uint64_t pb = plane_values(ndim, shape) * esize(dtype);
    // profiled sizes: the limit (or the array) halved down to about 1 MiB
    const uint64_t top = std::min<uint64_t>(planes_of(m.limit_chunk_bytes, pb), shape[0]);
    std::vector<uint64_t> sizes;
    for (uint64_t p = top; p >= 1; p /= 2) {
      sizes.push_back(p);
      if (p * pb < (1ull << 20)) break;
    }
    hipStream_t s;
    MGC_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    struct StreamGuard {
      hipStream_t s;
      ~StreamGuard() { (void)hipStreamDestroy(s); }
    } sg{s};
    uint64_t cs[3];
    chunk_shape(ndim, shape, top, cs);
    size_t ws_n = 0, so_n = 0;
    if (mgc_compress_query(ndim, cs, dtype, 0, &ws_n, &so_n) != MGC_OK) throw Fail{MGC_EINVAL};
    DevMem I, O, W, R;
    I.need(top * pb);
    O.need(so_n);
    W.need(ws_n);
    R.need(16);
    hipEvent_t a, b;
    MGC_HIP(hipEventCreate(&a));
    MGC_HIP(hipEventCreate(&b));
    struct EvGuard {
      hipEvent_t a, b;
      ~EvGuard() {
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
      }
    } eg{a, b};
    // copy bandwidth: the largest sample, twice (the first pages the
    // buffer in)
    float ms = 0.f;
    for (int rep = 0; rep < 2; ++rep) {
      MGC_HIP(hipEventRecord(a, s));
      MGC_HIP(hipMemcpyAsync(I.p, h_in, top * pb, hipMemcpyHostToDevice, s));
      MGC_HIP(hipEventRecord(b, s));
      MGC_HIP(hipEventSynchronize(b));
      MGC_HIP(hipEventElapsedTime(&ms, a, b));
    }
    m.h2d_bytes_per_s = (double)(top * pb) / (ms * 1e-3);
    // Phi at each size: the chunk's compression with the whole array's
    // bound treated as absolute for the chunk (a relative bound is kept
    // relative: the throughput, not the stream, is what is measured)
    std::vector<double> thr(sizes.size());
    for (size_t k = 0; k < sizes.size(); ++k) {
      chunk_shape(ndim, shape, sizes[k], cs);
      float best = 1e30f;
      for (int rep = 0; rep < 3; ++rep) {
        MGC_HIP(hipEventRecord(a, s));
        const mgc_status rc = mgc_compress(ctx, I.p, ndim, cs, dtype, error_bound, norm, mode, 0,
                                           O.p, O.n, W.p, W.n, static_cast<uint64_t*>(R.p), s);
        if (rc != MGC_OK) throw Fail{rc};
        MGC_HIP(hipEventRecord(b, s));
        MGC_HIP(hipEventSynchronize(b));
        MGC_HIP(hipEventElapsedTime(&ms, a, b));
        if (rep > 0) best = std::min(best, ms);
      }
      thr[k] = (double)(sizes[k] * pb) / (best * 1e-3);
    }
    // gamma from the largest size; the threshold is the smallest size whose
    // throughput stays within f = 0.1 of gamma; a least-squares line through
    // the sizes below it
    const double f = 0.1;
    m.phi_gamma = thr[0];
    size_t k_thr = 0;
    while (k_thr + 1 < sizes.size() && thr[k_thr + 1] >= (1.0 - f) * m.phi_gamma) ++k_thr;
    m.phi_threshold = sizes[k_thr] * pb;
    std::vector<std::pair<double, double>> pts;
    for (size_t k = k_thr + 1; k < sizes.size(); ++k) pts.push_back({(double)(sizes[k] * pb), thr[k]});
    if (pts.size() >= 2) {
      double sx = 0, sy = 0, sxx = 0, sxy = 0;
      for (auto& p : pts) {
        sx += p.first;
        sy += p.second;
        sxx += p.first * p.first;
        sxy += p.first * p.second;
      }
      const double n = (double)pts.size();
      const double den = n * sxx - sx * sx;
      m.phi_alpha = den != 0.0 ? (n * sxy - sx * sy) / den : 0.0;
      m.phi_beta = (sy - m.phi_alpha * sx) / n;
    } else if (pts.size() == 1) {
      m.phi_alpha = 0.0;
      m.phi_beta = pts[0].second;
    } else {
      m.phi_alpha = 0.0;
      m.phi_beta = m.phi_gamma;
    }
    *model = m;
  });
}

}  // extern "C"
