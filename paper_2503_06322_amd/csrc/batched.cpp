// Batched form: many arrays of uneven shapes (and bounds) compressed with one
// launch per stage over all of them, the whole sequence captured once into a
// HIP graph and replayed by a single graph launch per call.
//
// Every stage kernel of the plain compression has a batched twin that runs
// the same device code on a flattened list of blocks (array, block of the
// array), so each array's stream is bit-identical to what mgc_compress writes
// for it.  The per-array state lives in a device table of Job records; the
// error budget is derived on the device, so no host round trip sits between
// the stages.  Level loops run in steps: step s works on level L_j - s of
// every array j that still has one.
//
// Tile shapes of the three-axis decomposition kernel and the Thomas sweep
// widths have several candidates; on first use the autotuner times each on
// the caller's batch and keeps the fastest per kernel (outputs do not depend
// on the choice).
#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <limits>
#include <vector>

#include "host.hpp"

#pragma clang fp contract(off)

namespace mgc {

enum {
  TUNE_DEC_F32 = MGC_TUNE_DEC_F32,
  TUNE_DEC_F64 = MGC_TUNE_DEC_F64,
  TUNE_THOMAS_STRIDED = MGC_TUNE_THOMAS_STRIDED,
  TUNE_THOMAS_ROWS = MGC_TUNE_THOMAS_ROWS
};
constexpr int kTuneKinds = 4;
int tune_candidates(int kind) { return kind < 2 ? kDecCands : kThomasCands; }

// Candidates the autotuner compares: every tile shape of the decomposition
// kernel (identical results); the Thomas kinds stay at candidate 0 (the
// partitioned sweeps wherever lines fit), since candidates 1 and 2 force the
// serial sweeps, whose results agree only up to rounding.
int autotune_candidates(int kind) { return kind < 2 ? kDecCands : 1; }

enum class BK { Zero, Range, Budget, Dec, Thomas, ThomasPart, Level0, Hist, Codebook, ChunkW,
                Scan, OSort, Encode, Header };

struct BLaunch {
  BK kind;
  const char* name;
  int step = 0, axis = 0, D = 0;
  int part = 0, waves = 1;  // ThomasPart: class (thomas_part_class) and block wavefronts
  bool f32 = false;
  size_t map_off = 0;  // first entry of the launch in the map buffer
  uint32_t nb = 0;     // map entries (blocks)
  int tune = -1;       // tuning kind whose candidate the launch uses
};

struct BatchPlan {
  int n = 0;
  std::vector<const Plan*> plans;
  std::vector<mgc_dtype> dt;
  std::vector<int> ndim;
  std::vector<std::array<uint64_t, 3>> shape;
  std::vector<uint64_t> cap;
  std::vector<size_t> ws_off, out_off;
  size_t ws_total = 0, out_total = 0;
  Job* d_jobs = nullptr;
  Job* h_jobs = nullptr;  // pinned staging of the table
  std::vector<Job> last;  // table last uploaded
  bool uploaded = false;
  hipEvent_t up_ev = nullptr;    // after the last table upload
  hipEvent_t done_ev = nullptr;  // after the last run
  JobBlock* d_map = nullptr;
  std::vector<BLaunch> launches;
  int tune[kTuneKinds] = {-1, -1, -1, -1};  // candidates of the current maps and graph
  int autotuned[kTuneKinds] = {-1, -1, -1, -1};
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

void free_batch_plan(BatchPlan* b) {
  if (!b) return;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->d_jobs) (void)hipFree(b->d_jobs);
  if (b->d_map) (void)hipFree(b->d_map);
  if (b->h_jobs) (void)hipHostFree(b->h_jobs);
  if (b->up_ev) (void)hipEventDestroy(b->up_ev);
  if (b->done_ev) (void)hipEventDestroy(b->done_ev);
  delete b;
}

namespace {

static_assert(sizeof(Job) % 8 == 0, "job record without tail padding");

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

void check_batch_args(int n, const int* ndims, const uint64_t* shapes, const mgc_dtype* dtypes) {
  if (n < 1) fail(MGC_EINVAL, "a batch needs at least one array");
  if (!ndims || !shapes || !dtypes) fail(MGC_EINVAL, "null batch description");
  for (int j = 0; j < n; ++j)
    if (dtypes[j] != MGC_F32 && dtypes[j] != MGC_F64)
      fail(MGC_EINVAL, "array " + std::to_string(j) + ": dtype must be f32 or f64");
}

// Per-array workspace and output slot offsets (shared by the query and the call).
void layout_offsets(const std::vector<const Plan*>& plans, uint64_t outlier_cap,
                    std::vector<uint64_t>& cap, std::vector<size_t>& ws_off,
                    std::vector<size_t>& out_off, size_t& ws_total, size_t& out_total) {
  const size_t n = plans.size();
  cap.resize(n);
  ws_off.resize(n);
  out_off.resize(n);
  ws_total = out_total = 0;
  for (size_t j = 0; j < n; ++j) {
    const Plan& p = *plans[j];
    cap[j] = outlier_cap ? outlier_cap : default_outlier_cap(p.N);
    Carver c(nullptr);
    carve_compress(c, p, cap[j]);
    ws_off[j] = ws_total;
    ws_total += align256(c.off);
    out_off[j] = out_total;
    out_total += align256(max_stream_bytes(p, cap[j]));
  }
}

inline uint32_t ceil_div(int64_t a, int64_t b) { return (uint32_t)((a + b - 1) / b); }

uint32_t level0_blocks(int64_t m0) {
  int64_t b = (m0 + 255) / 256;
  return (uint32_t)std::min<int64_t>(std::max<int64_t>(b, 1), 65536);
}

// Launch list and block maps for the tuning choice t.
void build_launches(BatchPlan& b, const int t[kTuneKinds], std::vector<JobBlock>& map) {
  b.launches.clear();
  map.clear();
  const int n = b.n;
  auto per_job = [&](BK k, const char* name) {
    BLaunch L;
    L.kind = k;
    L.name = name;
    b.launches.push_back(L);
  };
  auto mapped = [&](BLaunch L, auto count) {
    L.map_off = map.size();
    for (int j = 0; j < n; ++j) {
      const uint32_t c = count(j);
      for (uint32_t k = 0; k < c; ++k) map.push_back(JobBlock{(uint32_t)j, k, c});
    }
    L.nb = (uint32_t)(map.size() - L.map_off);
    if (L.nb) b.launches.push_back(L);
  };
  auto live = [&](int j) { return b.plans[j]->N > 0; };

  per_job(BK::Zero, "b_zero");
  for (int f = 0; f < 2; ++f) {
    BLaunch L;
    L.kind = BK::Range;
    L.name = "b_range";
    L.f32 = f == 0;
    mapped(L, [&](int j) {
      return live(j) && (b.dt[j] == MGC_F32) == L.f32 ? range_blocks(b.plans[j]->N) : 0u;
    });
  }
  per_job(BK::Budget, "b_budget");
  int Lmax = 0;
  for (int j = 0; j < n; ++j) Lmax = std::max(Lmax, b.plans[j]->L);
  for (int s = 0; s < Lmax; ++s) {
    auto at = [&](int j) { return live(j) && b.plans[j]->L - s >= 1; };
    for (int D = 3; D >= 1; --D) {
      for (int f = 0; f < 2; ++f) {
        BLaunch L;
        L.kind = BK::Dec;
        L.name = s == 0 ? "b_dec_level[finest]" : "b_dec_level";
        L.step = s;
        L.D = D;
        L.f32 = f == 0;
        L.tune = D == 3 ? (L.f32 ? TUNE_DEC_F32 : TUNE_DEC_F64) : -1;
        const int cand = L.tune >= 0 ? t[L.tune] : 0;
        mapped(L, [&](int j) -> uint32_t {
          const Plan& p = *b.plans[j];
          if (!at(j) || p.D != D) return 0;
          const bool in_f32 = s == 0 && b.dt[j] == MGC_F32;
          if (in_f32 != L.f32) return 0;
          const PlanLevel& v = p.lv[p.L - s];
          const TileShape ts = dec_tile(D, in_f32, cand);
          return ceil_div(v.nc[0], ts.z) * ceil_div(v.nc[1], ts.y) * ceil_div(v.nc[2], ts.x);
        });
      }
    }
    for (int axis = 2; axis >= 0; --axis) {
      const int kind = axis == 2 ? TUNE_THOMAS_ROWS : TUNE_THOMAS_STRIDED;
      // the plain path's choice per array: serial sweeps for grids of the
      // one-launch grid kernel, for lines too long or when a candidate
      // forces them; the partitioned class otherwise
      auto cls = [&](int j) -> int {
        const Plan& p = *b.plans[j];
        if (t[kind] != 0) return kPartNone;
        const LevelGeom g = p.geom(p.L - s);
        if (thomas_grid_fits(g)) return kPartNone;
        const int c = thomas_part_class(axis, g.nc[axis]);
        return c == kPartScan && g.nc[2] > 256 ? kPartScanLong : c;
      };
      {
        BLaunch L;
        L.kind = BK::Thomas;
        L.name = s == 0 ? "b_thomas[finest]" : "b_thomas";
        L.step = s;
        L.axis = axis;
        L.tune = kind;
        mapped(L, [&](int j) -> uint32_t {
          const Plan& p = *b.plans[j];
          if (!at(j) || p.bit[axis] < 0 || cls(j) != kPartNone) return 0;
          const PlanLevel& v = p.lv[p.L - s];
          if (axis == 2) return ceil_div(v.nc[0] * v.nc[1], 64);
          if (axis == 1) return ceil_div(v.nc[0] * v.nc[2], 256);
          return ceil_div(v.nc[1] * v.nc[2], 256);
        });
      }
      for (int c : {kPart40, kPart64, kPartScan, kPartScanLong}) {
        if ((axis == 2) != (c >= kPartScan)) continue;
        BLaunch L;
        L.kind = BK::ThomasPart;
        L.name = s == 0 ? "b_thomas[finest]" : "b_thomas";
        L.step = s;
        L.axis = axis;
        L.part = c;
        const int seg = c == kPart40 ? 40 : 64;
        for (int j = 0; j < n; ++j) {
          const Plan& p = *b.plans[j];
          if (axis < 2 && at(j) && p.bit[axis] >= 0 && cls(j) == c)
            L.waves = std::max<int>(L.waves, (int)ceil_div(p.lv[p.L - s].nc[axis], seg));
        }
        mapped(L, [&](int j) -> uint32_t {
          const Plan& p = *b.plans[j];
          if (!at(j) || p.bit[axis] < 0 || cls(j) != c) return 0;
          const PlanLevel& v = p.lv[p.L - s];
          // (about four rows per wavefront: each wavefront loads its factors
          // once and the next row while it solves one)
          if (axis == 2) return std::min<uint32_t>(ceil_div(v.nc[0] * v.nc[1], 16), 1024);
          if (axis == 1) return ceil_div(v.nc[0] * v.nc[2], 64);
          return ceil_div(v.nc[1] * v.nc[2], 64);
        });
      }
    }
  }
  for (int f = 0; f < 2; ++f) {
    BLaunch L;
    L.kind = BK::Level0;
    L.name = "b_level0";
    L.f32 = f == 0;
    mapped(L, [&](int j) -> uint32_t {
      const Plan& p = *b.plans[j];
      if (!live(j)) return 0;
      const bool in_f32 = p.L == 0 && b.dt[j] == MGC_F32;
      return in_f32 == L.f32 ? level0_blocks(p.points(0)) : 0u;
    });
  }
  {
    BLaunch L;
    L.kind = BK::Hist;
    L.name = "b_histogram";
    // about 256K symbols per block: each block clears and flushes a
    // 32K-bin LDS window, which small slices would pay per few symbols
    mapped(L, [&](int j) {
      return live(j) ? (uint32_t)std::min<int64_t>(256, std::max<int64_t>(1, (b.plans[j]->N + 262143) / 262144))
                     : 0u;
    });
  }
  per_job(BK::Codebook, "b_codebook");
  {
    BLaunch L;
    L.kind = BK::ChunkW;
    L.name = "b_chunk_words";
    mapped(L, [&](int j) { return live(j) ? chunk_words_blocks(b.plans[j]->N, kChunk) : 0u; });
  }
  per_job(BK::Scan, "b_layout_scan");
  per_job(BK::OSort, "b_outlier_order");
  {
    BLaunch L;
    L.kind = BK::Encode;
    L.name = "b_encode";
    mapped(L, [&](int j) { return live(j) ? ceil_div(ceil_div(b.plans[j]->N, kChunk), 4) : 0u; });
  }
  per_job(BK::Header, "b_header");
}

void launch_one(const BatchPlan& b, const BLaunch& L, const int t[kTuneKinds], hipStream_t s) {
  const Job* J = b.d_jobs;
  const JobBlock* m = b.d_map + L.map_off;
  const int cand = L.tune >= 0 ? t[L.tune] : 0;
  switch (L.kind) {
    case BK::Zero: launch_b_zero(J, b.n, s); break;
    case BK::Range: launch_b_range(J, m, L.nb, L.f32, s); break;
    case BK::Budget: launch_b_budget(J, b.n, s); break;
    case BK::Dec: launch_b_dec_level(J, m, L.nb, L.step, L.D, L.f32, cand, s); break;
    case BK::Thomas: launch_b_thomas(L.axis, J, m, L.nb, L.step, cand, s); break;
    case BK::ThomasPart:
      launch_b_thomas_part(L.axis, L.part, L.waves, J, m, L.nb, L.step, s);
      break;
    case BK::Level0: launch_b_level0(J, m, L.nb, L.f32, s); break;
    case BK::Hist: launch_b_histogram(J, m, L.nb, s); break;
    case BK::Codebook: launch_b_codebook(J, b.n, s); break;
    case BK::ChunkW: launch_b_chunk_words(J, m, L.nb, s); break;
    case BK::Scan: launch_b_layout_scan(J, b.n, s); break;
    case BK::OSort: launch_b_escape_order(J, b.n, s); break;
    case BK::Encode: launch_b_encode(J, m, L.nb, s); break;
    case BK::Header: launch_b_header(J, b.n, s); break;
  }
}

// Every launch of the batch on stream s; optional per-launch stage timing,
// or per-tuning-kind times (ms, after a synchronisation) for the autotuner.
void run_eager(mgc_ctx ctx, const BatchPlan& b, hipStream_t s, std::vector<double>* kind_ms) {
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
  std::vector<int> ev_kind;
  for (const BLaunch& L : b.launches) {
    if (kind_ms && L.tune >= 0) {
      hipEvent_t e0, e1;
      MGC_HIP(hipEventCreate(&e0));
      MGC_HIP(hipEventCreate(&e1));
      MGC_HIP(hipEventRecord(e0, s));
      launch_one(b, L, b.tune, s);
      MGC_HIP(hipEventRecord(e1, s));
      ev.push_back({e0, e1});
      ev_kind.push_back(L.tune);
    } else {
      StageScope sc(kind_ms ? nullptr : &ctx->prof, L.name, s);
      launch_one(b, L, b.tune, s);
    }
  }
  MGC_HIP(hipGetLastError());
  if (kind_ms) {
    kind_ms->assign(kTuneKinds, 0.0);
    MGC_HIP(hipStreamSynchronize(s));
    for (size_t i = 0; i < ev.size(); ++i) {
      float ms = 0.f;
      MGC_HIP(hipEventElapsedTime(&ms, ev[i].first, ev[i].second));
      (*kind_ms)[ev_kind[i]] += ms;
    }
    for (auto& e : ev) {
      (void)hipEventDestroy(e.first);
      (void)hipEventDestroy(e.second);
    }
  }
}

// Rebuilds the block maps for tuning t (the graph is dropped).
void set_tuning(BatchPlan& b, const int t[kTuneKinds], hipStream_t s) {
  std::vector<JobBlock> map;
  build_launches(b, t, map);
  if (b.d_map) {
    MGC_HIP(hipStreamSynchronize(s));
    MGC_HIP(hipFree(b.d_map));
    b.d_map = nullptr;
  }
  MGC_HIP(hipMalloc(&b.d_map, std::max<size_t>(map.size(), 1) * sizeof(JobBlock)));
  if (!map.empty())
    MGC_HIP(hipMemcpy(b.d_map, map.data(), map.size() * sizeof(JobBlock), hipMemcpyHostToDevice));
  for (int k = 0; k < kTuneKinds; ++k) b.tune[k] = t[k];
  if (b.exec) {
    (void)hipGraphExecDestroy(b.exec);
    b.exec = nullptr;
  }
  if (b.graph) {
    (void)hipGraphDestroy(b.graph);
    b.graph = nullptr;
  }
}

void upload_jobs(BatchPlan& b, const std::vector<Job>& jobs, hipStream_t s) {
  const size_t bytes = jobs.size() * sizeof(Job);
  if (b.uploaded && std::memcmp(b.last.data(), jobs.data(), bytes) == 0) return;
  MGC_HIP(hipEventSynchronize(b.up_ev));  // the previous upload has read the staging
  std::memcpy(b.h_jobs, jobs.data(), bytes);
  MGC_HIP(hipStreamWaitEvent(s, b.done_ev, 0));  // the previous run has read the table
  MGC_HIP(hipMemcpyAsync(b.d_jobs, b.h_jobs, bytes, hipMemcpyHostToDevice, s));
  MGC_HIP(hipEventRecord(b.up_ev, s));
  b.last = jobs;
  b.uploaded = true;
}

void autotune(mgc_ctx ctx, BatchPlan& b, hipStream_t s) {
  std::vector<double> best(kTuneKinds, std::numeric_limits<double>::infinity());
  int choice[kTuneKinds] = {0, 0, 0, 0};
  int rounds = 0;
  for (int k = 0; k < kTuneKinds; ++k) rounds = std::max(rounds, autotune_candidates(k));
  for (int c = 0; c < rounds; ++c) {
    int t[kTuneKinds];
    for (int k = 0; k < kTuneKinds; ++k) t[k] = std::min(c, autotune_candidates(k) - 1);
    set_tuning(b, t, s);
    std::vector<double> ms;
    run_eager(ctx, b, s, &ms);  // warm-up
    run_eager(ctx, b, s, &ms);
    for (int k = 0; k < kTuneKinds; ++k)
      if (c < autotune_candidates(k) && ms[k] < best[k]) {
        best[k] = ms[k];
        choice[k] = c;
      }
  }
  for (int k = 0; k < kTuneKinds; ++k) b.autotuned[k] = choice[k];
}

BatchPlan* get_batch(mgc_ctx ctx, int n, const int* ndims, const uint64_t* shapes,
                     const mgc_dtype* dtypes, uint64_t outlier_cap) {
  std::vector<uint64_t> key{(uint64_t)n, outlier_cap};
  for (int j = 0; j < n; ++j) {
    key.push_back((uint64_t)ndims[j]);
    for (int d = 0; d < 3; ++d) key.push_back(shapes[3 * j + d]);
    key.push_back((uint64_t)dtypes[j]);
  }
  auto it = ctx->batches.find(key);
  if (it != ctx->batches.end()) return it->second;
  auto* b = new BatchPlan;
  try {
    b->n = n;
    for (int j = 0; j < n; ++j) {
      b->plans.push_back(&get_plan(ctx, ndims[j], shapes + 3 * j));
      b->dt.push_back(dtypes[j]);
      b->ndim.push_back(ndims[j]);
      b->shape.push_back({shapes[3 * j], shapes[3 * j + 1], shapes[3 * j + 2]});
    }
    layout_offsets(b->plans, outlier_cap, b->cap, b->ws_off, b->out_off, b->ws_total,
                   b->out_total);
    MGC_HIP(hipMalloc(&b->d_jobs, n * sizeof(Job)));
    MGC_HIP(hipHostMalloc((void**)&b->h_jobs, n * sizeof(Job), hipHostMallocDefault));
    MGC_HIP(hipEventCreateWithFlags(&b->up_ev, hipEventDisableTiming));
    MGC_HIP(hipEventCreateWithFlags(&b->done_ev, hipEventDisableTiming));
    MGC_HIP(hipEventRecord(b->up_ev, nullptr));
    MGC_HIP(hipEventRecord(b->done_ev, nullptr));
  } catch (...) {
    free_batch_plan(b);
    throw;
  }
  ctx->batches.emplace(key, b);
  return b;
}

}  // namespace
}  // namespace mgc

using namespace mgc;

extern "C" {

mgc_status mgc_batch_query(int n, const int* ndims, const uint64_t* shapes,
                           const mgc_dtype* dtypes, uint64_t outlier_cap, size_t* ws_bytes,
                           size_t* out_bytes, uint64_t* h_out_offsets) {
  return guard([&] {
    check_batch_args(n, ndims, shapes, dtypes);
    std::vector<Plan> plans;
    plans.reserve(n);
    for (int j = 0; j < n; ++j) plans.push_back(build_plan(ndims[j], shapes + 3 * j));
    std::vector<const Plan*> pp;
    for (auto& p : plans) pp.push_back(&p);
    std::vector<uint64_t> cap;
    std::vector<size_t> ws_off, out_off;
    size_t ws_total = 0, out_total = 0;
    layout_offsets(pp, outlier_cap, cap, ws_off, out_off, ws_total, out_total);
    if (ws_bytes) *ws_bytes = ws_total;
    if (out_bytes) *out_bytes = out_total;
    if (h_out_offsets)
      for (int j = 0; j < n; ++j) h_out_offsets[j] = out_off[j];
  });
}

mgc_status mgc_compress_batched(mgc_ctx ctx, int n, const void* const* d_in, const int* ndims,
                                const uint64_t* shapes, const mgc_dtype* dtypes,
                                const double* bounds, mgc_norm norm, mgc_mode mode,
                                uint64_t outlier_cap, void* d_out, size_t out_cap, void* d_ws,
                                size_t ws_bytes, uint64_t* d_sizes, int32_t* d_status,
                                int flags, void* stream) {
  return guard([&] {
    check_ctx(ctx);
    check_batch_args(n, ndims, shapes, dtypes);
    if (norm != MGC_LINF && norm != MGC_L2) fail(MGC_EINVAL, "norm must be L-inf or L2");
    if (mode != MGC_REL && mode != MGC_ABS) fail(MGC_EINVAL, "mode must be rel or abs");
    if (!d_in || !bounds || !d_out || !d_ws || !d_sizes || !d_status)
      fail(MGC_EINVAL, "null argument");
    if (flags & ~(MGC_BATCH_EAGER | MGC_BATCH_NO_TUNE)) fail(MGC_EINVAL, "unknown flags");
    for (int j = 0; j < n; ++j)
      if (!(bounds[j] > 0.0) || !std::isfinite(bounds[j]))
        fail(MGC_EINVAL, "array " + std::to_string(j) + ": bound must be positive and finite");
    BatchPlan& b = *get_batch(ctx, n, ndims, shapes, dtypes, outlier_cap);
    if (ws_bytes < b.ws_total) fail(MGC_ENOSPC, "workspace too small");
    if (out_cap < b.out_total) fail(MGC_ENOSPC, "output capacity too small");
    for (int j = 0; j < n; ++j)
      if (b.plans[j]->N > 0 && !d_in[j]) fail(MGC_EINVAL, "null input pointer");
    hipStream_t s = static_cast<hipStream_t>(stream);

    std::vector<Job> jobs(n);
    std::memset(jobs.data(), 0, n * sizeof(Job));
    for (int j = 0; j < n; ++j) {
      const Plan& p = *b.plans[j];
      Carver c(static_cast<uint8_t*>(d_ws) + b.ws_off[j]);
      const CompressWs w = carve_compress(c, p, b.cap[j]);
      Job& J = jobs[j];
      J.in = d_in[j];
      J.out = static_cast<uint8_t*>(d_out) + b.out_off[j];
      J.N = p.N;
      J.L = p.L;
      J.dtype = (int32_t)b.dt[j];
      J.cap = b.cap[j];
      J.n_chunks = (uint64_t)((p.N + kChunk - 1) / kChunk);
      J.key_bits = key_bits(p.N);
      J.geo = p.d_geo;
      J.bi.dtype = (int)b.dt[j];
      J.bi.norm = (int)norm;
      J.bi.mode = (int)mode;
      J.bi.L = p.L;
      J.bi.bound = bounds[j];
      J.bi.N = p.N;
      J.bi.K = p.d_K[norm == MGC_LINF ? 0 : 1];
      J.part = w.part;
      J.bud = w.bud;
      J.sym = w.sym;
      J.gA = w.gA;
      J.gB = w.gB;
      J.status = w.status;
      J.n_out = w.n_out;
      J.lay = w.lay;
      J.hist = w.hist;
      J.code = w.code;
      J.clen = w.clen;
      J.cbs = carve_codebook_scratch(w.cbs);
      J.cw = w.cw;
      J.opos = w.opos;
      J.oval = w.oval;
      J.okA = w.okA;
      J.ovA = w.ovA;
      J.okB = w.okB;
      J.ovB = w.ovB;
      J.zc = w.zc;
      J.zpre = w.zpre;
      J.zl = w.zl;
      J.size_out = d_sizes + j;
      J.status_out = d_status + j;
      J.hdr = make_header(p, b.ndim[j], b.shape[j].data(), b.dt[j], bounds[j], norm, mode);
    }
    upload_jobs(b, jobs, s);

    // tuning: forced candidates, else the autotuner's (run once per batch)
    bool need_tune = false;
    for (int k = 0; k < kTuneKinds; ++k)
      if (ctx->forced_tuning[k] < 0 && b.autotuned[k] < 0) need_tune = true;
    if (need_tune && !(flags & MGC_BATCH_NO_TUNE)) autotune(ctx, b, s);
    int want[kTuneKinds];
    for (int k = 0; k < kTuneKinds; ++k)
      want[k] = ctx->forced_tuning[k] >= 0 ? ctx->forced_tuning[k]
                                           : (b.autotuned[k] >= 0 ? b.autotuned[k] : 0);
    if (!std::equal(want, want + kTuneKinds, b.tune)) set_tuning(b, want, s);
    for (int k = 0; k < kTuneKinds; ++k) ctx->last_tuning[k] = b.tune[k];

    if (flags & MGC_BATCH_EAGER) {
      run_eager(ctx, b, s, nullptr);
    } else {
      if (!b.exec) {
        if (!ctx->capture_stream)
          MGC_HIP(hipStreamCreateWithFlags(&ctx->capture_stream, hipStreamNonBlocking));
        hipStream_t cs = ctx->capture_stream;
        MGC_HIP(hipStreamSynchronize(s));
        MGC_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
        try {
          for (const BLaunch& L : b.launches) launch_one(b, L, b.tune, cs);
        } catch (...) {
          hipGraph_t g = nullptr;
          (void)hipStreamEndCapture(cs, &g);
          if (g) (void)hipGraphDestroy(g);
          throw;
        }
        MGC_HIP(hipStreamEndCapture(cs, &b.graph));
        MGC_HIP(hipGraphInstantiate(&b.exec, b.graph, nullptr, nullptr, 0));
      }
      StageScope sc(&ctx->prof, "batched_graph", s);
      MGC_HIP(hipGraphLaunch(b.exec, s));
    }
    MGC_HIP(hipEventRecord(b.done_ev, s));
    MGC_HIP(hipGetLastError());
  });
}

mgc_status mgc_set_tuning(mgc_ctx ctx, int kind, int candidate) {
  return guard([&] {
    if (!ctx) fail(MGC_EINVAL, "null context");
    if (kind < 0 || kind >= kTuneKinds) fail(MGC_EINVAL, "unknown tuning kind");
    if (candidate < -1 || candidate >= tune_candidates(kind))
      fail(MGC_EINVAL, "candidate out of range");
    ctx->forced_tuning[kind] = candidate;
  });
}

mgc_status mgc_tuning_info(mgc_ctx ctx, int kind, int* n_candidates, int* last_choice) {
  return guard([&] {
    if (kind < 0 || kind >= kTuneKinds) fail(MGC_EINVAL, "unknown tuning kind");
    if (n_candidates) *n_candidates = tune_candidates(kind);
    if (last_choice) *last_choice = ctx ? ctx->last_tuning[kind] : -1;
  });
}

}  // extern "C"
