// Host-side pieces shared by the plain entry points (api.cpp) and the
// batched form (batched.cpp): stage timing, workspace carving, the context.
#pragma once

#include <map>
#include <string>
#include <vector>

#include "kernels.hpp"
#include "plan.hpp"

namespace mgc {

struct Profiler {
  bool enabled = false;
  std::vector<std::string> names;
  std::map<std::string, int> slot_of;
  std::vector<double> ms;
  std::vector<uint64_t> counts;
  struct Pending {
    int slot;
    hipEvent_t a, b;
  };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> pool;

  int slot(const char* name) {
    auto it = slot_of.find(name);
    if (it != slot_of.end()) return it->second;
    int s = (int)names.size();
    names.push_back(name);
    slot_of[name] = s;
    ms.push_back(0.0);
    counts.push_back(0);
    return s;
  }
  hipEvent_t get() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e;
    MGC_HIP(hipEventCreate(&e));
    return e;
  }
  void flush() {
    for (auto& p : pending) {
      MGC_HIP(hipEventSynchronize(p.b));
      float t = 0.f;
      MGC_HIP(hipEventElapsedTime(&t, p.a, p.b));
      ms[p.slot] += t;
      counts[p.slot] += 1;
      pool.push_back(p.a);
      pool.push_back(p.b);
    }
    pending.clear();
  }
  ~Profiler() {
    for (auto& p : pending) {
      (void)hipEventDestroy(p.a);
      (void)hipEventDestroy(p.b);
    }
    for (auto e : pool) (void)hipEventDestroy(e);
  }
};

// bump allocator over a caller workspace (measure-only when base is null)
struct Carver {
  uint8_t* base;
  size_t off = 0;
  explicit Carver(void* b) : base(static_cast<uint8_t*>(b)) {}
  template <typename T>
  T* take(size_t n) {
    off = (off + 255) & ~size_t(255);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += n * sizeof(T);
    return p;
  }
};

constexpr uint32_t kChunk = kChunkSyms;

uint64_t default_outlier_cap(int64_t N);
int key_bits(int64_t N);

// Work buffers of one compression.
struct CompressWs {
  uint16_t* sym;
  double *gA, *gB, *part, *bud;
  unsigned* status;
  unsigned long long* n_out;
  Layout* lay;
  unsigned* hist;
  uint32_t* code;
  uint8_t* clen;
  void* cbs;
  uint32_t* cw;
  uint32_t* opos;
  int64_t* oval;
  uint32_t *okA, *ovA, *okB, *ovB;
  unsigned long long* info;
  uint32_t *zc, *zpre, *zsums, *zl;  // escape counts, their prefix, lane masks
};
CompressWs carve_compress(Carver& c, const Plan& p, uint64_t cap);
size_t max_stream_bytes(const Plan& p, uint64_t cap);
// Header fields known before the data is read (request, shape, counts).
Header make_header(const Plan& p, int ndim, const uint64_t* shape, mgc_dtype dtype,
                   double bound, mgc_norm norm, mgc_mode mode);

template <typename F>
mgc_status guard(F&& f) {
  try {
    f();
    return MGC_OK;
  } catch (const Fail& e) {
    return e.st;
  } catch (const std::exception& e) {
    set_error(e.what());
    return MGC_EDEVICE;
  }
}

struct BatchPlan;
void free_batch_plan(BatchPlan* b);

}  // namespace mgc

struct mgc_ctx_s {
  int device = 0;
  std::map<std::vector<uint64_t>, mgc::Plan> plans;
  mgc::Profiler prof;
  uint8_t* pinned = nullptr;      // 4 KiB host staging (pinned, mapped)
  uint8_t* pinned_dev = nullptr;  // the same memory as seen by the device
  // batched form: plans by batch signature, the stream graphs are captured
  // on, and tuning choices forced by the caller (-1 = autotune)
  std::map<std::vector<uint64_t>, mgc::BatchPlan*> batches;
  hipStream_t capture_stream = nullptr;
  int forced_tuning[4] = {-1, -1, -1, -1};
  int last_tuning[4] = {-1, -1, -1, -1};
  // decoder launch shape forced by the caller (0 = automatic) and the one
  // the latest decode used
  mgc::DecodeShape dec_force, dec_last;
};

namespace mgc {
void check_ctx(mgc_ctx ctx);
const Plan& get_plan(mgc_ctx ctx, int ndim, const uint64_t* shape);
// Decompression launches on stream s for a stream whose header and bins
// (the first head_bytes, at least 128 + 8 (L + 1)) the host already holds;
// returns the device status word the decoder sets (ST_FORMAT on corrupt
// data), or null when nothing was decoded (empty or constant arrays).
const unsigned* decompress_enqueue(mgc_ctx ctx, const uint8_t* head, size_t head_bytes,
                                   const void* d_in, size_t in_bytes, void* d_out,
                                   size_t out_cap, void* d_ws, size_t ws_bytes, hipStream_t s);
// Decompression workspace bytes of an array (its plan).
size_t decompress_ws_bytes(const Plan& p);
}  // namespace mgc
