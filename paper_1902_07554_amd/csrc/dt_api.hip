// C ABI entry points of libdt (declared in include/dt.h).
#include <string.h>

#include <algorithm>
#include <chrono>
#include <mutex>
#include <vector>

#include "dt_common.hpp"
#include "dt_internal.hpp"
#include "dt_pipeline.hpp"
#include "dt_prep.hpp"

using namespace dtk;

extern "C" void dt_default_options(dt_options* o) {
  if (!o) return;
  memset(o, 0, sizeof(*o));
  o->divide = DT_DIVIDE_SAMPLE;
  o->weight = DT_WEIGHT_LOG;
  o->precision = DT_PREC_FP64;
  o->sort_output = 0;
  o->eps = 0.05;
  o->grid_cell = 1.0;
  o->seed = 1;
  o->refine_iters = 16;
  o->keep_stages = 0;
  o->border = DT_BORDER_REGION;
}

extern "C" const char* dt_strerror(int s) {
  switch (s) {
    case DT_OK: return "ok";
    case DT_E_INVALID_ARG: return "invalid argument";
    case DT_E_NONFINITE: return "non-finite coordinate";
    case DT_E_DUPLICATE: return "duplicate point";
    case DT_E_DEGENERATE: return "degenerate input (too few points or all in one hyperplane)";
    case DT_E_NOMEM: return "out of device memory";
    case DT_E_DEVICE: return "HIP runtime error";
    case DT_E_INTERNAL: return "device invariant failed";
    case DT_E_NOT_READY: return "not ready";
    default: return "unknown status";
  }
}

namespace dtk {

// Cache of large device blocks (see cached_malloc).  Blocks of at least
// CACHE_MIN bytes are rounded up to CACHE_GRAIN; a request takes the
// smallest free block of its device that is at most a quarter larger.  At
// most CACHE_CAP bytes are kept; an allocation that fails first returns the
// kept blocks of its device to the driver.  The blocks are never freed at
// exit (the runtime may be gone by then; the process end releases them).
namespace {
constexpr size_t CACHE_MIN = size_t(16) << 20;
constexpr size_t CACHE_GRAIN = size_t(2) << 20;
constexpr size_t CACHE_CAP = size_t(48) << 30;
struct CachedBlock {
  void* p;
  size_t size;
  int dev;
  hipEvent_t ready;   // recorded after the block's last uses (null: none pending)
};
std::mutex g_cache_mu;
std::vector<CachedBlock>* g_cache = new std::vector<CachedBlock>();
size_t g_cached = 0;

struct UseStream {
  bool set = false;
  hipStream_t s = nullptr;
};
thread_local UseStream g_use;
thread_local int g_quiescent = 0;

void drop_block(const CachedBlock& b) {
  if (b.ready) (void)hipEventDestroy(b.ready);
  (void)hipFree(b.p);
}
}  // namespace

UseStreamScope::UseStreamScope(hipStream_t s) : prev_set(g_use.set), prev(g_use.s) {
  g_use.set = true;
  g_use.s = s;
}
UseStreamScope::~UseStreamScope() {
  g_use.set = prev_set;
  g_use.s = prev;
}
QuiescentScope::QuiescentScope() { g_quiescent++; }
QuiescentScope::~QuiescentScope() { g_quiescent--; }

hipError_t cached_malloc(void** p, size_t n, size_t* blk) {
  *blk = 0;
  if (n < CACHE_MIN) return hipMalloc(p, n);
  const size_t want = (n + CACHE_GRAIN - 1) / CACHE_GRAIN * CACHE_GRAIN;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  {
    std::lock_guard<std::mutex> g(g_cache_mu);
    size_t best = g_cache->size();
    for (size_t i = 0; i < g_cache->size(); i++) {
      const CachedBlock& b = (*g_cache)[i];
      if (b.dev == dev && b.size >= want && b.size - want <= want / 4 &&
          (best == g_cache->size() || b.size < (*g_cache)[best].size))
        best = i;
    }
    if (best < g_cache->size()) {
      const CachedBlock b = (*g_cache)[best];
      g_cached -= b.size;
      g_cache->erase(g_cache->begin() + best);
      *p = b.p;
      *blk = b.size;
      if (b.ready) {
        // order this call's work after the releasing call's last uses
        e = g_use.set ? hipStreamWaitEvent(g_use.s, b.ready, 0) : hipEventSynchronize(b.ready);
        (void)hipEventDestroy(b.ready);
        if (e != hipSuccess) {
          (void)hipFree(b.p);
          *p = nullptr;
          *blk = 0;
          return e;
        }
      }
      return hipSuccess;
    }
  }
  e = hipMalloc(p, want);
  if (e == hipErrorOutOfMemory) {
    (void)hipGetLastError();
    std::vector<CachedBlock> mine;
    {
      std::lock_guard<std::mutex> g(g_cache_mu);
      for (size_t i = 0; i < g_cache->size();) {
        if ((*g_cache)[i].dev == dev) {
          mine.push_back((*g_cache)[i]);
          g_cached -= (*g_cache)[i].size;
          g_cache->erase(g_cache->begin() + i);
        } else {
          i++;
        }
      }
    }
    for (const CachedBlock& b : mine) drop_block(b);
    e = hipMalloc(p, want);
  }
  if (e == hipSuccess) *blk = want;
  return e;
}

void cached_free(void* p, size_t blk) {
  // the block's own device (the current one may have changed since)
  hipPointerAttribute_t at;
  int cur = 0;
  if (hipPointerGetAttributes(&at, p) != hipSuccess || hipGetDevice(&cur) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipFree(p);
    return;
  }
  const int dev = at.device;
  hipEvent_t ready = nullptr;
  if (g_quiescent) {
    // every operation on the block has been synchronised
  } else if (g_use.set && dev == cur &&
             hipEventCreateWithFlags(&ready, hipEventDisableTiming) == hipSuccess) {
    // the block's uses are all on the call's stream: mark their end
    if (hipEventRecord(ready, g_use.s) != hipSuccess) {
      (void)hipEventDestroy(ready);
      ready = nullptr;
      (void)hipGetLastError();
      (void)hipDeviceSynchronize();
    }
  } else {
    // unknown stream: kernels queued on any stream of that device may
    // still use the block
    (void)hipGetLastError();
    if (dev != cur) (void)hipSetDevice(dev);
    (void)hipDeviceSynchronize();
    if (dev != cur) (void)hipSetDevice(cur);
  }
  std::vector<CachedBlock> drop;
  {
    std::lock_guard<std::mutex> g(g_cache_mu);
    g_cache->push_back({p, blk, dev, ready});
    g_cached += blk;
    // over the cap: return the largest blocks
    while (g_cached > CACHE_CAP && !g_cache->empty()) {
      size_t big = 0;
      for (size_t i = 1; i < g_cache->size(); i++)
        if ((*g_cache)[i].size > (*g_cache)[big].size) big = i;
      drop.push_back((*g_cache)[big]);
      g_cached -= (*g_cache)[big].size;
      g_cache->erase(g_cache->begin() + big);
    }
  }
  for (const CachedBlock& b : drop) drop_block(b);
}

int release_cached_memory() {
  std::vector<CachedBlock> all;
  {
    std::lock_guard<std::mutex> g(g_cache_mu);
    all.swap(*g_cache);
    g_cached = 0;
  }
  if (all.empty()) return DT_OK;
  int cur = 0;
  if (hipGetDevice(&cur) != hipSuccess) cur = -1;
  int status = DT_OK;
  std::sort(all.begin(), all.end(),
            [](const CachedBlock& x, const CachedBlock& y) { return x.dev < y.dev; });
  for (size_t i = 0; i < all.size(); i++) {
    if (i == 0 || all[i].dev != all[i - 1].dev) {
      if (hipSetDevice(all[i].dev) != hipSuccess || hipDeviceSynchronize() != hipSuccess)
        status = DT_E_DEVICE;
    }
    if (all[i].ready) (void)hipEventDestroy(all[i].ready);
    if (hipFree(all[i].p) != hipSuccess) status = DT_E_DEVICE;
  }
  if (cur >= 0 && hipSetDevice(cur) != hipSuccess) status = DT_E_DEVICE;
  return status;
}

// Pinned host words of the call contexts, kept per thread and reused
// (freeing pinned memory synchronises the device).
namespace {
struct PinnedCache {
  std::vector<void*> free_blocks;
  ~PinnedCache() {
    for (void* b : free_blocks) (void)hipHostFree(b);
  }
};
thread_local PinnedCache g_pinned;
constexpr size_t PINNED_BLOCK = 512;
static_assert(sizeof(Counters) + 16 <= PINNED_BLOCK, "pinned block too small");

// Host words of a call running in a workspace: plain (pageable) memory,
// so that such a call asks for no pinned allocation either; every copy
// into it is followed by a stream synchronisation before it is read.
alignas(64) thread_local char g_ws_host[PINNED_BLOCK];
}  // namespace

Ctx::~Ctx() {
  if (hctr && pinned) g_pinned.free_blocks.push_back(hctr);
}

int Ctx::init() {
  DT_TRY(dctr.alloc(sizeof(Counters)));
  DT_TRY(dflag.alloc(16));
  void* b = nullptr;
  if (workspace()) {
    b = g_ws_host;
    pinned = false;
  } else if (!g_pinned.free_blocks.empty()) {
    b = g_pinned.free_blocks.back();
    g_pinned.free_blocks.pop_back();
  } else {
    DT_HIP(hipHostMalloc(&b, PINNED_BLOCK, hipHostMallocDefault));
  }
  hctr = static_cast<Counters*>(b);
  hflag = reinterpret_cast<uint32_t*>(static_cast<char*>(b) + sizeof(Counters));
  return DT_OK;
}

static thread_local Workspace* g_workspace = nullptr;
Workspace* workspace() { return g_workspace; }
WorkspaceScope::WorkspaceScope(Workspace* w) : prev(g_workspace) { g_workspace = w; }
WorkspaceScope::~WorkspaceScope() { g_workspace = prev; }

static thread_local hipStream_t g_alloc_stream = nullptr;
hipStream_t alloc_stream() { return g_alloc_stream; }
AllocStreamScope::AllocStreamScope(hipStream_t s) : prev(g_alloc_stream) { g_alloc_stream = s; }
AllocStreamScope::~AllocStreamScope() { g_alloc_stream = prev; }

static thread_local Profiler* g_prof = nullptr;
Profiler* active_profiler() { return g_prof; }
void set_active_profiler(Profiler* p) { g_prof = p; }

double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

// Sort rows lexicographically on the host (verification output only).
int sort_rows_inplace(dt_result* r, hipStream_t st) {
  int w = r->D + 1;
  std::vector<int32_t> h((size_t)r->m * w);
  if (r->m == 0) return DT_OK;
  DT_HIP(hipMemcpyAsync(h.data(), r->rows.p, h.size() * 4, hipMemcpyDeviceToHost, st));
  DT_HIP(hipStreamSynchronize(st));
  std::vector<int64_t> idx((size_t)r->m);
  for (int64_t i = 0; i < r->m; i++) idx[i] = i;
  std::sort(idx.begin(), idx.end(), [&](int64_t a, int64_t b) {
    return std::lexicographical_compare(&h[a * w], &h[a * w] + w, &h[b * w], &h[b * w] + w);
  });
  std::vector<int32_t> o(h.size());
  for (int64_t i = 0; i < r->m; i++)
    for (int j = 0; j < w; j++) o[i * w + j] = h[idx[i] * w + j];
  DT_HIP(hipMemcpyAsync(r->rows.p, o.data(), o.size() * 4, hipMemcpyHostToDevice, st));
  DT_HIP(hipStreamSynchronize(st));
  return DT_OK;
}

int check_options(const dt_options* in, dt_options& o) {
  dt_default_options(&o);
  if (in) o = *in;
  if (o.divide < DT_DIVIDE_SAMPLE || o.divide > DT_DIVIDE_AUTO) return DT_E_INVALID_ARG;
  if (o.weight < 0 || o.weight > 3) return DT_E_INVALID_ARG;
  if (o.precision != DT_PREC_FP64 && o.precision != DT_PREC_FP32) return DT_E_INVALID_ARG;
  if (!(o.eps >= 0.0) || !(o.grid_cell > 0.0)) return DT_E_INVALID_ARG;
  if (o.refine_iters < 0) return DT_E_INVALID_ARG;
  if (o.border < DT_BORDER_REGION || o.border > DT_BORDER_REFINED) return DT_E_INVALID_ARG;
  if (o.start_active < 0 || o.start_active > (1 << 24)) return DT_E_INVALID_ARG;
  if (o.grow_div < 0 || o.grow_div > (1 << 20)) return DT_E_INVALID_ARG;
  if (o.cand_blocks < 0 || o.cand_blocks > (1 << 20)) return DT_E_INVALID_ARG;
  if (o.grow_num != 0 && (o.grow_num < 9 || o.grow_num > 32)) return DT_E_INVALID_ARG;
  if (o.recursive != 0 && o.recursive != 1) return DT_E_INVALID_ARG;
  if (o.gift_wrap != 0 && o.gift_wrap != -1) return DT_E_INVALID_ARG;
  if (o.refine_swaps != 0 && o.refine_swaps != -1) return DT_E_INVALID_ARG;
  return DT_OK;
}

}  // namespace dtk

extern "C" int dt_release_cached_memory(void) { return dtk::release_cached_memory(); }

extern "C" int dt_triangulate(const double* points, int64_t n, int D, int k, double sample_rate,
                              const dt_options* opt, int points_on_device, void* stream,
                              dt_result** out) {
  if (!out) return DT_E_INVALID_ARG;
  *out = nullptr;
  if ((D != 2 && D != 3) || n < 0 || n > 0x7FFFFFF0ll || k < 1 || !points) return DT_E_INVALID_ARG;
  if (!(sample_rate >= 0.0 && sample_rate <= 1.0)) return DT_E_INVALID_ARG;
  dt_options o;
  DT_TRY(check_options(opt, o));
  if (n < D + 1) return DT_E_DEGENERATE;
  hipStream_t st = (hipStream_t)stream;
  UseStreamScope use(st);
  dt_result* r = new dt_result();
  r->D = D;
  Profiler prof;
  if (o.profile) set_active_profiler(&prof);
  int s = run_triangulate(points, n, D, k, sample_rate, o, points_on_device != 0, st, r);
  set_active_profiler(nullptr);
  prof.resolve();
  for (int i = 0; i < DT_NUM_KERN; i++) {
    r->stats.kern_ms[i] = prof.ms[i];
    r->stats.kern_launches[i] = prof.launches[i];
  }
  if (s != DT_OK) {
    delete r;
    return s;
  }
  if (o.sort_output) {
    s = sort_rows_inplace(r, st);
    if (s != DT_OK) { delete r; return s; }
  }
  *out = r;
  return DT_OK;
}

extern "C" int dt_batch_triangulate(const double* points, const int64_t* ids,
                                    const int64_t* offsets, int64_t num_sets, int D,
                                    const dt_options* opt, int points_on_device, void* stream,
                                    dt_result** out) {
  if (!out) return DT_E_INVALID_ARG;
  *out = nullptr;
  if ((D != 2 && D != 3) || num_sets < 1 || !offsets || num_sets > 0x7FFFFFF0ll)
    return DT_E_INVALID_ARG;
  if (offsets[0] != 0) return DT_E_INVALID_ARG;
  for (int64_t s = 0; s < num_sets; s++)
    if (offsets[s + 1] < offsets[s]) return DT_E_INVALID_ARG;
  int64_t n = offsets[num_sets];
  if (n > 0x7FFFFFF0ll || (n > 0 && !points)) return DT_E_INVALID_ARG;
  dt_options o;
  DT_TRY(check_options(opt, o));
  hipStream_t st = (hipStream_t)stream;
  UseStreamScope use(st);
  dt_result* r = new dt_result();
  r->D = D;
  Profiler prof;
  if (o.profile) set_active_profiler(&prof);
  int s = run_batch(points, ids, offsets, num_sets, D, o, points_on_device != 0, st, r);
  set_active_profiler(nullptr);
  prof.resolve();
  for (int i = 0; i < DT_NUM_KERN; i++) {
    r->stats.kern_ms[i] = prof.ms[i];
    r->stats.kern_launches[i] = prof.launches[i];
  }
  if (s != DT_OK) {
    delete r;
    return s;
  }
  if (o.sort_output && num_sets == 1) {
    s = sort_rows_inplace(r, st);
    if (s != DT_OK) { delete r; return s; }
  }
  *out = r;
  return DT_OK;
}

extern "C" int64_t dt_result_count(const dt_result* r) { return r ? r->m : -1; }
extern "C" int dt_result_dim(const dt_result* r) { return r ? r->D : -1; }

extern "C" int dt_result_copy(const dt_result* r, int32_t* dst, int64_t cap_rows, int dst_on_device,
                              void* stream) {
  if (!r || (!dst && r->m > 0) || cap_rows < r->m) return DT_E_INVALID_ARG;
  if (r->m == 0) return DT_OK;
  hipStream_t st = (hipStream_t)stream;
  size_t bytes = (size_t)r->m * (r->D + 1) * 4;
  DT_HIP(hipMemcpyAsync(dst, r->rows.p, bytes,
                        dst_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, st));
  DT_HIP(hipStreamSynchronize(st));
  return DT_OK;
}

extern "C" int dt_result_neighbors(const dt_result* r, int32_t* dst, int64_t cap_rows,
                                   int dst_on_device, void* stream) {
  if (!r || (!dst && r->m > 0) || cap_rows < r->m) return DT_E_INVALID_ARG;
  if (r->m == 0) return DT_OK;
  hipStream_t st = (hipStream_t)stream;
  UseStreamScope use(st);
  if (!r->nbr_ready) {
    DT_TRY(compute_neighbors(*r, r->nbr, st));
    r->nbr_ready = true;
  }
  size_t bytes = (size_t)r->m * (r->D + 1) * 4;
  DT_HIP(hipMemcpyAsync(dst, r->nbr.p, bytes,
                        dst_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, st));
  DT_HIP(hipStreamSynchronize(st));
  return DT_OK;
}

extern "C" int dt_result_stats(const dt_result* r, dt_stats* s) {
  if (!r || !s) return DT_E_INVALID_ARG;
  *s = r->stats;
  return DT_OK;
}

extern "C" void dt_result_free(dt_result* r) {
  // every call that touches a result synchronises its stream before it
  // returns, so nothing is pending on the result's memory
  QuiescentScope q;
  delete r;
}

extern "C" int dt_result_set_offsets(const dt_result* r, int64_t* dst, int64_t cap) {
  if (!r || !dst || cap < (int64_t)r->set_offsets.size()) return DT_E_INVALID_ARG;
  for (size_t i = 0; i < r->set_offsets.size(); i++) dst[i] = r->set_offsets[i];
  return DT_OK;
}

extern "C" int dt_result_stage(const dt_result* r, int which, void* dst, int64_t cap,
                               int64_t* count) {
  if (!r || which < 0 || which >= DT_NUM_ARR || !count) return DT_E_INVALID_ARG;
  const std::vector<char>& a = r->stage[which];
  int64_t esz = (which == DT_ARR_SAMPLE || which == DT_ARR_WEIGHTS) ? 8 : 4;
  *count = (int64_t)a.size() / esz;
  if (!dst) return DT_OK;
  if (cap < *count) return DT_E_INVALID_ARG;
  memcpy(dst, a.data(), a.size());
  return DT_OK;
}
