// Host-side internal interfaces of libdt (not part of the C ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "dt_common.hpp"

namespace dtk {

// Status plumbing: HIP failures become DT_E_DEVICE (or DT_E_NOMEM).
#define DT_HIP(call)                                                   \
  do {                                                                 \
    hipError_t e_ = (call);                                            \
    if (e_ != hipSuccess) return (e_ == hipErrorOutOfMemory) ? DT_E_NOMEM : DT_E_DEVICE; \
  } while (0)
#define DT_TRY(call)            \
  do {                          \
    int s_ = (call);            \
    if (s_ != DT_OK) return s_; \
  } while (0)

// Stream-ordered allocation: while a thread has an allocation stream set,
// DevBuf::alloc takes memory from the device's stream-ordered pool on that
// stream (no device-wide synchronisation at free, so concurrent calls on
// other streams keep running); otherwise plain hipMalloc/hipFree.  Every
// use of such a buffer must be on that stream.
hipStream_t alloc_stream();
struct AllocStreamScope {
  hipStream_t prev;
  explicit AllocStreamScope(hipStream_t s);
  ~AllocStreamScope();
};

// Workspace mode: while a thread has a workspace set, DevBuf::alloc and
// DevBuf::alloc_plain carve their memory from it (256-byte aligned, bump
// order) and never call an allocator; releasing the most recent block
// gives it back, any other release keeps its bytes until the workspace is
// reset.  All work of such a call runs on one stream, so a block reused
// after its release is ordered after every earlier use.
struct Workspace {
  char* base = nullptr;
  size_t cap = 0;
  size_t used = 0;
  size_t peak = 0;
};
Workspace* workspace();
struct WorkspaceScope {
  Workspace* prev;
  explicit WorkspaceScope(Workspace* w);
  ~WorkspaceScope();
};

// The stream every device operation of the current call runs on (set by
// the entry points for the duration of a call).
struct UseStreamScope {
  bool prev_set;
  hipStream_t prev;
  explicit UseStreamScope(hipStream_t s);
  ~UseStreamScope();
};
// Blocks released inside this scope carry no pending device work (every
// operation on them has been synchronised, e.g. a result being freed).
struct QuiescentScope {
  QuiescentScope();
  ~QuiescentScope();
};

// Large plain allocations go through a process-wide cache of device
// blocks: a released block is kept and handed out again for a request of
// about its size.  Repeated runs of one workload then reuse the same blocks
// instead of asking the driver for gigabytes per call, which on a busy
// machine can stall for seconds.  A block released during a call keeps an
// event recorded on the call's stream (after its last uses); the next call
// to take it makes its own stream wait for that event (or waits on the
// host when it has none), so no release synchronises the device.  A block
// released outside any call and not in a quiescent scope waits for its
// device to finish, as hipFree would.  *blk receives the block size (0:
// plain hipMalloc).
hipError_t cached_malloc(void** p, size_t n, size_t* blk);
void cached_free(void* p, size_t blk);

// Owning device buffer.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  size_t blk = 0;              // size of a cached block (0: not cached)
  hipStream_t ast = nullptr;   // stream of a stream-ordered allocation
  bool ordered = false;
  Workspace* ws = nullptr;     // carved from this workspace
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept
      : p(o.p), bytes(o.bytes), blk(o.blk), ast(o.ast), ordered(o.ordered), ws(o.ws) {
    o.p = nullptr;
    o.bytes = 0;
    o.blk = 0;
    o.ordered = false;
    o.ws = nullptr;
  }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) {
      release();
      p = o.p; bytes = o.bytes; blk = o.blk; ast = o.ast; ordered = o.ordered; ws = o.ws;
      o.p = nullptr; o.bytes = 0; o.blk = 0; o.ordered = false; o.ws = nullptr;
    }
    return *this;
  }
  ~DevBuf() { release(); }
  static size_t ws_round(size_t n) { return (n + 255) & ~(size_t)255; }
  void release() {
    if (p) {
      if (ws) {
        if (static_cast<char*>(p) + ws_round(bytes) == ws->base + ws->used)
          ws->used = static_cast<size_t>(static_cast<char*>(p) - ws->base);
      } else if (ordered) {
        (void)hipFreeAsync(p, ast);
      } else if (blk) {
        cached_free(p, blk);
      } else {
        (void)hipFree(p);
      }
    }
    p = nullptr;
    bytes = 0;
    blk = 0;
    ordered = false;
    ws = nullptr;
  }
  static int status_of(hipError_t e) { return e == hipErrorOutOfMemory ? DT_E_NOMEM : DT_E_DEVICE; }
  // Memory from the thread's workspace (see Workspace).
  int alloc_ws(Workspace* w, size_t n) {
    release();
    if (n == 0) n = 16;
    const size_t r = ws_round(n);
    if (w->used > w->cap || r > w->cap - w->used) return DT_E_NOMEM;
    p = w->base + w->used;
    w->used += r;
    if (w->used > w->peak) w->peak = w->used;
    bytes = n;
    ws = w;
    return DT_OK;
  }
  // Scratch memory (stream-ordered when the thread has an allocation stream).
  int alloc(size_t n) {
    if (Workspace* w = workspace()) return alloc_ws(w, n);
    hipStream_t s = alloc_stream();
    if (!s) return alloc_plain(n);
    release();
    if (n == 0) n = 16;
    hipError_t e = hipMallocAsync(&p, n, s);
    if (e != hipSuccess) { p = nullptr; return status_of(e); }
    bytes = n;
    ast = s;
    ordered = true;
    return DT_OK;
  }
  // Memory that outlives the call (result rows): never stream-ordered.
  int alloc_plain(size_t n) {
    if (Workspace* w = workspace()) return alloc_ws(w, n);
    release();
    if (n == 0) n = 16;
    hipError_t e = cached_malloc(&p, n, &blk);
    if (e != hipSuccess) { p = nullptr; blk = 0; return status_of(e); }
    bytes = n;
    return DT_OK;
  }
  template <class T> T* as() const { return static_cast<T*>(p); }
};

// A batch of point sets to triangulate with one sequence of launches.
// Points are device-resident as double4 (x, y, z or 0, key bits in w);
// key = global id, the perturbation order and output label.
struct LocalJob {
  int D = 3;
  uint32_t npts = 0;
  uint32_t nsets = 0;
  const double4* pts = nullptr;   // [npts]
  const uint32_t* pset = nullptr; // [npts] set of each point
  const uint32_t* set_off = nullptr;  // [nsets+1]
  bool fp32 = false;
  // launch tunables (timing only)
  uint32_t start_active = 256;    // active points per set in the first level
  uint32_t grow_div = 64;         // next level when pending < inserted / grow_div
  uint32_t cand_blocks = 32768;   // cap on cavity/insert wavefronts
  uint32_t grow_num = 0;          // threshold growth per level in eighths; 0: by set count
  bool seed = true;               // a large single set starts from a gift-wrapped seed
  void tune(const dt_options& o) {
    seed = o.gift_wrap >= 0;
    if (o.start_active > 0) start_active = (uint32_t)o.start_active;
    if (o.grow_div > 0) grow_div = (uint32_t)o.grow_div;
    if (o.cand_blocks > 0) cand_blocks = (uint32_t)o.cand_blocks;
    if (o.grow_num > 0) grow_num = (uint32_t)o.grow_num;
  }
};

// Cell pool: cells live at indices [0, ncells); cfwd == ALIVE marks a live
// cell, vertices are indices into the job's point array (INF_V = infinite).
struct CellPool {
  DevBuf cells;   // Cell[cap]
  uint32_t cap = 0;
  uint32_t ncells = 0;
  DevBuf set_cell0;   // [nsets] initial finite cell, DONE for a degenerate set
};

struct K4Stats {
  unsigned long long cavity_cells = 0;
  unsigned long long candidates = 0;
  unsigned long long verified = 0;    // cavity searches that completed
  int rounds = 0;
  uint32_t giant_rounds = 0;   // rounds in which a cavity used the pool-sized list
  uint32_t seeded = 0;         // 1: the set started from a gift-wrapped seed
  uint32_t maxcav = 0;
  unsigned long long pred[4][4] = {};
};

// Optional kernel timing: HIP events recorded around launches on the
// launch stream, resolved when the call finishes.  The active profiler is
// per host thread (one call at a time per thread).
struct Profiler {
  struct Rec { int id; hipEvent_t a, b; };
  std::vector<Rec> recs;
  double ms[DT_NUM_KERN] = {};
  long long launches[DT_NUM_KERN] = {};
  void begin(int id, hipStream_t st) {
    Rec r{id, nullptr, nullptr};
    if (hipEventCreate(&r.a) != hipSuccess || hipEventCreate(&r.b) != hipSuccess) return;
    (void)hipEventRecord(r.a, st);
    recs.push_back(r);
  }
  void end(hipStream_t st) {
    if (!recs.empty()) (void)hipEventRecord(recs.back().b, st);
  }
  void resolve() {
    for (auto& r : recs) {
      float t = 0.f;
      if (hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&t, r.a, r.b) == hipSuccess) {
        ms[r.id] += t;
        launches[r.id]++;
      }
      (void)hipEventDestroy(r.a);
      (void)hipEventDestroy(r.b);
    }
    recs.clear();
  }
};
Profiler* active_profiler();
void set_active_profiler(Profiler* p);
#define DT_PROF_BEGIN(id, st) \
  do { if (::dtk::active_profiler()) ::dtk::active_profiler()->begin((id), (st)); } while (0)
#define DT_PROF_END(st) \
  do { if (::dtk::active_profiler()) ::dtk::active_profiler()->end((st)); } while (0)

// Triangulate every set of `job` (one batched sequence of launches).
int k4_run(const LocalJob& job, CellPool& pool, Counters* dctr, Counters* hctr,
           hipStream_t st, K4Stats& ks);

// Compact the live finite cells of the pool to rows of D+1 keys (global
// ids, ascending inside a row).  rows may be null to only count.  If
// set_rows is non-null it receives per-set counts (nsets entries).
int k4_extract(const LocalJob& job, const CellPool& pool, int32_t* rows, uint32_t* count_dev,
               uint32_t* set_rows, hipStream_t st);

}  // namespace dtk
