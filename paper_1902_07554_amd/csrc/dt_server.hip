// Serving: continuous batching of triangulation jobs under a device-memory
// budget.
//
// A job's points are copied to device memory when it is submitted and stay
// there until it finishes.  A job is admitted (FIFO) when its estimated
// footprint fits the remaining budget.  Two worker threads, each with its
// own HIP stream, repeatedly take the admitted jobs that have not started:
// a run of consecutive jobs of at most DIRECT_MAX points (whatever their k)
// is triangulated together as one batched run of independent sets (all of
// them share every kernel launch); a larger job runs on its own with its
// divide-and-conquer.  Jobs that arrive while a batch runs are admitted as
// memory frees up and start with the next batch, which may run concurrently
// with the other workers' batches.  A job's result is DT of its own points
// labelled by row index, with the row index as tie-break order: what
// dt_triangulate returns for it alone, since the triangulation depends only
// on the point set.  If a batched run fails, its jobs run again one by one
// so that each gets its own status.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "dt_common.hpp"
#include "dt_internal.hpp"
#include "dt_pipeline.hpp"

using namespace dtk;

#define DT_HIP_DEL(call, obj)   \
  do {                          \
    if ((call) != hipSuccess) { \
      delete (obj);             \
      return DT_E_DEVICE;       \
    }                           \
  } while (0)

namespace {

struct Job {
  uint64_t ticket = 0;
  int64_t n = 0;
  int D = 3, k = 1;
  double rate = 0.0;
  DevBuf dev;                  // points (device copy, n x D doubles)
  size_t footprint = 0;
  double t[3] = {0, 0, 0};    // submitted, admitted, done
  int status = DT_OK;
  dt_result* res = nullptr;
  bool admitted = false, started = false, done = false;
};

double mono_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// Estimated device bytes of one job: point records, input copy, cell pool
// (12 or 40 cells of 64 B per point), location and candidate buffers; the
// divide-and-conquer path also holds the bucketed copy, the border pool and
// the merge table.
size_t footprint_of(int64_t n, int D, int k) {
  size_t per = (D == 3) ? (32 + 24 + 40 * 64 + 1600) : (32 + 16 + 12 * 64 + 900);
  if (k > 1) per += per / 2 + 64;
  return (size_t)n * per + (64u << 20);
}

// Up to 32 Mi points per batched run: a batch's rounds are about those of
// its largest set, so larger batches amortise them (64 Mi no longer fits
// the device with its cell pool).
constexpr int64_t MAX_BATCH_POINTS = 32 << 20;
// Jobs up to this size join batched runs of independent sets: one set of a
// batch costs far less than a divide-and-conquer run of its own, whose
// rounds are latency-bound (the result is the same either way).
constexpr int64_t DIRECT_MAX = 1 << 21;
// Two workers: a batch can start while another runs.  Measured on the
// Poisson stream of 3D jobs (200 jobs/s, n log-uniform in [1e3, 1e6]): two
// workers with 32 Mi-point batches served 16.3 Mpoints/s, four workers 10.7
// (the rounds of four batches contend for the device) and four workers with
// 8 Mi-point batches 9.2.
constexpr int NUM_WORKERS = 2;

}  // namespace

struct dt_server {
  size_t budget = 0, used = 0;
  dt_options opt{};
  double t0 = 0;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Job*> waiting;     // submitted, not admitted
  std::deque<Job*> ready;       // admitted, not started
  std::map<uint64_t, Job*> jobs;
  std::vector<std::thread> workers;
  bool stop = false;
  uint64_t next = 1;
  int device = 0;
  bool trace = false;   // DT_DEBUG set: one line per batch on stderr

  // admit from the front while the budget allows (called with mu held)
  void admit() {
    while (!waiting.empty()) {
      Job* j = waiting.front();
      if (used + j->footprint > budget && used > 0) break;
      waiting.pop_front();
      used += j->footprint;
      j->admitted = true;
      j->t[1] = mono_s() - t0;
      ready.push_back(j);
    }
  }

  // Finish job j from a standalone run (own status, own statistics).
  void run_alone(Job* j, hipStream_t st) {
    dt_result* r = new dt_result();
    r->D = j->D;
    const int k = j->n <= DIRECT_MAX ? 1 : j->k;
    int s = run_triangulate(j->dev.as<double>(), j->n, j->D, k, j->rate, opt, true, st, r);
    if (s == DT_OK && opt.sort_output) s = sort_rows_inplace(r, st);
    if (s != DT_OK) {
      delete r;
      r = nullptr;
    }
    j->status = s;
    j->res = r;
  }

  // Split row range [a, e) of a batched result into job j's own result.
  int split_out(Job* j, const dt_result& all, int64_t a, int64_t e, hipStream_t st) {
    int D = j->D;
    dt_result* r = new dt_result();
    r->D = D;
    r->m = e - a;
    r->set_offsets = {0, r->m};
    r->stats = all.stats;
    r->stats.n = j->n;
    r->stats.k = 1;
    r->stats.num_simplices = r->m;
    r->stats.local_simplices = r->m;
    r->stats.max_part = r->stats.min_part = j->n;
    int s = r->rows.alloc_plain((size_t)r->m * (D + 1) * 4);
    if (s == DT_OK && r->m > 0) {
      hipError_t he = hipMemcpyAsync(r->rows.p, all.rows.as<int32_t>() + (size_t)a * (D + 1),
                                     (size_t)r->m * (D + 1) * 4, hipMemcpyDeviceToDevice, st);
      if (he == hipSuccess) he = hipStreamSynchronize(st);
      if (he != hipSuccess) s = DT_E_DEVICE;
    }
    if (s == DT_OK && r->m == 0) s = DT_E_DEGENERATE;
    if (s == DT_OK && opt.sort_output) s = sort_rows_inplace(r, st);
    if (s != DT_OK) {
      delete r;
      r = nullptr;
    }
    j->status = s;
    j->res = r;
    return s;
  }

  void run_batch_of(std::vector<Job*>& b, hipStream_t st) {
    if (b.size() == 1) {
      run_alone(b[0], st);
      return;
    }
    int D = b[0]->D;   // a batch holds jobs of one dimension
    std::vector<int64_t> off(b.size() + 1, 0);
    for (size_t i = 0; i < b.size(); i++) off[i + 1] = off[i] + b[i]->n;
    // the jobs' points side by side (device to device); every point is
    // labelled by its index inside its job
    DevBuf pts;
    int s = pts.alloc((size_t)off.back() * D * 8);
    for (size_t i = 0; s == DT_OK && i < b.size(); i++)
      if (hipMemcpyAsync(pts.as<double>() + off[i] * D, b[i]->dev.p, (size_t)b[i]->n * D * 8,
                         hipMemcpyDeviceToDevice, st) != hipSuccess)
        s = DT_E_DEVICE;
    dt_result all;
    all.D = D;
    if (s == DT_OK)
      s = run_batch(pts.as<double>(), nullptr, off.data(), (int64_t)b.size(), D, opt, true, st,
                    &all, true);
    for (size_t i = 0; i < b.size(); i++) {
      if (s == DT_OK) split_out(b[i], all, all.set_offsets[i], all.set_offsets[i + 1], st);
      else run_alone(b[i], st);
    }
  }

  void worker() {
    hipStream_t st = nullptr;
    if (hipSetDevice(device) != hipSuccess ||
        hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess)
      st = nullptr;
    // scratch of the runs comes from the stream-ordered pool on this stream,
    // and blocks of the block cache released here are marked with events on it
    AllocStreamScope scope(st);
    UseStreamScope use(st);
    for (;;) {
      std::vector<Job*> b;
      {
        std::unique_lock<std::mutex> lk(mu);
        cv_work.wait(lk, [&] { return !ready.empty() || (stop && waiting.empty()); });
        if (ready.empty()) break;
        int64_t pts = 0;
        while (!ready.empty()) {
          Job* j = ready.front();
          if (!b.empty() && (j->n > DIRECT_MAX || b[0]->n > DIRECT_MAX || j->D != b[0]->D ||
                             pts + j->n > MAX_BATCH_POINTS))
            break;
          ready.pop_front();
          j->started = true;
          pts += j->n;
          b.push_back(j);
        }
      }
      const double tb0 = mono_s();
      if (!b.empty()) {
        try {
          run_batch_of(b, st);
        } catch (const std::bad_alloc&) {   // host memory of the batch's bookkeeping
          for (Job* j : b)
            if (!j->res && j->status == DT_OK) j->status = DT_E_NOMEM;
        }
      }
      if (trace && !b.empty()) {
        int64_t pts = 0, mx = 0;
        for (Job* j : b) {
          pts += j->n;
          mx = j->n > mx ? j->n : mx;
        }
        fprintf(stderr, "[srv] t %.3f batch %zu jobs %lld points (largest %lld) %.1f ms\n",
                mono_s() - t0, b.size(), (long long)pts, (long long)mx, (mono_s() - tb0) * 1e3);
      }
      {
        std::lock_guard<std::mutex> lk(mu);
        double now = mono_s() - t0;
        for (Job* j : b) {
          j->done = true;
          j->t[2] = now;
          used -= j->footprint;
          j->dev.release();   // its last uses were on this worker's stream
        }
        admit();
      }
      cv_done.notify_all();
      cv_work.notify_all();
    }
    if (st) (void)hipStreamDestroy(st);
  }
};

extern "C" int dt_server_create(size_t hbm_budget_bytes, const dt_options* opt, dt_server** srv) {
  if (!srv || hbm_budget_bytes == 0) return DT_E_INVALID_ARG;
  *srv = nullptr;
  dt_options o;
  DT_TRY(check_options(opt, o));
  dt_server* s = new dt_server();
  s->opt = o;
  s->opt.profile = 0;
  s->opt.keep_stages = 0;
  s->budget = hbm_budget_bytes;
  s->t0 = mono_s();
  s->trace = getenv("DT_DEBUG") != nullptr;
  DT_HIP_DEL(hipGetDevice(&s->device), s);
  // keep memory freed by the workers in the device's stream-ordered pool
  hipMemPool_t pool;
  if (hipDeviceGetDefaultMemPool(&pool, s->device) == hipSuccess) {
    uint64_t keep = UINT64_MAX;
    (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
  }
  for (int i = 0; i < NUM_WORKERS; i++) s->workers.emplace_back([s] { s->worker(); });
  *srv = s;
  return DT_OK;
}

extern "C" int dt_server_submit(dt_server* s, const double* points, int64_t n, int D, int k,
                                double sample_rate, int points_on_device, uint64_t* ticket) {
  if (!s || !ticket || !points || (D != 2 && D != 3) || n < 0 || n > 0x7FFFFFF0ll || k < 1)
    return DT_E_INVALID_ARG;
  if (!(sample_rate >= 0.0 && sample_rate <= 1.0)) return DT_E_INVALID_ARG;
  if (n < D + 1) return DT_E_DEGENERATE;
  Job* j = new Job();
  j->n = n;
  j->D = D;
  j->k = k;
  j->rate = sample_rate;
  j->footprint = footprint_of(n, D, n <= DIRECT_MAX ? 1 : k);
  if (j->footprint > s->budget) {
    delete j;
    return DT_E_NOMEM;
  }
  // the job's points live on the device from now until the job is done
  int as = j->dev.alloc_plain((size_t)n * D * 8);
  if (as != DT_OK) {
    delete j;
    return as;
  }
  if (hipMemcpy(j->dev.p, points, (size_t)n * D * 8,
                points_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice) !=
      hipSuccess) {
    delete j;
    return DT_E_DEVICE;
  }
  {
    std::lock_guard<std::mutex> lk(s->mu);
    j->ticket = s->next++;
    j->t[0] = mono_s() - s->t0;
    s->jobs[j->ticket] = j;
    s->waiting.push_back(j);
    s->admit();
    *ticket = j->ticket;
  }
  s->cv_work.notify_all();
  return DT_OK;
}

static int take_result(dt_server* s, Job* j, dt_result** out) {
  int st = j->status;
  *out = st == DT_OK ? j->res : nullptr;
  if (st != DT_OK) delete j->res;
  j->res = nullptr;
  return st;
}

extern "C" int dt_server_poll(dt_server* s, uint64_t ticket, dt_result** out) {
  if (!s || !out) return DT_E_INVALID_ARG;
  *out = nullptr;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->jobs.find(ticket);
  if (it == s->jobs.end()) return DT_E_INVALID_ARG;
  if (!it->second->done) return DT_E_NOT_READY;
  return take_result(s, it->second, out);
}

extern "C" int dt_server_wait(dt_server* s, uint64_t ticket, dt_result** out) {
  if (!s || !out) return DT_E_INVALID_ARG;
  *out = nullptr;
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->jobs.find(ticket);
  if (it == s->jobs.end()) return DT_E_INVALID_ARG;
  Job* j = it->second;
  s->cv_done.wait(lk, [&] { return j->done; });
  return take_result(s, j, out);
}

extern "C" int dt_server_times(dt_server* s, uint64_t ticket, double t[3]) {
  if (!s || !t) return DT_E_INVALID_ARG;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->jobs.find(ticket);
  if (it == s->jobs.end()) return DT_E_INVALID_ARG;
  if (!it->second->done) return DT_E_NOT_READY;
  for (int i = 0; i < 3; i++) t[i] = it->second->t[i];
  return DT_OK;
}

extern "C" void dt_server_destroy(dt_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  for (auto& w : s->workers) w.join();
  for (auto& kv : s->jobs) {
    delete kv.second->res;
    delete kv.second;
  }
  // hand the workers' cached scratch memory back to the device
  hipMemPool_t pool;
  if (hipDeviceGetDefaultMemPool(&pool, s->device) == hipSuccess) (void)hipMemPoolTrimTo(pool, 0);
  delete s;
}
