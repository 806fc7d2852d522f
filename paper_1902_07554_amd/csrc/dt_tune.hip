// Autotuner of the batched local triangulation's launch parameters.
//
// The tunables (first-level activation per set, level growth rule and
// step, cap on the cavity/insert wavefronts) change only how the rounds of the parallel
// insertion are scheduled, never the triangulation.  The tuner times
// batched runs on a sample of the batch's sets that keeps its size mix
// (every s-th set), one tunable at a time (coordinate descent from the
// defaults); a choice other than the defaults is kept only if it also wins
// on the whole batch.  The winner is remembered per (dimension, precision,
// size class) for the life of the process.
#include <string.h>

#include <algorithm>
#include <chrono>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "dt_common.hpp"
#include "dt_internal.hpp"
#include "dt_pipeline.hpp"

using namespace dtk;

namespace {

// size class: dimension, precision, log2 of the mean set size, log2 of the
// number of sets
using TuneKey = std::tuple<int, int, int, int>;
std::mutex g_tune_mu;
std::map<TuneKey, dt_options> g_tune_cache;

int ilog2(uint64_t v) {
  int r = 0;
  while (v > 1) {
    v >>= 1;
    r++;
  }
  return r;
}

double wall_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

}  // namespace

extern "C" int dt_batch_autotune(const double* points, const int64_t* offsets, int64_t num_sets,
                                 int D, const dt_options* opt, int points_on_device, void* stream,
                                 int64_t sample_points, dt_options* tuned) {
  if (!points || !offsets || !tuned || num_sets < 1 || (D != 2 && D != 3)) return DT_E_INVALID_ARG;
  if (offsets[0] != 0) return DT_E_INVALID_ARG;
  for (int64_t s = 0; s < num_sets; s++)
    if (offsets[s + 1] < offsets[s]) return DT_E_INVALID_ARG;
  int64_t total = offsets[num_sets];
  if (total > 0x7FFFFFF0ll) return DT_E_INVALID_ARG;
  dt_options o;
  DT_TRY(check_options(opt, o));
  o.profile = 0;
  o.keep_stages = 0;
  o.sort_output = 0;
  hipStream_t st = (hipStream_t)stream;
  UseStreamScope use(st);
  if (total == 0) {
    *tuned = o;
    return DT_OK;
  }
  TuneKey key{D, o.precision, ilog2((uint64_t)(total / num_sets) + 1), ilog2((uint64_t)num_sets)};
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune_cache.find(key);
    if (it != g_tune_cache.end()) {
      dt_options r = o;
      r.start_active = it->second.start_active;
      r.grow_div = it->second.grow_div;
      r.cand_blocks = it->second.cand_blocks;
      r.grow_num = it->second.grow_num;
      *tuned = r;
      return DT_OK;
    }
  }
  // every s-th set, about sample_points points in all
  if (sample_points <= 0) sample_points = 4 << 20;
  int64_t stride = total > sample_points ? (total + sample_points - 1) / sample_points : 1;
  std::vector<int64_t> pick;
  for (int64_t s = 0; s < num_sets; s += stride) pick.push_back(s);
  std::vector<int64_t> soff(pick.size() + 1, 0);
  for (size_t i = 0; i < pick.size(); i++)
    soff[i + 1] = soff[i] + (offsets[pick[i] + 1] - offsets[pick[i]]);
  int64_t sn = soff.back();
  DevBuf dpts;
  DT_TRY(dpts.alloc((size_t)(sn ? sn : 1) * D * 8));
  for (size_t i = 0; i < pick.size(); i++) {
    size_t bytes = (size_t)(soff[i + 1] - soff[i]) * D * 8;
    if (!bytes) continue;
    DT_HIP(hipMemcpyAsync(dpts.as<double>() + soff[i] * D, points + offsets[pick[i]] * D, bytes,
                          points_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, st));
  }
  DT_HIP(hipStreamSynchronize(st));

  // a trial is the faster of two runs; a change must gain 3 % to be taken
  auto trial = [&](const dt_options& t, double* ms) -> int {
    *ms = 1e300;
    for (int rep = 0; rep < 2; rep++) {
      dt_result r;
      r.D = D;
      double a = wall_ms();
      int s = run_batch(dpts.as<double>(), nullptr, soff.data(), (int64_t)pick.size(), D, t, true,
                        st, &r);
      if (s != DT_OK) return s;
      *ms = std::min(*ms, wall_ms() - a);
    }
    return DT_OK;
  };
  const double GAIN = 0.97;
  dt_options best = o;
  best.start_active = 256;
  best.grow_div = 64;
  best.cand_blocks = 32768;
  best.grow_num = num_sets > 1 ? 10 : 12;
  double best_ms = 0;
  DT_TRY(trial(best, &best_ms));
  const int starts[] = {64, 1024};
  const int grows[] = {8, 1024};
  const int blocks[] = {16384, 65536};
  for (int v : starts) {
    dt_options t = best;
    t.start_active = v;
    double ms;
    DT_TRY(trial(t, &ms));
    if (ms < GAIN * best_ms) { best_ms = ms; best = t; }
  }
  for (int v : grows) {
    dt_options t = best;
    t.grow_div = v;
    double ms;
    DT_TRY(trial(t, &ms));
    if (ms < GAIN * best_ms) { best_ms = ms; best = t; }
  }
  for (int v : blocks) {
    dt_options t = best;
    t.cand_blocks = v;
    double ms;
    DT_TRY(trial(t, &ms));
    if (ms < GAIN * best_ms) { best_ms = ms; best = t; }
  }
  const int steps[] = {9, 12, 16};
  for (int v : steps) {
    if (v == best.grow_num) continue;
    dt_options t = best;
    t.grow_num = v;
    double ms;
    DT_TRY(trial(t, &ms));
    if (ms < GAIN * best_ms) { best_ms = ms; best = t; }
  }
  // the sample may mislead: a choice other than the defaults must also
  // win on the whole batch (the faster of two runs each, by 2 %)
  if (best.start_active != 256 || best.grow_div != 64 || best.cand_blocks != 32768 ||
      best.grow_num != (num_sets > 1 ? 10 : 12)) {
    auto full = [&](const dt_options& t, double* ms) -> int {
      *ms = 1e300;
      for (int rep = 0; rep < 2; rep++) {
        dt_result r;
        r.D = D;
        double a = wall_ms();
        int s = run_batch(points, nullptr, offsets, num_sets, D, t, points_on_device != 0, st, &r);
        if (s != DT_OK) return s;
        *ms = std::min(*ms, wall_ms() - a);
      }
      return DT_OK;
    };
    dt_options def = best;
    def.start_active = 256;
    def.grow_div = 64;
    def.cand_blocks = 32768;
    def.grow_num = num_sets > 1 ? 10 : 12;
    double ms_best = 0, ms_def = 0;
    DT_TRY(full(best, &ms_best));
    DT_TRY(full(def, &ms_def));
    if (!(ms_best < 0.98 * ms_def)) best = def;
  }
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[key] = best;
  }
  dt_options r = o;
  r.start_active = best.start_active;
  r.grow_div = best.grow_div;
  r.cand_blocks = best.cand_blocks;
  r.grow_num = best.grow_num;
  *tuned = r;
  return DT_OK;
}
