// The divide-and-conquer pipeline (host orchestration over device stages).
#pragma once
#include <vector>

#include "dt_internal.hpp"

struct dt_result {
  int D = 3;
  int64_t m = 0;                      // simplices
  dtk::DevBuf rows;                   // m x (D+1) int32, device
  std::vector<int64_t> set_offsets;   // batch results: row offsets per set
  dt_stats stats{};
  std::vector<char> stage[DT_NUM_ARR];
  // neighbours of every row, computed on the first request
  mutable dtk::DevBuf nbr;
  mutable bool nbr_ready = false;
};

namespace dtk {

// Per-call context: counters and flags in device and pinned host memory.
struct Ctx {
  DevBuf dctr, dflag;
  Counters* hctr = nullptr;
  uint32_t* hflag = nullptr;
  bool pinned = true;   // hctr is a pinned block of the per-thread cache
  ~Ctx();
  int init();
  Counters* dc() const { return dctr.as<Counters>(); }
};

double now_ms();
// Validate options (NULL = defaults) into o.
int check_options(const dt_options* in, dt_options& o);
// Sort the rows of r lexicographically (host round trip).
int sort_rows_inplace(dt_result* r, hipStream_t st);

int run_triangulate(const double* points, int64_t n, int D, int k, double sample_rate,
                    const dt_options& o, bool on_device, hipStream_t st, dt_result* r);
int run_dc(const double* points, int64_t n, int D, int k, double sample_rate,
           const dt_options& o, bool on_device, hipStream_t st, dt_result* r);
// local_ids: label every point by its index inside its set (ids unused).
int run_batch(const double* points, const int64_t* ids, const int64_t* offsets, int64_t num_sets,
              int D, const dt_options& o, bool on_device, hipStream_t st, dt_result* r,
              bool local_ids = false);
// Recursive bisection: log2 k levels of 2-way division, k-1 merges.
int run_recursive(const double* points, int64_t n, int D, int k, double sample_rate,
                  const dt_options& o, bool on_device, hipStream_t st, dt_result* r);
// Rows of the live finite cells of a batched job, grouped by set at the
// given row offsets (order inside a set unspecified).
int extract_grouped(const LocalJob& job, const CellPool& pool,
                    const std::vector<int64_t>& set_offsets, int32_t* rows, hipStream_t st);
// Neighbours of every row of r (m x (D+1) int32: row sharing the facet
// opposite each vertex, -1 on the hull), within each set.
int compute_neighbors(const dt_result& r, DevBuf& nbr, hipStream_t st);

}  // namespace dtk
