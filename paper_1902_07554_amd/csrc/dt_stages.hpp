// Stage functions of the divide-and-conquer pipeline (device work, host
// orchestration).  All pointers are device pointers.
#pragma once
#include "dt_internal.hpp"

namespace dtk {

// Divide (dt_divide.hip)
int select_sample(uint32_t n, uint32_t eta, uint64_t seed, DevBuf& sid, hipStream_t st);
int gather_points(const double4* P, const uint32_t* idx, uint32_t m, double4* out,
                  hipStream_t st);
int partition_sample(const double4* S, uint32_t eta, int D, const CellPool& pool, uint32_t k,
                     const dt_options& o, const double lo[3], const double hi[3],
                     DevBuf& part, double* cut, hipStream_t st);
int assign_points(const double4* P, uint32_t n, const double4* S, uint32_t eta, int D,
                  const uint32_t* part, const double lo[3], const double hi[3], DevBuf& pid,
                  DevBuf& nearest, hipStream_t st);
int kd_divide(const double4* P, uint32_t n, int D, uint32_t k, DevBuf& pid, hipStream_t st);
int count_by(const uint32_t* x, uint32_t m, uint32_t k, uint32_t* cnt, hipStream_t st);

// Border and merge (dt_merge.hip)
struct BorderOut {
  DevBuf cflag;         // [pool.ncells] 1 = border simplex (or hull cell)
  DevBuf vb;            // border vertices (global ids, ascending)
  uint32_t nvb = 0;
  uint64_t nb_finite = 0;   // |B| (finite flagged cells)
};
int border_detect(const LocalJob& job, const CellPool& pool, const uint32_t* pid_by_id,
                  uint32_t n, uint32_t k, int D, double cellsize, const double lo[3],
                  const double hi[3], BorderOut& out, hipStream_t st);
int merge_output(const LocalJob& job, const CellPool& pool, const BorderOut& b,
                 const LocalJob& bjob, const CellPool& bpool, const uint32_t* pid_by_id, int D,
                 DevBuf& rows, int64_t* m, int64_t probe_hist[16], hipStream_t st);

}  // namespace dtk
