// Stage functions of the divide-and-conquer pipeline (device work, host
// orchestration).  All pointers are device pointers.
#pragma once
#include "dt_grid.hpp"
#include "dt_internal.hpp"

namespace dtk {

// Divide (dt_divide.hip)
int select_sample(uint32_t n, uint32_t eta, uint64_t seed, DevBuf& sid, hipStream_t st);
int gather_points(const double4* P, const uint32_t* idx, uint32_t m, double4* out,
                  hipStream_t st);
// Reorder pts[0..n) along a space-filling curve over [lo, hi], grouped by
// prefix (prefix[i] < 2^prefix_bits; null = one group, groups contiguous
// and in order, so each keeps its range).  Labels travel with the points.
int spatial_sort(DevBuf& pts, uint32_t n, int D, const double lo[3], const double hi[3],
                 const uint32_t* prefix, int prefix_bits, hipStream_t st);
// The Delaunay graph of a sample (Algorithm 2) from its triangulation (any
// batch: edges join vertices of one set): CSR offsets goff[eta+1], sorted
// adjacency lists gadj, and the weight of every adjacency entry gw (Table
// "weights", d* the bounding-box diagonal of the input).
int sample_graph(const double4* S, uint32_t eta, int D, const CellPool& pool, int weight,
                 double dstar, DevBuf& goff, DevBuf& gadj, DevBuf& gw, hipStream_t st);
// Label propagation on that graph: part[v] in [0, k); a move never takes a
// block above its bound (lmax_of[b] if given, else lmax); with swaps, pairs
// of vertices may also exchange full blocks.
int refine_partition(uint32_t eta, const uint32_t* goff, const uint32_t* gadj, const double* gw,
                     uint32_t* part, uint32_t k, int lmax, const int* lmax_of, int iters,
                     bool swaps, hipStream_t st);
// goff/gadj receive the sample's Delaunay graph (CSR, sorted lists) and
// gw the weight of every adjacency entry.
int partition_sample(const double4* S, uint32_t eta, int D, const CellPool& pool, uint32_t k,
                     const dt_options& o, const double lo[3], const double hi[3],
                     DevBuf& part, double* cut, DevBuf& goff, DevBuf& gadj, DevBuf& gw,
                     hipStream_t st);
// Samples bucketed by grid cell (cells in start[0..ncell], items).
struct SampleGrid {
  Grid G;
  DevBuf start, items;
};
// goff/gadj: the sample's Delaunay graph (the descent search starts on it;
// the grid is its fallback and the region test's).
int assign_points(const double4* P, uint32_t n, const double4* S, uint32_t eta, int D,
                  const uint32_t* part, const double lo[3], const double hi[3],
                  const uint32_t* goff, const uint32_t* gadj, DevBuf& pid,
                  DevBuf& nearest, SampleGrid& sg, hipStream_t st);
// boxes: k x 6 doubles (lo xyz, hi xyz) of every block's region.
int kd_divide(const double4* P, uint32_t n, int D, uint32_t k, DevBuf& pid, DevBuf& boxes,
              hipStream_t st);
int count_by(const uint32_t* x, uint32_t m, uint32_t k, uint32_t* cnt, hipStream_t st);

// Border and merge (dt_merge.hip)
struct BorderOut {
  // bit masks over the local pool's cells (bit c % 64 of word c / 64):
  // finite live cells to output as they are, and the finite border
  // simplices B; nwords words each (whole blocks of tiles)
  DevBuf emitm, hashm;
  size_t nwords = 0;
  DevBuf vb;            // border vertices (global ids, ascending)
  uint32_t nvb = 0;
  uint64_t nb_finite = 0;   // |B| (finite flagged cells)
};
// How a simplex's circumball is tested against the other partitions:
// the grid of occupied cells (the paper's grid test), or the exact regions
// of the divide (sample Voronoi cells, kd boxes).
enum { BORDER_GRID = 0, BORDER_VORONOI = 1, BORDER_BOXES = 2, BORDER_BBOX = 3, BORDER_EXACT = 4 };
struct Region {
  int kind = BORDER_GRID;
  const double4* S = nullptr;      // samples (Voronoi)
  const uint32_t* part = nullptr;  // block of every sample
  uint32_t ns = 0;                 // number of samples (Voronoi)
  const uint32_t* start = nullptr; // sample grid
  const uint32_t* items = nullptr;
  Grid G{};
  const double* boxes = nullptr;   // k x 6 (boxes)
  const uint32_t* nearest = nullptr;  // nearest sample of every point, by id (Voronoi)
  const double* margin = nullptr;     // filled by border_detect (Voronoi), by job point index
  const uint32_t* near_loc = nullptr; // nearest sample of every job point (Voronoi), by job index
  const uint32_t* goff = nullptr;     // Delaunay graph of the sample (Voronoi)
  const uint32_t* gadj = nullptr;
  // filled by border_detect: bounding boxes of the partitions (bbox), and
  // the points of every grid cell (exact)
  const double* pboxes = nullptr;     // nparts x 6
  uint32_t nparts = 0;
  const uint32_t* cstart = nullptr;   // grid cell c: items[cstart[c] .. cstart[c+1])
  const uint32_t* citems = nullptr;   // point indices of the job
  bool refine = false;                // region test, then the exact test on its hits
};
int border_detect(const LocalJob& job, const CellPool& pool, const Region& reg, uint32_t n,
                  int D, double cells_target, const double lo[3], const double hi[3],
                  BorderOut& out, hipStream_t st);
// rows: the output (cell order: local cells, then border cells); *m their
// number; *local_finite / *border_finite: finite cells of the T_i / T_B.
int merge_output(const LocalJob& job, const CellPool& pool, const BorderOut& b,
                 const LocalJob& bjob, const CellPool& bpool, const uint32_t* pid_by_id, int D,
                 DevBuf& rows, int64_t* m, int64_t* local_finite, int64_t* border_finite,
                 int64_t probe_hist[16], hipStream_t st);

}  // namespace dtk
