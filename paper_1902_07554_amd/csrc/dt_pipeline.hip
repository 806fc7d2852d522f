// Host orchestration of the divide-and-conquer triangulation (Algorithm 1)
// and of batched independent triangulations.
#include <math.h>
#include <string.h>

#include <vector>

#include "dt_common.hpp"
#include "dt_internal.hpp"
#include "dt_pipeline.hpp"
#include "dt_prims.hpp"
#include "dt_prep.hpp"
#include "dt_stages.hpp"

namespace dtk {

constexpr int TB = 256;
static inline uint32_t blocks(uint64_t n) { return (uint32_t)((n + TB - 1) / TB); }

// pset[p] = set of point p, by binary search in the set offsets.
__global__ void k_set_of_point(const uint32_t* off, uint32_t nsets, uint32_t n, uint32_t* pset) {
  uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  uint32_t lo = 0, hi = nsets;   // find s with off[s] <= p < off[s+1]
  while (hi - lo > 1) {
    uint32_t mid = (lo + hi) >> 1;
    if (off[mid] <= p) lo = mid;
    else hi = mid;
  }
  pset[p] = lo;
}

// Write the live finite cells grouped by set: row slot = set_base[s] +
// cursor[s]++ (order inside a set is unspecified).  The cells of one star
// are allocated together, so neighbouring lanes mostly hold cells of one
// set: the lanes of each set in a wavefront share one cursor atomic.
template <int D>
__global__ void k_extract_grouped(const double4* pts, const uint32_t* pset, const Cell* cells, uint32_t ncells, const uint32_t* set_base,
                                  uint32_t* cursor, int32_t* rows) {
  uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  bool live = c < ncells && cells[c].fwd == ALIVE;
  uint4 v = make_uint4(0, 0, 0, 0);
  if (live) v = cells[c].v;
  uint32_t vv[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
  for (int i = 0; i <= D; i++)
    if (vv[i] == INF_V) live = false;
  const uint32_t s = live ? pset[v.x] : 0xFFFFFFFFu;
  const uint32_t lane = __lane_id();
  uint32_t slot = 0;
  unsigned long long todo = __ballot(live);
  while (todo) {
    const int lead = __ffsll(todo) - 1;
    const uint32_t ls = __shfl(s, lead, 64);
    const unsigned long long same = __ballot(live && s == ls);
    uint32_t base = 0;
    if ((int)lane == lead) base = atomicAdd(&cursor[ls], (uint32_t)__popcll(same));
    base = __shfl(base, lead, 64);
    if (live && s == ls)
      slot = set_base[ls] + base + (uint32_t)__popcll(same & ((1ull << lane) - 1ull));
    todo &= ~same;
  }
  if (!live) return;
  int32_t k[4];
#pragma unroll
  for (int i = 0; i <= D; i++) k[i] = (int32_t)__double_as_longlong(pts[vv[i]].w);
#pragma unroll
  for (int i = 1; i <= D; i++)
#pragma unroll
    for (int j = i; j > 0; j--)
      if (k[j] < k[j - 1]) { int32_t t = k[j]; k[j] = k[j - 1]; k[j - 1] = t; }
#pragma unroll
  for (int i = 0; i <= D; i++) rows[(size_t)slot * (D + 1) + i] = k[i];
}

// Label of every point: its index inside its set.
__global__ void k_local_labels(const uint32_t* off, const uint32_t* pset, uint32_t n,
                               long long* keys) {
  uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  keys[p] = (long long)(p - off[pset[p]]);
}

int extract_grouped(const LocalJob& job, const CellPool& pool,
                    const std::vector<int64_t>& set_offsets, int32_t* rows, hipStream_t st) {
  const uint32_t ns = job.nsets;
  if (pool.ncells == 0 || ns == 0) return DT_OK;
  DevBuf base, cursor;
  DT_TRY(base.alloc((size_t)ns * 4));
  DT_TRY(cursor.alloc((size_t)ns * 4));
  std::vector<uint32_t> hb(ns);
  for (uint32_t i = 0; i < ns; i++) hb[i] = (uint32_t)set_offsets[i];
  DT_HIP(hipMemcpyAsync(base.p, hb.data(), (size_t)ns * 4, hipMemcpyHostToDevice, st));
  DT_HIP(hipMemsetAsync(cursor.p, 0, (size_t)ns * 4, st));
  if (job.D == 2)
    hipLaunchKernelGGL(k_extract_grouped<2>, dim3(blocks(pool.ncells)), dim3(TB), 0, st, job.pts,
                       job.pset, pool.cells.as<Cell>(), pool.ncells, base.as<uint32_t>(),
                       cursor.as<uint32_t>(), rows);
  else
    hipLaunchKernelGGL(k_extract_grouped<3>, dim3(blocks(pool.ncells)), dim3(TB), 0, st, job.pts,
                       job.pset, pool.cells.as<Cell>(), pool.ncells, base.as<uint32_t>(),
                       cursor.as<uint32_t>(), rows);
  DT_HIP(hipGetLastError());
  DT_HIP(hipStreamSynchronize(st));
  return DT_OK;
}

static void fill_pred_stats(dt_stats& s, const K4Stats& ks) {
  for (int i = 0; i < 4; i++)
    for (int j = 0; j < 4; j++) s.pred[i][j] += (int64_t)ks.pred[i][j];
}

// Bring row-major points to the device (copy if host memory).
static int stage_input(const double* points, uint64_t n, int D, bool on_device, DevBuf& holder,
                       const double** dptr, hipStream_t st) {
  if (on_device) {
    *dptr = points;
    return DT_OK;
  }
  DT_TRY(holder.alloc(n * D * sizeof(double)));
  DT_HIP(hipMemcpyAsync(holder.p, points, n * D * sizeof(double), hipMemcpyHostToDevice, st));
  *dptr = holder.as<double>();
  return DT_OK;
}

int run_batch(const double* points, const int64_t* ids, const int64_t* offsets, int64_t num_sets,
              int D, const dt_options& o, bool on_device, hipStream_t st, dt_result* r,
              bool local_ids) {
  double t0 = now_ms();
  Ctx cx;
  DT_TRY(cx.init());
  uint32_t n = (uint32_t)offsets[num_sets];
  uint32_t ns = (uint32_t)num_sets;
  r->set_offsets.assign(num_sets + 1, 0);
  r->stats.n = n;
  r->stats.D = D;
  r->stats.k = (int32_t)ns;
  if (n == 0) return DT_OK;
  DevBuf din, dkeys, pts, scratch, pset, setoff;
  const double* dp = nullptr;
  DT_TRY(stage_input(points, n, D, on_device, din, &dp, st));
  if (ids && !local_ids) {
    DT_TRY(dkeys.alloc((size_t)n * 8));
    DT_HIP(hipMemcpyAsync(dkeys.p, ids, (size_t)n * 8, hipMemcpyHostToDevice, st));
  }
  std::vector<uint32_t> off32(num_sets + 1);
  for (int64_t s = 0; s <= num_sets; s++) off32[s] = (uint32_t)offsets[s];
  DT_TRY(setoff.alloc((size_t)(ns + 1) * 4));
  DT_HIP(hipMemcpyAsync(setoff.p, off32.data(), (size_t)(ns + 1) * 4, hipMemcpyHostToDevice, st));
  DT_TRY(pset.alloc((size_t)n * 4));
  hipLaunchKernelGGL(k_set_of_point, dim3(blocks(n)), dim3(TB), 0, st, setoff.as<uint32_t>(), ns,
                     n, pset.as<uint32_t>());
  if (local_ids) {
    DT_TRY(dkeys.alloc((size_t)n * 8));
    hipLaunchKernelGGL(k_local_labels, dim3(blocks(n)), dim3(TB), 0, st, setoff.as<uint32_t>(),
                       pset.as<uint32_t>(), n, dkeys.as<long long>());
    DT_HIP(hipGetLastError());
  }
  DT_TRY(pts.alloc((size_t)n * sizeof(double4)));
  DT_TRY(prep_points(dp, (ids || local_ids) ? dkeys.as<long long>() : nullptr,
                     ns > 1 ? pset.as<uint32_t>() : nullptr,
                     n, D, pts.as<double4>(), scratch, cx.dflag.as<uint32_t>(), cx.hflag, st));
  {
    // order every set along a space-filling curve (the set is the major
    // key, so sets keep their ranges); labels travel with the points, so no
    // triangulation changes, but neighbouring points share cache lines
    double lo[3], hi[3];
    DT_TRY(bbox(pts.as<double4>(), n, lo, hi, st));
    int sbits = 0;
    while ((1u << sbits) < ns) sbits++;
    DT_TRY(spatial_sort(pts, n, D, lo, hi, ns > 1 ? pset.as<uint32_t>() : nullptr, sbits, st));
  }
  double t1 = now_ms();
  LocalJob job;
  job.D = D;
  job.npts = n;
  job.nsets = ns;
  job.pts = pts.as<double4>();
  job.pset = pset.as<uint32_t>();
  job.set_off = setoff.as<uint32_t>();
  job.fp32 = o.precision == DT_PREC_FP32;
  job.tune(o);
  CellPool pool;
  K4Stats ks;
  int s = k4_run(job, pool, cx.dc(), cx.hctr, st, ks);
  if (s != DT_OK) {
    r->stats.fail = cx.hctr->flags;
    return s;
  }
  double t2 = now_ms();
  if (ns == 1) {
    // single set: count the rows per block, scan, write them in cell order
    DT_TRY(k4_extract(job, pool, nullptr, cx.dflag.as<uint32_t>(), nullptr, st));
    uint32_t hcount = 0;
    DT_HIP(hipMemcpyAsync(cx.hflag, cx.dflag.p, 4, hipMemcpyDeviceToHost, st));
    DT_HIP(hipStreamSynchronize(st));
    hcount = *cx.hflag;
    r->m = hcount;
    r->set_offsets[1] = hcount;
    DT_TRY(r->rows.alloc_plain((size_t)hcount * (D + 1) * 4));
    DT_TRY(k4_extract(job, pool, r->rows.as<int32_t>(), cx.dflag.as<uint32_t>(), nullptr, st));
  } else {
    // per-set counts, then rows grouped by set
    DevBuf cnt;
    DT_TRY(cnt.alloc((size_t)ns * 4));
    DT_HIP(hipMemsetAsync(cnt.p, 0, (size_t)ns * 4, st));
    DT_TRY(k4_extract(job, pool, nullptr, cx.dflag.as<uint32_t>(), cnt.as<uint32_t>(), st));
    std::vector<uint32_t> hc(ns);
    DT_HIP(hipMemcpyAsync(hc.data(), cnt.p, (size_t)ns * 4, hipMemcpyDeviceToHost, st));
    DT_HIP(hipStreamSynchronize(st));
    for (uint32_t i = 0; i < ns; i++) r->set_offsets[i + 1] = r->set_offsets[i] + hc[i];
    r->m = r->set_offsets[ns];
    DT_TRY(r->rows.alloc_plain((size_t)r->m * (D + 1) * 4));
    DT_TRY(extract_grouped(job, pool, r->set_offsets, r->rows.as<int32_t>(), st));
  }  DT_HIP(hipStreamSynchronize(st));
  double t3 = now_ms();
  r->stats.num_simplices = r->m;
  r->stats.rounds = ks.rounds;
  r->stats.large_cavities = ks.giant_rounds;
  r->stats.seeded_sets = ks.seeded;
  r->stats.cavity_cells = (int64_t)ks.cavity_cells;
  r->stats.candidates = (int64_t)ks.candidates;
  fill_pred_stats(r->stats, ks);
  r->stats.stage_ms[DT_STAGE_VALIDATE] = t1 - t0;
  r->stats.stage_ms[DT_STAGE_LOCAL_DT] = t2 - t1;
  r->stats.stage_ms[DT_STAGE_OUTPUT] = t3 - t2;
  r->stats.stage_ms[DT_STAGE_TOTAL] = t3 - t0;
  int64_t mn = -1, mx = 0;
  for (uint32_t i = 0; i < ns; i++) {
    int64_t sz = offsets[i + 1] - offsets[i];
    if (mn < 0 || sz < mn) mn = sz;
    if (sz > mx) mx = sz;
  }
  r->stats.max_part = mx;
  r->stats.min_part = mn;
  r->stats.local_simplices = r->m;
  return DT_OK;
}

int run_triangulate(const double* points, int64_t n, int D, int k, double sample_rate,
                    const dt_options& o, bool on_device, hipStream_t st, dt_result* r) {
  if (k > 1 && o.recursive) return run_recursive(points, n, D, k, sample_rate, o, on_device, st, r);
  if (k == 1) {
    int64_t off[2] = {0, n};
    int s = run_batch(points, nullptr, off, 1, D, o, on_device, st, r);
    if (s == DT_OK && r->m == 0) return DT_E_DEGENERATE;
    r->stats.k = 1;
    return s;
  }
  return run_dc(points, n, D, k, sample_rate, o, on_device, st, r);
}

}  // namespace dtk
