// Divide-and-conquer pipeline: Algorithm 1 of the paper with the
// sample-based divide of Algorithm 2 (or the cyclic kd median split).
//   divide       -> pid of every point (dt_divide.hip)
//   buckets      -> points grouped by partition, stable (radix pass on pid)
//   local DTs    -> all T_i in one batched run (dt_k4.hip)
//   border       -> flagged simplices B and their vertices V_B (dt_merge.hip)
//   border DT    -> T_B = DT(V_B) (dt_k4.hip)
//   merge        -> (union T_i minus B) + spanning or matching T_B simplices
#include <math.h>
#include <string.h>

#include <vector>

#include "dt_common.hpp"
#include "dt_internal.hpp"
#include "dt_gwrap.hpp"
#include "dt_pipeline.hpp"
#include "dt_prep.hpp"
#include "dt_prims.hpp"
#include "dt_stages.hpp"

namespace dtk {

constexpr int CB = 256;
static inline uint32_t cblocks(uint64_t n) { return (uint32_t)((n + CB - 1) / CB); }

// eta = round-half-up(rate * n), at least D+2, at most n; rate 0 = sqrt(n).
static uint32_t sample_size(uint32_t n, double rate, int D) {
  double e = (rate == 0.0) ? floor(sqrt((double)n) + 0.5) : floor(rate * (double)n + 0.5);
  if (e < D + 2) e = D + 2;
  if (e > n) e = n;
  return (uint32_t)e;
}

__global__ void k_set_of_point2(const uint32_t* off, uint32_t nsets, uint32_t n, uint32_t* pset) {
  uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  uint32_t lo = 0, hi = nsets;
  while (hi - lo > 1) {
    uint32_t mid = (lo + hi) >> 1;
    if (off[mid] <= p) lo = mid;
    else hi = mid;
  }
  pset[p] = lo;
}

// Finite live cells of a pool with their border flag (stage output).
template <int D>
__global__ void k_rows_with_flag(const double4* P, const Cell* cells,
                                 uint32_t ncells, const unsigned long long* hashm, int32_t* rows,
                                 uint32_t* count) {
  uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncells || cells[c].fwd != ALIVE) return;
  uint4 v = cells[c].v;
  uint32_t vv[4] = {v.x, v.y, v.z, v.w};
  int32_t k[4];
  for (int i = 0; i <= D; i++) {
    if (vv[i] == INF_V) return;
    k[i] = (int32_t)__double_as_longlong(P[vv[i]].w);
  }
  for (int i = 1; i <= D; i++)
    for (int j = i; j > 0 && k[j] < k[j - 1]; j--) {
      int32_t t = k[j]; k[j] = k[j - 1]; k[j - 1] = t;
    }
  uint32_t s = atomicAdd(count, 1u);
  for (int i = 0; i <= D; i++) rows[(size_t)s * (D + 2) + i] = k[i];
  rows[(size_t)s * (D + 2) + D + 1] = (int32_t)((hashm[c >> 6] >> (c & 63u)) & 1ull);
}

template <class T>
static int to_host(std::vector<char>& dst, const void* src, size_t count, hipStream_t st) {
  dst.resize(count * sizeof(T));
  if (count) DT_HIP(hipMemcpyAsync(dst.data(), src, count * sizeof(T), hipMemcpyDeviceToHost, st));
  DT_HIP(hipStreamSynchronize(st));
  return DT_OK;
}

static int pool_rows_host(const LocalJob& job, const CellPool& pool, int D, std::vector<char>& dst,
                          hipStream_t st) {
  DevBuf cnt, rows;
  DT_TRY(cnt.alloc(16));
  uint32_t m = 0;
  DT_TRY(k4_extract(job, pool, nullptr, cnt.as<uint32_t>(), nullptr, st));
  DT_HIP(hipMemcpyAsync(&m, cnt.p, 4, hipMemcpyDeviceToHost, st));
  DT_HIP(hipStreamSynchronize(st));
  DT_TRY(rows.alloc((size_t)(m ? m : 1) * (D + 1) * 4));
  DT_TRY(k4_extract(job, pool, rows.as<int32_t>(), cnt.as<uint32_t>(), nullptr, st));
  return to_host<int32_t>(dst, rows.p, (size_t)m * (D + 1), st);
}

static void add_pred(dt_stats& s, const K4Stats& ks) {
  for (int i = 0; i < 4; i++)
    for (int j = 0; j < 4; j++) s.pred[i][j] += (int64_t)ks.pred[i][j];
  s.rounds += ks.rounds;
  s.large_cavities += ks.giant_rounds;
  s.seeded_sets += ks.seeded;
  s.cavity_cells += (int64_t)ks.cavity_cells;
  s.candidates += (int64_t)ks.candidates;
}

// Coefficient of variation of the sample's counts over a uniform grid of
// about eta/4 cells spanning the input's box (empty cells included): near
// 1/2 for an evenly spread sample, far above 1 for a clustered one.
static double sample_spread(const std::vector<double4>& s, int D, const double lo[3],
                            const double hi[3]) {
  const size_t m = s.size();
  const double target = m / 4.0 > 1.0 ? m / 4.0 : 1.0;
  int g = (int)floor(pow(target, 1.0 / D));
  if (g < 1) g = 1;
  std::vector<uint32_t> cnt((size_t)(D == 3 ? g * g * g : g * g), 0);
  auto cell = [&](double x, int a) {
    const double w = hi[a] - lo[a];
    int c = w > 0 ? (int)((x - lo[a]) / w * g) : 0;
    return c < 0 ? 0 : (c >= g ? g - 1 : c);
  };
  for (const double4& p : s) {
    size_t c = (size_t)cell(p.x, 0) + (size_t)g * cell(p.y, 1);
    if (D == 3) c += (size_t)g * g * cell(p.z, 2);
    cnt[c]++;
  }
  const double mean = (double)m / cnt.size();
  double ss = 0.0;
  for (uint32_t c : cnt) ss += (c - mean) * (c - mean);
  return mean > 0 ? sqrt(ss / cnt.size()) / mean : 0.0;
}

int run_dc(const double* points, int64_t n64, int D, int k, double rate, const dt_options& o,
           bool on_device, hipStream_t st, dt_result* r) {
  double t0 = now_ms();
  dt_stats& S = r->stats;
  S.n = n64;
  S.D = D;
  S.k = k;
  uint32_t n = (uint32_t)n64;
  uint32_t eta = sample_size(n, rate, D);
  if (o.divide != DT_DIVIDE_KD && (uint32_t)k > eta) return DT_E_INVALID_ARG;
  if (o.divide == DT_DIVIDE_KD && (k & (k - 1)) != 0) return DT_E_INVALID_ARG;
  if ((uint32_t)k > n) return DT_E_INVALID_ARG;
  Ctx cx;
  DT_TRY(cx.init());
  // ---- input
  DevBuf din, P, scratch;
  const double* dp = points;
  if (!on_device) {
    DT_TRY(din.alloc((size_t)n * D * 8));
    DT_HIP(hipMemcpyAsync(din.p, points, (size_t)n * D * 8, hipMemcpyHostToDevice, st));
    dp = din.as<double>();
  }
  DT_TRY(P.alloc((size_t)n * sizeof(double4)));
  DT_TRY(prep_points(dp, nullptr, nullptr, n, D, P.as<double4>(), scratch, cx.dflag.as<uint32_t>(),
                     cx.hflag, st));
  scratch.release();
  double lo[3], hi[3];
  DT_TRY(bbox(P.as<double4>(), n, lo, hi, st));
  double t1 = now_ms();
  S.stage_ms[DT_STAGE_VALIDATE] = t1 - t0;

  // ---- divide
  DevBuf pid, sid, Sp, part, nearest, boxes, goff, gadj, gw;
  SampleGrid sgrid;
  CellPool spool;
  LocalJob sjob;
  DevBuf sset, soff;
  double cut = 0.0;
  int divide = o.divide;
  if (divide != DT_DIVIDE_KD) {
    DT_TRY(select_sample(n, eta, o.seed, sid, st));
    DT_TRY(Sp.alloc((size_t)eta * sizeof(double4)));
    DT_TRY(gather_points(P.as<double4>(), sid.as<uint32_t>(), eta, Sp.as<double4>(), st));
  }
  if (divide == DT_DIVIDE_AUTO) {
    // how evenly the sample fills its box: counts over a grid of ~eta/4 cells
    std::vector<double4> hs(eta);
    DT_HIP(hipMemcpyAsync(hs.data(), Sp.p, (size_t)eta * sizeof(double4), hipMemcpyDeviceToHost,
                          st));
    DT_HIP(hipStreamSynchronize(st));
    S.divide_stat = sample_spread(hs, D, lo, hi);
    divide = (S.divide_stat <= DT_AUTO_CV && (k & (k - 1)) == 0) ? DT_DIVIDE_KD : DT_DIVIDE_SAMPLE;
  }
  S.divide_used = divide;
  if (divide == DT_DIVIDE_SAMPLE) {
    double ta = now_ms();
    S.stage_ms[DT_STAGE_SAMPLE] = ta - t1;
    DT_TRY(sset.alloc((size_t)eta * 4));
    DT_TRY(soff.alloc(8));
    DT_HIP(hipMemsetAsync(sset.p, 0, (size_t)eta * 4, st));
    uint32_t so[2] = {0, eta};
    DT_HIP(hipMemcpyAsync(soff.p, so, 8, hipMemcpyHostToDevice, st));
    sjob.D = D;
    sjob.npts = eta;
    sjob.nsets = 1;
    sjob.pts = Sp.as<double4>();
    sjob.pset = sset.as<uint32_t>();
    sjob.set_off = soff.as<uint32_t>();
    sjob.fp32 = o.precision == DT_PREC_FP32;
    // a sample of a few thousand points is gift-wrapped; a larger one, or
    // one the wrap declines, is triangulated by parallel insertion
    uint32_t wrap = 0;
    int s = DT_E_NOT_READY;
    if (eta <= GW_MAX_POINTS && o.gift_wrap >= 0)
      s = gift_wrap(Sp.as<double4>(), eta, D, spool, &wrap, st);
    if (s == DT_E_NOT_READY) {
      K4Stats ks;
      wrap = 0;
      s = k4_run(sjob, spool, cx.dc(), cx.hctr, st, ks);
      add_pred(S, ks);
      if (s != DT_OK) { S.fail = cx.hctr->flags; return s; }
    } else if (s != DT_OK) {
      return s;
    }
    S.wrap_levels = wrap;
    if (spool.ncells == 0) return DT_E_DEGENERATE;
    double tb = now_ms();
    S.stage_ms[DT_STAGE_SAMPLE_DT] = tb - ta;
    DT_TRY(partition_sample(Sp.as<double4>(), eta, D, spool, (uint32_t)k, o, lo, hi, part, &cut,
                            goff, gadj, gw, st));
    double tc = now_ms();
    S.stage_ms[DT_STAGE_PARTITION] = tc - tb;
    DT_TRY(assign_points(P.as<double4>(), n, Sp.as<double4>(), eta, D, part.as<uint32_t>(), lo, hi,
                         goff.as<uint32_t>(), gadj.as<uint32_t>(), pid, nearest, sgrid, st));
    S.stage_ms[DT_STAGE_ASSIGN] = now_ms() - tc;
    S.eta = eta;
    S.cut_weight = cut;
  } else {
    DT_TRY(kd_divide(P.as<double4>(), n, D, (uint32_t)k, pid, boxes, st));
    S.stage_ms[DT_STAGE_ASSIGN] = now_ms() - t1;
    S.eta = 0;
  }

  // ---- buckets (stable by partition)
  double td = now_ms();
  DevBuf keys, order, Pp, cnt, off, pset;
  DT_TRY(keys.alloc((size_t)n * 8));
  DT_TRY(order.alloc((size_t)n * 4));
  // key: partition, then position along a space-filling curve (the order
  // inside a bucket does not change any triangulation; a spatial order
  // makes the gathers of neighbouring points and cells share cache lines)
  DT_TRY(spatial_keys(P.as<double4>(), n, D, lo, hi, pid.as<uint32_t>(),
                      keys.as<unsigned long long>(), order.as<uint32_t>(), st));
  int kbits = 1;
  while ((1u << kbits) < (uint32_t)k) kbits++;
  DT_TRY(Pp.alloc((size_t)n * sizeof(double4)));
  DT_PROF_BEGIN(DT_KERN_BUCKET, st);
  DT_TRY(radix_sort_pairs(keys.as<unsigned long long>(), order.as<uint32_t>(), n,
                          kbits + MORTON_BITS, st));
  DT_TRY(gather_points(P.as<double4>(), order.as<uint32_t>(), n, Pp.as<double4>(), st));
  DT_PROF_END(st);
  keys.release();
  DT_TRY(cnt.alloc((size_t)(k + 1) * 4));
  DT_TRY(off.alloc((size_t)(k + 1) * 4));
  DT_TRY(count_by(pid.as<uint32_t>(), n, (uint32_t)k + 1, cnt.as<uint32_t>(), st));
  DT_TRY(exclusive_scan(cnt.as<uint32_t>(), off.as<uint32_t>(), (uint32_t)k + 1, st));
  std::vector<uint32_t> hcnt(k + 1);
  DT_HIP(hipMemcpyAsync(hcnt.data(), cnt.p, (size_t)(k + 1) * 4, hipMemcpyDeviceToHost, st));
  DT_TRY(pset.alloc((size_t)n * 4));
  hipLaunchKernelGGL(k_set_of_point2, dim3(cblocks(n)), dim3(CB), 0, st, off.as<uint32_t>(),
                     (uint32_t)k, n, pset.as<uint32_t>());
  DT_HIP(hipGetLastError());
  DT_HIP(hipStreamSynchronize(st));
  double te = now_ms();
  S.stage_ms[DT_STAGE_SCATTER] = te - td;
  {
    double mu = (double)n / k, ss = 0.0;
    int64_t mx = 0, mn = -1;
    for (int i = 0; i < k; i++) {
      double d = hcnt[i] - mu;
      ss += d * d;
      if ((int64_t)hcnt[i] > mx) mx = hcnt[i];
      if (mn < 0 || (int64_t)hcnt[i] < mn) mn = hcnt[i];
    }
    S.cv = (k > 1) ? sqrt(ss / (k - 1)) / mu : 0.0;
    S.max_dev = mx / mu - 1.0;
    S.max_part = mx;
    S.min_part = mn;
  }

  // ---- local triangulations
  LocalJob job;
  job.D = D;
  job.npts = n;
  job.nsets = (uint32_t)k;
  job.pts = Pp.as<double4>();
  job.pset = pset.as<uint32_t>();
  job.set_off = off.as<uint32_t>();
  job.fp32 = o.precision == DT_PREC_FP32;
  job.tune(o);
  CellPool pool;
  {
    K4Stats ks;
    int s = k4_run(job, pool, cx.dc(), cx.hctr, st, ks);
    add_pred(S, ks);
    if (s != DT_OK) { S.fail = cx.hctr->flags; return s; }
  }
  double tf = now_ms();
  S.stage_ms[DT_STAGE_LOCAL_DT] = tf - te;

  // ---- border
  BorderOut bo;
  // grid of about one input point per cell at c_G = 1
  double cells = (double)n;
  for (int a = 0; a < D; a++) cells /= o.grid_cell;
  Region reg;
  if (o.border == DT_BORDER_REGION || o.border == DT_BORDER_REFINED) {
    reg.refine = o.border == DT_BORDER_REFINED;
    if (divide == DT_DIVIDE_SAMPLE) {
      reg.kind = BORDER_VORONOI;
      reg.S = Sp.as<double4>();
      reg.part = part.as<uint32_t>();
      reg.ns = eta;
      reg.start = sgrid.start.as<uint32_t>();
      reg.items = sgrid.items.as<uint32_t>();
      reg.G = sgrid.G;
      reg.nearest = nearest.as<uint32_t>();
      reg.goff = goff.as<uint32_t>();
      reg.gadj = gadj.as<uint32_t>();
    } else {
      reg.kind = BORDER_BOXES;
      reg.boxes = boxes.as<double>();
    }
  } else if (o.border == DT_BORDER_BBOX) {
    reg.kind = BORDER_BBOX;
  } else if (o.border == DT_BORDER_EXACT) {
    reg.kind = BORDER_EXACT;
  }
  DT_TRY(border_detect(job, pool, reg, n, D, cells, lo, hi, bo, st));
  double tg = now_ms();
  S.stage_ms[DT_STAGE_BORDER] = tg - tf;
  S.border_simplices = (int64_t)bo.nb_finite;
  S.border_vertices = bo.nvb;

  // ---- border triangulation
  DevBuf Pb, bset, boff;
  LocalJob bjob;
  CellPool bpool;
  if (bo.nvb > 0) {
    DT_TRY(Pb.alloc((size_t)bo.nvb * sizeof(double4)));
    DT_TRY(gather_points(P.as<double4>(), bo.vb.as<uint32_t>(), bo.nvb, Pb.as<double4>(), st));
    DT_TRY(spatial_sort(Pb, bo.nvb, D, lo, hi, nullptr, 0, st));
    DT_TRY(bset.alloc((size_t)bo.nvb * 4));
    DT_TRY(boff.alloc(8));
    DT_HIP(hipMemsetAsync(bset.p, 0, (size_t)bo.nvb * 4, st));
    uint32_t bo2[2] = {0, bo.nvb};
    DT_HIP(hipMemcpyAsync(boff.p, bo2, 8, hipMemcpyHostToDevice, st));
    bjob.D = D;
    bjob.npts = bo.nvb;
    bjob.nsets = 1;
    bjob.pts = Pb.as<double4>();
    bjob.pset = bset.as<uint32_t>();
    bjob.set_off = boff.as<uint32_t>();
    bjob.fp32 = o.precision == DT_PREC_FP32;
    bjob.tune(o);
    K4Stats ks;
    int s = k4_run(bjob, bpool, cx.dc(), cx.hctr, st, ks);
    add_pred(S, ks);
    if (s != DT_OK) { S.fail = cx.hctr->flags; return s; }
  }
  double th = now_ms();
  S.stage_ms[DT_STAGE_BORDER_DT] = th - tg;

  // ---- merge
  int64_t local_finite = 0, border_finite = 0;
  DT_TRY(merge_output(job, pool, bo, bjob, bpool, pid.as<uint32_t>(), D, r->rows, &r->m,
                      &local_finite, &border_finite, S.probe_hist, st));
  double ti = now_ms();
  S.stage_ms[DT_STAGE_MERGE] = ti - th;
  S.num_simplices = r->m;
  r->set_offsets = {0, r->m};
  S.o_dt = ((double)n + (divide == DT_DIVIDE_SAMPLE ? eta : 0) + bo.nvb) / (double)n;
  S.local_simplices = local_finite;
  S.tb_simplices = border_finite;

  if (o.keep_stages) {
    if (divide == DT_DIVIDE_SAMPLE) {
      std::vector<uint32_t> h(eta);
      DT_HIP(hipMemcpyAsync(h.data(), sid.p, (size_t)eta * 4, hipMemcpyDeviceToHost, st));
      DT_HIP(hipStreamSynchronize(st));
      r->stage[DT_ARR_SAMPLE].resize((size_t)eta * 8);
      int64_t* d = (int64_t*)r->stage[DT_ARR_SAMPLE].data();
      for (uint32_t i = 0; i < eta; i++) d[i] = h[i];
      DT_TRY(pool_rows_host(sjob, spool, D, r->stage[DT_ARR_SAMPLE_DT], st));
      DT_TRY(to_host<uint32_t>(r->stage[DT_ARR_PART], part.p, eta, st));
      // the sample graph as edges (u < v, input ids) with their weights
      {
        std::vector<uint32_t> ho(eta + 1);
        DT_HIP(hipMemcpyAsync(ho.data(), goff.p, (size_t)(eta + 1) * 4, hipMemcpyDeviceToHost, st));
        DT_HIP(hipStreamSynchronize(st));
        const uint32_t na = ho[eta];
        std::vector<uint32_t> ha(na);
        std::vector<double> hw(na);
        if (na) {
          DT_HIP(hipMemcpyAsync(ha.data(), gadj.p, (size_t)na * 4, hipMemcpyDeviceToHost, st));
          DT_HIP(hipMemcpyAsync(hw.data(), gw.p, (size_t)na * 8, hipMemcpyDeviceToHost, st));
          DT_HIP(hipStreamSynchronize(st));
        }
        // sample-local index v is the v-th smallest sample id, and every
        // adjacency list is sorted, so v's entries above v come out in
        // (u, v) order
        std::vector<int32_t> ed;
        std::vector<double> ew;
        for (uint32_t v = 0; v < eta; v++)
          for (uint32_t i = ho[v]; i < ho[v + 1]; i++)
            if (ha[i] > v) {
              ed.push_back((int32_t)h[v]);
              ed.push_back((int32_t)h[ha[i]]);
              ew.push_back(hw[i]);
            }
        r->stage[DT_ARR_GRAPH].resize(ed.size() * 4);
        if (!ed.empty()) memcpy(r->stage[DT_ARR_GRAPH].data(), ed.data(), ed.size() * 4);
        r->stage[DT_ARR_WEIGHTS].resize(ew.size() * 8);
        if (!ew.empty()) memcpy(r->stage[DT_ARR_WEIGHTS].data(), ew.data(), ew.size() * 8);
      }
      DT_TRY(to_host<uint32_t>(r->stage[DT_ARR_NEAREST], nearest.p, n, st));
    }
    DT_TRY(to_host<uint32_t>(r->stage[DT_ARR_PID], pid.p, n, st));
    DT_TRY(to_host<uint32_t>(r->stage[DT_ARR_ORDER], order.p, n, st));
    DT_TRY(to_host<uint32_t>(r->stage[DT_ARR_BORDER_V], bo.vb.p, bo.nvb, st));
    {
      DevBuf rows, c2;
      DT_TRY(rows.alloc((size_t)(S.local_simplices + 1) * (D + 2) * 4));
      DT_TRY(c2.alloc(16));
      DT_HIP(hipMemsetAsync(c2.p, 0, 4, st));
      if (pool.ncells) {
        if (D == 2)
          hipLaunchKernelGGL(k_rows_with_flag<2>, dim3(cblocks(pool.ncells)), dim3(CB), 0, st,
                             job.pts, pool.cells.as<Cell>(), pool.ncells,
                             bo.hashm.as<unsigned long long>(), rows.as<int32_t>(),
                             c2.as<uint32_t>());
        else
          hipLaunchKernelGGL(k_rows_with_flag<3>, dim3(cblocks(pool.ncells)), dim3(CB), 0, st,
                             job.pts, pool.cells.as<Cell>(), pool.ncells,
                             bo.hashm.as<unsigned long long>(), rows.as<int32_t>(),
                             c2.as<uint32_t>());
        DT_HIP(hipGetLastError());
      }
      DT_TRY(to_host<int32_t>(r->stage[DT_ARR_LOCAL], rows.p, (size_t)S.local_simplices * (D + 2),
                              st));
    }
    if (bpool.ncells) DT_TRY(pool_rows_host(bjob, bpool, D, r->stage[DT_ARR_BORDER_DT], st));
  }
  S.stage_ms[DT_STAGE_TOTAL] = now_ms() - t0;
  return DT_OK;
}

}  // namespace dtk
