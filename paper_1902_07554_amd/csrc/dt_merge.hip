// Border detection and merge (paper, Algorithm 1, "Border triangulation"
// and "Merging"; the grid-based intersection test of Section "Geometric
// Primitives").
//
// Border: a finite simplex of T_i is a border simplex if its circumball
// may contain a point of another partition.  Two tests:
//   grid (the paper's grid-based primitive): a uniform grid of cell edge
//     c_G (V/n)^(1/D) (about one input point per cell at c_G = 1) records
//     the partition owning each cell's points (or "mixed", or empty); the
//     ball is tested against the cells of other partitions (box-sphere);
//   region (default): the exact regions of the divide -- Voronoi cells of
//     the sample for the sample divide (searched over the sample's Delaunay
//     graph), boxes for the kd divide.  The circumball is computed in FP64 and
// enlarged by a bound far above its rounding error, and nearly flat
// simplices are always flagged, so the test can only over-flag.  Every
// simplex is tested, not only those reachable from the hull: partitions of
// the sample divide are unions of Voronoi cells and need not be convex.
// Hull cells of T_i (the infinite vertex) are always flagged, which is the
// conservative form of the test for the outer half-space of a hull facet.
//
// Merge: T = (union T_i minus B) plus every simplex of T_B that spans
// several partitions or whose vertex set is that of a simplex of B, found
// in an open-addressing hash table keyed by the sorted vertex ids.
#include <math.h>

#include "dt_block.hpp"
#include "dt_common.hpp"
#include "dt_geom.hpp"
#include "dt_internal.hpp"
#include "dt_pred.hpp"
#include "dt_prims.hpp"
#include "dt_stages.hpp"
#include "dt_region.hpp"

namespace dtk {

constexpr int MB = 256;
static inline uint32_t mblocks(uint64_t n) { return (uint32_t)((n + MB - 1) / MB); }
constexpr uint32_t OWN_EMPTY = 0xFFFFFFFFu;
constexpr uint32_t OWN_MIXED = 0xFFFFFFFEu;


__global__ void k_occupancy(const double4* P, const uint32_t* pset, uint32_t n, BGrid G,
                            uint32_t* owner) {
  uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double4 p = P[i];
  uint32_t c = ((uint32_t)bcoord(p.z, G, 2) * G.g[1] + bcoord(p.y, G, 1)) * G.g[0] + bcoord(p.x, G, 0);
  uint32_t me = pset[i];
  uint32_t cur = owner[c];
  if (cur == me || cur == OWN_MIXED) return;
  uint32_t old = atomicCAS(&owner[c], OWN_EMPTY, me);
  if (old != OWN_EMPTY && old != me) atomicExch(&owner[c], OWN_MIXED);
}

__device__ __forceinline__ uint32_t key_of(const double4* P, uint32_t v) {
  return (uint32_t)__double_as_longlong(P[v].w);
}

// Does the ball (ctr, r) of a simplex of partition `me` reach the region
// of another partition?  kd boxes: the ball leaves the block's box.
// Sample Voronoi cells: let t be the sample nearest to the centre; a point
// of the ball belongs to another block only if it is (up to rounding) at
// least as close to a foreign sample s as to t, which needs the ball to
// reach the bisector of s and t; such s lie within |t - ctr| + 2r of the
// centre.  Margins cover the rounding of the assignment's distance keys.
// hint: a sample of the own block to measure against (the test holds for
// any own sample; the one nearest the centre is the tightest).  Without a
// hint the centre's nearest sample is searched.
template <int D>
__device__ bool region_hit(const Region& R, uint32_t me, const double* ctr, double r,
                           uint32_t hint = 0xFFFFFFFFu) {
  if (R.kind == BORDER_BOXES) {
    const double* b = R.boxes + (size_t)me * 6;
    for (int k = 0; k < D; k++)
      if (ctr[k] - r <= b[k] || ctr[k] + r >= b[3 + k]) return true;
    return false;
  }
  double d2t;
  uint32_t t = hint;
  if (t == 0xFFFFFFFFu) {
    t = grid_nearest(R.S, R.start, R.items, R.G, ctr[0], ctr[1], D == 3 ? ctr[2] : 0.0, &d2t);
    if (R.part[t] != me) return true;
  } else {
    const double4 q = R.S[t];
    const double dx = ctr[0] - q.x, dy = ctr[1] - q.y, dz = (D == 3 ? ctr[2] : 0.0) - q.z;
    d2t = (dx * dx + dy * dy) + dz * dz;
  }
  double4 tp = R.S[t];
  double rad = sqrt(d2t) * (1.0 + 1e-9) + 2.0 * r;
  int lo[3], hi[3];
  for (int k = 0; k < 3; k++) {
    double x = k < D ? ctr[k] : 0.0;
    lo[k] = cell_coord(x - rad, R.G.lo[k], R.G.h, R.G.g[k]);
    hi[k] = cell_coord(x + rad, R.G.lo[k], R.G.h, R.G.g[k]);
  }
  double cz = D == 3 ? ctr[2] : 0.0;
  for (int z = lo[2]; z <= hi[2]; z++)
    for (int y = lo[1]; y <= hi[1]; y++)
      for (int x = lo[0]; x <= hi[0]; x++) {
        uint32_t cell = ((uint32_t)z * R.G.g[1] + y) * R.G.g[0] + x;
        for (uint32_t j = R.start[cell]; j < R.start[cell + 1]; j++) {
          uint32_t s = R.items[j];
          if (R.part[s] == me) continue;
          double4 sp = R.S[s];
          double ax = ctr[0] - sp.x, ay = ctr[1] - sp.y, az = cz - sp.z;
          double bx = ctr[0] - tp.x, by = ctr[1] - tp.y, bz = cz - tp.z;
          double ds = ax * ax + ay * ay + az * az, dt = bx * bx + by * by + bz * bz;
          double ex = sp.x - tp.x, ey = sp.y - tp.y, ez = sp.z - tp.z;
          double gap = sqrt(ex * ex + ey * ey + ez * ez);
          // distance of the centre from the bisector, on t's side: (ds - dt) / (2 gap)
          if (ds - dt <= 2.0 * gap * r + 1e-12 * (ds + dt)) return true;
        }
      }
  return false;
}

// Bounding box of every partition (one block per partition; the job's
// points are grouped by partition).
__global__ void k_part_boxes(const double4* pts, const uint32_t* set_off, double* boxes) {
  __shared__ double s_v[6][MB];
  const uint32_t s = blockIdx.x, lo = set_off[s], hi = set_off[s + 1];
  double v[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
  for (uint32_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
    const double4 q = pts[i];
    v[0] = fmin(v[0], q.x); v[1] = fmin(v[1], q.y); v[2] = fmin(v[2], q.z);
    v[3] = fmax(v[3], q.x); v[4] = fmax(v[4], q.y); v[5] = fmax(v[5], q.z);
  }
  for (int k = 0; k < 6; k++) s_v[k][threadIdx.x] = v[k];
  __syncthreads();
  for (uint32_t w = MB / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w)
      for (int k = 0; k < 6; k++)
        s_v[k][threadIdx.x] = k < 3 ? fmin(s_v[k][threadIdx.x], s_v[k][threadIdx.x + w])
                                    : fmax(s_v[k][threadIdx.x], s_v[k][threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x < 6) boxes[(size_t)s * 6 + threadIdx.x] = s_v[threadIdx.x][0];
}

__device__ __forceinline__ uint32_t grid_cell_of(const double4& p, const BGrid& G) {
  return ((uint32_t)bcoord(p.z, G, 2) * G.g[1] + bcoord(p.y, G, 1)) * G.g[0] + bcoord(p.x, G, 0);
}

// Points listed by grid cell (counting sort: count, scan, fill).
__global__ void k_cell_count(const double4* pts, uint32_t n, BGrid G, uint32_t* cnt) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) atomicAdd(&cnt[grid_cell_of(pts[i], G)], 1u);
}
__global__ void k_cell_fill(const double4* pts, uint32_t n, BGrid G, const uint32_t* start,
                            uint32_t* cur, uint32_t* items) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t c = grid_cell_of(pts[i], G);
  items[start[c] + atomicAdd(&cur[c], 1u)] = i;
}

// Exact test: is a point of another partition strictly inside the
// circumsphere of the (positively oriented) finite cell v, under the same
// perturbed in-sphere predicate as the triangulations?  The grid cells
// covering the inflated ball hold every such point.
template <int D>
__device__ bool exact_hit(const double4* P, const uint32_t* pset, const uint32_t* v, uint32_t me,
                          const double* ctr, double r, const BGrid& G, const Region& R,
                          uint32_t* flags) {
  int lo[3], hi[3];
  long ncover = 1;
  for (int k = 0; k < 3; k++) {
    if (k < D) {
      lo[k] = bcoord(ctr[k] - r, G, k);
      hi[k] = bcoord(ctr[k] + r, G, k);
    } else {
      lo[k] = hi[k] = 0;
    }
    ncover *= (hi[k] - lo[k] + 1);
  }
  if (ncover > 4096) return true;
  PredT<false> pr;
  pr.init(flags);
  PtsX X;
  for (int i = 0; i <= D; i++) {
    const double4 a = P[v[i]];
    X.p[i][0] = a.x; X.p[i][1] = a.y; X.p[i][2] = a.z;
    X.key[i] = (unsigned long long)__double_as_longlong(a.w);
  }
  for (int z = lo[2]; z <= hi[2]; z++)
    for (int y = lo[1]; y <= hi[1]; y++)
      for (int x = lo[0]; x <= hi[0]; x++) {
        const uint32_t cell = ((uint32_t)z * G.g[1] + y) * G.g[0] + x;
        for (uint32_t j = R.cstart[cell]; j < R.cstart[cell + 1]; j++) {
          const uint32_t q = R.citems[j];
          if (pset[q] == me) continue;
          const double4 b = P[q];
          X.p[D + 1][0] = b.x; X.p[D + 1][1] = b.y; X.p[D + 1][2] = b.z;
          X.key[D + 1] = (unsigned long long)__double_as_longlong(b.w);
          if (pr.template insphere<D>(X) > 0) return true;
        }
      }
  return false;
}

// Bounding-box test: does the ball meet the box of another partition?
template <int D>
__device__ bool bbox_hit(const Region& R, uint32_t me, const double* ctr, double r) {
  const double r2 = r * r;
  for (uint32_t j = 0; j < R.nparts; j++) {
    if (j == me) continue;
    const double* b = R.pboxes + (size_t)j * 6;
    if (!(b[0] <= b[3])) continue;   // empty partition
    double d2 = 0.0;
    for (int k = 0; k < D; k++) {
      const double t = ctr[k] < b[k] ? b[k] - ctr[k] : (ctr[k] > b[3 + k] ? ctr[k] - b[3 + k] : 0.0);
      d2 += t * t;
    }
    if (d2 <= r2) return true;
  }
  return false;
}

// Lower bound of a point's clearance from the foreign Voronoi cells: with t
// its own (assigned) sample, the least signed distance of the point from
// the bisector of t and any foreign sample s, on t's side.  Foreign samples
// within rho = |x - t| + h / 2 of the point are scanned; any other s is at
// least (rho - |x - t|) / 2 away from its bisector.  Each bisector distance
// is 1-Lipschitz in x, so a ball through the point of radius r with
// clearance above 2 r holds no point of another block.
template <int D>
__global__ void k_point_margin(const double4* pts, uint32_t n, const uint32_t* nearest,
                               Region R, double* margin, uint32_t* near_loc) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double4 q = pts[i];
  const uint32_t id = (uint32_t)__double_as_longlong(q.w);
  const uint32_t t = nearest[id];
  const uint32_t me = R.part[t];
  const double4 tp = R.S[t];
  const double qz = D == 3 ? q.z : 0.0;
  const double tx = q.x - tp.x, ty = q.y - tp.y, tz = qz - tp.z;
  const double dt = tx * tx + ty * ty + tz * tz;
  const double rt = sqrt(dt);
  const double rho = rt * (1.0 + 1e-9) + 0.5 * R.G.h;
  double f = 0.5 * (rho - rt * (1.0 + 1e-9));
  const double c[3] = {q.x, q.y, qz};
  int lo[3], hi[3];
  for (int k = 0; k < 3; k++) {
    lo[k] = cell_coord(c[k] - rho, R.G.lo[k], R.G.h, R.G.g[k]);
    hi[k] = cell_coord(c[k] + rho, R.G.lo[k], R.G.h, R.G.g[k]);
  }
  for (int z = lo[2]; z <= hi[2]; z++)
    for (int y = lo[1]; y <= hi[1]; y++)
      for (int x = lo[0]; x <= hi[0]; x++) {
        const uint32_t cell = ((uint32_t)z * R.G.g[1] + y) * R.G.g[0] + x;
        for (uint32_t j = R.start[cell]; j < R.start[cell + 1]; j++) {
          const uint32_t s = R.items[j];
          if (R.part[s] == me) continue;
          const double4 sp = R.S[s];
          const double ax = q.x - sp.x, ay = q.y - sp.y, az = qz - sp.z;
          const double ds = ax * ax + ay * ay + az * az;
          const double ex = sp.x - tp.x, ey = sp.y - tp.y, ez = sp.z - tp.z;
          const double gap = sqrt(ex * ex + ey * ey + ez * ez);
          // signed distance from the bisector, less the rounding slack of
          // the assignment keys (as in region_hit)
          const double d = (ds - dt - 1e-12 * (ds + dt)) / (2.0 * gap);
          f = fmin(f, d);
        }
      }
  // by the point's index in the job (cells' vertices index the job's
  // points, which are in spatial order: the border test's loads of
  // neighbouring vertices share cache lines)
  margin[i] = f;
  near_loc[i] = t;
}

// Barrier of one wavefront (LDS written by some lanes, read by others).
__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// The same clearance from a short list per sample.  For the sample t, the
// foreign samples (of other blocks) are ranked by their distance from t;
// the nearest ML of them are listed with their distance gap = |s - t|, and
// rho_t is half the distance of the nearest one not listed (infinite when
// all are listed).  A foreign sample s not listed has |s - t| >= 2 rho_t,
// and any point x that the assignment gives to s is at least about
// |s - t| / 2 from t (it is no farther from s than from t, up to the
// rounding of the keys), so for a point q of t's cell such an x lies at
// least rho_t - |q - t| from q.  The clearance of q is the least of that
// bound and the bisector distances of the listed samples: it needs no
// grid and no scan of the block's own samples.
constexpr uint32_t ML = 32;               // foreign samples listed per sample
constexpr uint32_t ML_MAX_SAMPLES = 65536;  // larger samples use the grid scan

// One wavefront per sample t: the (ML+1)-th smallest key (squared distance
// rounded to FP32, whose bit patterns order as the values) by four 8-bit
// radix passes over the foreign samples, then the samples with a smaller
// key are listed and the least distance of the others gives rho_t.
__global__ __launch_bounds__(64) void k_margin_lists(const double4* S, const uint32_t* part,
                                                     uint32_t ns, double4* lent, uint32_t* lcnt,
                                                     double* rho) {
  __shared__ uint32_t s_h[256];
  __shared__ uint32_t s_pick[2];
  const uint32_t t = blockIdx.x, lane = threadIdx.x;
  if (t >= ns) return;
  const uint32_t me = part[t];
  const double4 tp = S[t];
  auto key_of_s = [&](uint32_t s, double& gap2) {
    const double4 q = S[s];
    const double ex = q.x - tp.x, ey = q.y - tp.y, ez = q.z - tp.z;
    gap2 = ex * ex + ey * ey + ez * ez;
    return (uint32_t)__float_as_uint((float)gap2);
  };
  uint32_t nf = 0;
  for (uint32_t b = 0; b < ns; b += 64) {
    const uint32_t s = b + lane;
    nf += (uint32_t)__popcll(__ballot(s < ns && part[s] != me));
  }
  uint32_t thr = 0xFFFFFFFFu;   // keys below it are listed
  if (nf > ML) {
    uint32_t prefix = 0, pmask = 0, rank = ML;
    for (int shift = 24; shift >= 0; shift -= 8) {
      for (uint32_t j = lane; j < 256; j += 64) s_h[j] = 0;
      wave_sync_lds();
      for (uint32_t s = lane; s < ns; s += 64) {
        if (part[s] == me) continue;
        double g2;
        const uint32_t key = key_of_s(s, g2);
        if ((key & pmask) == prefix) atomicAdd(&s_h[(key >> shift) & 255u], 1u);
      }
      wave_sync_lds();
      if (lane == 0) {
        uint32_t below = 0, bin = 255;
        for (uint32_t j = 0; j < 256; j++) {
          if (below + s_h[j] > rank) { bin = j; break; }
          below += s_h[j];
        }
        s_pick[0] = bin;
        s_pick[1] = below;
      }
      wave_sync_lds();
      prefix |= s_pick[0] << shift;
      pmask |= 255u << shift;
      rank -= s_pick[1];
      wave_sync_lds();
    }
    thr = prefix;
  }
  uint32_t n = 0;
  double rmin = INFINITY;
  for (uint32_t b = 0; b < ns; b += 64) {
    const uint32_t s = b + lane;
    bool take = false;
    double g2 = 0.0;
    if (s < ns && part[s] != me) {
      const uint32_t key = key_of_s(s, g2);
      take = nf <= ML || key < thr;
      if (!take) rmin = fmin(rmin, sqrt(g2));
    }
    const unsigned long long m = __ballot(take);
    if (take) {
      const double4 q = S[s];
      lent[(size_t)t * ML + n + (uint32_t)__popcll(m & ((1ull << lane) - 1ull))] =
          make_double4(q.x, q.y, q.z, sqrt(g2));
    }
    n += (uint32_t)__popcll(m);
  }
  for (int o = 32; o > 0; o >>= 1) rmin = fmin(rmin, __shfl_xor(rmin, o, 64));
  if (lane == 0) {
    lcnt[t] = n;
    rho[t] = 0.5 * rmin;
  }
}

template <int D>
__global__ void k_point_margin_list(const double4* pts, uint32_t n, const uint32_t* nearest,
                                    const double4* S, const double4* lent, const uint32_t* lcnt,
                                    const double* rho, double* margin, uint32_t* near_loc) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double4 q = pts[i];
  const uint32_t id = (uint32_t)__double_as_longlong(q.w);
  const uint32_t t = nearest[id];
  const double4 tp = S[t];
  const double qz = D == 3 ? q.z : 0.0;
  const double tx = q.x - tp.x, ty = q.y - tp.y, tz = qz - tp.z;
  const double dt = tx * tx + ty * ty + tz * tz;
  const double rt = sqrt(dt);
  // the samples not listed: rho_t - |q - t|, with slack for the rounding
  // of both distances (rho_t is infinite when every foreign one is listed)
  double f = rho[t] * (1.0 - 1e-9) - rt * (1.0 + 1e-9);
  const uint32_t cnt = lcnt[t];
  const double4* e = lent + (size_t)t * ML;
  for (uint32_t j = 0; j < cnt; j++) {
    const double4 sp = e[j];
    const double ax = q.x - sp.x, ay = q.y - sp.y, az = qz - sp.z;
    const double ds = ax * ax + ay * ay + az * az;
    // signed distance from the bisector, less the rounding slack of the
    // assignment keys (as in k_point_margin)
    f = fmin(f, (ds - dt - 1e-12 * (ds + dt)) / (2.0 * sp.w));
  }
  margin[i] = f;
  near_loc[i] = t;
}

constexpr uint32_t NB_STRIPES = 64;   // copies of the border-simplex counter

// The test of one live cell c: flag it, and its vertices (vbflag), when
// its circumsphere may reach another partition.  finite: no vertex is the
// infinite one.  vis: the thread's slots in the walk's LDS list.  defer:
// a cell whose Voronoi test needs the walk over the sample's graph is left
// undecided (walk = true, nothing written) for a second pass.
template <int D>
__device__ __forceinline__ void border_cell(const double4* P, const uint32_t* pset,
                                            const Cell* cells, uint32_t c, const BGrid& G,
                                            const uint32_t* owner, const Region& R,
                                            uint32_t* vbflag, uint32_t* flags, uint32_t* vis,
                                            bool defer, bool& flag, bool& finite, bool& walk) {
  flag = false;
  finite = false;
  walk = false;
  uint4 v4 = cells[c].v;
  uint32_t v[4] = {v4.x, v4.y, v4.z, v4.w};
  bool inf = false;
#pragma unroll
  for (int i = 0; i <= D; i++)
    if (v[i] == INF_V) inf = true;
  if (inf) {
    flag = true;
  } else {
    finite = true;
    double ctr[3], r = 0.0;
    // the ball from the vertices in index order, so that its rounding (and
    // the decisions near the margins) depends on the simplex alone, not on
    // the order in which its cell lists them
    uint32_t w[4] = {v[0], v[1], v[2], v[3]};
#pragma unroll
    for (int i = 1; i <= D; i++)
#pragma unroll
      for (int j = i; j > 0; j--)
        if (w[j] < w[j - 1]) {
          const uint32_t t = w[j];
          w[j] = w[j - 1];
          w[j - 1] = t;
        }
    const bool sliver = !circumball<D>(P[w[0]], P[w[1]], P[w[2]], P[w[D == 3 ? 3 : 2]], ctr, &r);
    if (sliver) {
      flag = true;
    } else if (R.kind == BORDER_VORONOI && R.margin) {
      // clearance of the vertices first (every vertex lies on the sphere)
      double m = R.margin[v[0]];
#pragma unroll
      for (int i = 1; i <= D; i++) m = fmax(m, R.margin[v[i]]);
      if (!(m > 2.0 * r) && defer) {
        walk = true;
        return;
      }
      if (!(m > 2.0 * r)) {
        // the own sample nearest the centre among the vertices' samples
        uint32_t t = 0xFFFFFFFFu;
        double best = INFINITY;
        const double cz = D == 3 ? ctr[2] : 0.0;
#pragma unroll
        for (int i = 0; i <= D; i++) {
          const uint32_t s = R.near_loc[v[i]];
          const double4 q = R.S[s];
          const double dx = ctr[0] - q.x, dy = ctr[1] - q.y, dz = cz - q.z;
          const double d2 = (dx * dx + dy * dy) + dz * dz;
          if (d2 < best) { best = d2; t = s; }
        }
        flag = R.gadj ? voronoi_walk_hit<D, MB>(R, pset[v[0]], ctr, r, t, vis)
                      : region_hit<D>(R, pset[v[0]], ctr, r, t);
      }
      // refined: of the region test's simplices keep those whose sphere
      // really holds a point of another partition
      if (flag && R.refine) flag = exact_hit<D>(P, pset, v, pset[v[0]], ctr, r, G, R, flags);
    } else if (R.kind == BORDER_BBOX) {
      flag = bbox_hit<D>(R, pset[v[0]], ctr, r);
    } else if (R.kind == BORDER_EXACT) {
      flag = exact_hit<D>(P, pset, v, pset[v[0]], ctr, r, G, R, flags);
    } else if (R.kind != BORDER_GRID) {
      flag = region_hit<D>(R, pset[v[0]], ctr, r);
      if (flag && R.refine) flag = exact_hit<D>(P, pset, v, pset[v[0]], ctr, r, G, R, flags);
    } else {
      uint32_t me = pset[v[0]];
      int lo[3], hi[3];
      long ncover = 1;
      for (int k = 0; k < 3; k++) {
        if (k < D) {
          lo[k] = bcoord(ctr[k] - r, G, k);
          hi[k] = bcoord(ctr[k] + r, G, k);
        } else {
          lo[k] = hi[k] = 0;
        }
        ncover *= (hi[k] - lo[k] + 1);
      }
      if (ncover > 4096) {
        flag = true;
      } else {
        double r2 = r * r;
        for (int z = lo[2]; z <= hi[2] && !flag; z++)
          for (int y = lo[1]; y <= hi[1] && !flag; y++)
            for (int x = lo[0]; x <= hi[0] && !flag; x++) {
              uint32_t own = owner[((uint32_t)z * G.g[1] + y) * G.g[0] + x];
              if (own == OWN_EMPTY || own == me) continue;
              // squared distance from the centre to the grid cell (box)
              int cc[3] = {x, y, z};
              double d2 = 0.0;
              for (int k = 0; k < D; k++) {
                double bl = G.lo[k] + cc[k] * G.h, bh = bl + G.h;
                // the first and last cells extend to infinity (points are clamped)
                if (cc[k] == 0) bl = -INFINITY;
                if (cc[k] == G.g[k] - 1) bh = INFINITY;
                double t = ctr[k] < bl ? bl - ctr[k] : (ctr[k] > bh ? ctr[k] - bh : 0.0);
                d2 += t * t;
              }
              if (d2 <= r2) flag = true;
            }
      }
    }
  }
  if (flag) {
#pragma unroll
    for (int i = 0; i <= D; i++)
      if (v[i] != INF_V) vbflag[key_of(P, v[i])] = 1u;
  }
}

// Tiles of the cell pool.  The pool holds every cell ever created, about
// four for each live one (destroyed cells keep their records), so each
// wavefront takes a tile of BT * 64 consecutive cells, lists the ones it
// has to work on in LDS (from the cells' forward words, or from a bit mask
// of the tile), and then works on the listed cells with all its lanes.
// A block of MB threads takes BTILES_PER_BLOCK consecutive tiles.
constexpr uint32_t BT = 4;
constexpr uint32_t BTILE = BT * 64;
constexpr uint32_t BTILES_PER_BLOCK = MB / 64;
constexpr uint32_t BWORDS = BT * BTILES_PER_BLOCK;   // mask words of a block
static inline uint32_t btiles(uint64_t n) {
  return (uint32_t)((n + BTILE * BTILES_PER_BLOCK - 1) / (BTILE * BTILES_PER_BLOCK));
}

// The live cells of the wavefront's tile, in cell order, listed in LDS;
// returns their number (the same in every lane).
__device__ __forceinline__ uint32_t list_live(const Cell* cells, uint32_t ncells, uint32_t tile0,
                                              uint32_t lane, uint32_t* list) {
  uint32_t n = 0;
#pragma unroll
  for (uint32_t j = 0; j < BT; j++) {
    const uint32_t c = tile0 + j * 64 + lane;
    const bool alive = c < ncells && cells[c].fwd == ALIVE;
    const unsigned long long m = __ballot(alive);
    if (alive) list[n + (uint32_t)__popcll(m & ((1ull << lane) - 1ull))] = c;
    n += (uint32_t)__popcll(m);
  }
  wave_sync_lds();
  return n;
}

// The cells of the tile whose bits are set in its BT mask words.
__device__ __forceinline__ uint32_t list_masked(const unsigned long long* words, uint32_t tile0,
                                                uint32_t lane, uint32_t* list) {
  uint32_t n = 0;
#pragma unroll
  for (uint32_t j = 0; j < BT; j++) {
    const unsigned long long m = words[j];
    if ((m >> lane) & 1ull)
      list[n + (uint32_t)__popcll(m & ((1ull << lane) - 1ull))] = tile0 + j * 64 + lane;
    n += (uint32_t)__popcll(m);
  }
  wave_sync_lds();
  return n;
}

// Border test of every live cell.  Output per tile: two bit masks over its
// cells, emitm (finite and not flagged: output as it is) and hashm (finite
// and flagged: the border simplices B), and the border vertices (vbflag).
template <int D>
__global__ void k_border(const double4* P, const uint32_t* pset, const Cell* cells,
                         uint32_t ncells, BGrid G, const uint32_t* owner, Region R,
                         unsigned long long* emitm, unsigned long long* hashm,
                         uint32_t* vbflag, unsigned long long* nb, uint32_t* flags) {
  __shared__ uint32_t s_vis[VW_CAP * MB];
  __shared__ uint32_t s_live[BTILES_PER_BLOCK][BTILE];
  __shared__ unsigned long long s_em[BTILES_PER_BLOCK][BT], s_hm[BTILES_PER_BLOCK][BT];
  const uint32_t lane = threadIdx.x & 63u, w = threadIdx.x >> 6;
  const uint32_t tile0 = (blockIdx.x * BTILES_PER_BLOCK + w) * BTILE;
  if (lane < BT) {
    s_em[w][lane] = 0;
    s_hm[w][lane] = 0;
  }
  uint32_t* live = s_live[w];
  const uint32_t nlive = list_live(cells, ncells, tile0, lane, live);
  unsigned long long cnt = 0;
  // First pass: every cell the cheap tests decide; the cells whose Voronoi
  // test needs the walk are listed again (at the front of the same list,
  // behind the entries already read) and walked in a second pass with all
  // lanes.
  uint32_t nwalk = 0;
  for (uint32_t b = 0; b < nlive; b += 64) {
    bool flag = false, finite = false, walk = false;
    uint32_t c = 0;
    if (b + lane < nlive) {
      c = live[b + lane];
      border_cell<D>(P, pset, cells, c, G, owner, R, vbflag, flags, s_vis + threadIdx.x, true,
                     flag, finite, walk);
      const uint32_t o = c - tile0;
      if (finite && !walk)
        atomicOr(flag ? &s_hm[w][o >> 6] : &s_em[w][o >> 6], 1ull << (o & 63u));
    }
    cnt += (unsigned long long)__popcll(__ballot(flag && finite));
    const unsigned long long m = __ballot(walk);
    wave_sync_lds();
    if (walk) live[nwalk + (uint32_t)__popcll(m & ((1ull << lane) - 1ull))] = c;
    nwalk += (uint32_t)__popcll(m);
    wave_sync_lds();
  }
  for (uint32_t b = 0; b < nwalk; b += 64) {
    bool flag = false, finite = false, walk = false;
    if (b + lane < nwalk) {
      const uint32_t c = live[b + lane];
      border_cell<D>(P, pset, cells, c, G, owner, R, vbflag, flags, s_vis + threadIdx.x, false,
                     flag, finite, walk);
      const uint32_t o = c - tile0;
      if (finite) atomicOr(flag ? &s_hm[w][o >> 6] : &s_em[w][o >> 6], 1ull << (o & 63u));
    }
    cnt += (unsigned long long)__popcll(__ballot(flag && finite));
  }
  wave_sync_lds();
  if (lane < BT) {
    emitm[tile0 / 64 + lane] = s_em[w][lane];
    hashm[tile0 / 64 + lane] = s_hm[w][lane];
  }
  // striped count (one address for every wavefront would serialise)
  if (lane == 0 && cnt)
    atomicAdd(&nb[(blockIdx.x * BTILES_PER_BLOCK + w) % NB_STRIPES], cnt);
}

// Points of partitions that have no full-dimensional triangulation (fewer
// than D+1 points or all in one hyperplane) all join the border set.
__global__ void k_degenerate_parts(const double4* P, const uint32_t* pset, uint32_t n,
                                   const uint32_t* set_cell0, uint32_t* vbflag) {
  uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (set_cell0[pset[i]] == DONE) vbflag[key_of(P, i)] = 1u;
}

int border_detect(const LocalJob& job, const CellPool& pool, const Region& reg, uint32_t n,
                  int D, double cells_target, const double lo[3], const double hi[3],
                  BorderOut& out, hipStream_t st) {
  uint64_t total = 1;
  const BGrid G = make_bgrid(lo, hi, D, cells_target, &total);
  const bool grid = reg.kind == BORDER_GRID;
  DevBuf owner, vbflag, nb, margin, near_loc;
  DT_TRY(owner.alloc(grid ? total * 4 : 16));
  DT_TRY(vbflag.alloc((size_t)n * 4));
  const size_t nwords = (size_t)btiles(pool.ncells) * BWORDS;
  DT_TRY(out.emitm.alloc((nwords ? nwords : 1) * 8));
  DT_TRY(out.hashm.alloc((nwords ? nwords : 1) * 8));
  out.nwords = nwords;
  DT_TRY(nb.alloc(NB_STRIPES * 8));
  DT_HIP(hipMemsetAsync(vbflag.p, 0, (size_t)n * 4, st));
  DT_HIP(hipMemsetAsync(nb.p, 0, NB_STRIPES * 8, st));
  if (grid) {
    // occupancy of the grid cells (only the grid primitive uses it)
    DT_HIP(hipMemsetAsync(owner.p, 0xFF, total * 4, st));
    hipLaunchKernelGGL(k_occupancy, dim3(mblocks(job.npts)), dim3(MB), 0, st, job.pts, job.pset,
                       job.npts, G, owner.as<uint32_t>());
  }
  Region R = reg;
  DevBuf pflags, pboxes, cstart, ccount, ccur, citems;
  DT_TRY(pflags.alloc(4));
  DT_HIP(hipMemsetAsync(pflags.p, 0, 4, st));
  if (reg.kind == BORDER_BBOX && job.nsets) {
    DT_TRY(pboxes.alloc((size_t)job.nsets * 6 * sizeof(double)));
    hipLaunchKernelGGL(k_part_boxes, dim3(job.nsets), dim3(MB), 0, st, job.pts, job.set_off,
                       pboxes.as<double>());
    R.pboxes = pboxes.as<double>();
    R.nparts = job.nsets;
  }
  if (reg.kind == BORDER_EXACT || reg.refine) {
    // the job's points listed by grid cell
    DT_TRY(ccount.alloc((total + 1) * 4));
    DT_TRY(cstart.alloc((total + 1) * 4));
    DT_TRY(ccur.alloc(total * 4));
    DT_TRY(citems.alloc((size_t)(job.npts ? job.npts : 1) * 4));
    DT_HIP(hipMemsetAsync(ccount.p, 0, (total + 1) * 4, st));
    DT_HIP(hipMemsetAsync(ccur.p, 0, total * 4, st));
    hipLaunchKernelGGL(k_cell_count, dim3(mblocks(job.npts)), dim3(MB), 0, st, job.pts, job.npts,
                       G, ccount.as<uint32_t>());
    DT_TRY(exclusive_scan(ccount.as<uint32_t>(), cstart.as<uint32_t>(), (uint32_t)total + 1, st));
    hipLaunchKernelGGL(k_cell_fill, dim3(mblocks(job.npts)), dim3(MB), 0, st, job.pts, job.npts,
                       G, cstart.as<uint32_t>(), ccur.as<uint32_t>(), citems.as<uint32_t>());
    R.cstart = cstart.as<uint32_t>();
    R.citems = citems.as<uint32_t>();
  }
  DevBuf lent, lcnt, lrho;
  const bool lists = reg.kind == BORDER_VORONOI && reg.nearest && job.npts && reg.ns > 0 &&
                     reg.ns <= ML_MAX_SAMPLES;
  if (lists) {
    DT_TRY(lent.alloc((size_t)reg.ns * ML * sizeof(double4)));
    DT_TRY(lcnt.alloc((size_t)reg.ns * 4));
    DT_TRY(lrho.alloc((size_t)reg.ns * 8));
    hipLaunchKernelGGL(k_margin_lists, dim3(reg.ns), dim3(64), 0, st, reg.S, reg.part, reg.ns,
                       lent.as<double4>(), lcnt.as<uint32_t>(), lrho.as<double>());
  }
  DT_PROF_BEGIN(DT_KERN_BORDER, st);
  if (lists) {
    DT_TRY(margin.alloc((size_t)job.npts * sizeof(double)));
    DT_TRY(near_loc.alloc((size_t)job.npts * 4));
    if (D == 2)
      hipLaunchKernelGGL(k_point_margin_list<2>, dim3(mblocks(job.npts)), dim3(MB), 0, st,
                         job.pts, job.npts, reg.nearest, reg.S, lent.as<double4>(),
                         lcnt.as<uint32_t>(), lrho.as<double>(), margin.as<double>(),
                         near_loc.as<uint32_t>());
    else
      hipLaunchKernelGGL(k_point_margin_list<3>, dim3(mblocks(job.npts)), dim3(MB), 0, st,
                         job.pts, job.npts, reg.nearest, reg.S, lent.as<double4>(),
                         lcnt.as<uint32_t>(), lrho.as<double>(), margin.as<double>(),
                         near_loc.as<uint32_t>());
    R.margin = margin.as<double>();
    R.near_loc = near_loc.as<uint32_t>();
  } else if (reg.kind == BORDER_VORONOI && reg.nearest && job.npts) {
    DT_TRY(margin.alloc((size_t)job.npts * sizeof(double)));
    DT_TRY(near_loc.alloc((size_t)job.npts * sizeof(uint32_t)));
    if (D == 2)
      hipLaunchKernelGGL(k_point_margin<2>, dim3(mblocks(job.npts)), dim3(MB), 0, st, job.pts,
                         job.npts, reg.nearest, reg, margin.as<double>(),
                         near_loc.as<uint32_t>());
    else
      hipLaunchKernelGGL(k_point_margin<3>, dim3(mblocks(job.npts)), dim3(MB), 0, st, job.pts,
                         job.npts, reg.nearest, reg, margin.as<double>(),
                         near_loc.as<uint32_t>());
    R.margin = margin.as<double>();
    R.near_loc = near_loc.as<uint32_t>();
  }
  if (pool.ncells == 0) {
    // nothing to test (every partition degenerate)
  } else if (D == 2)
    hipLaunchKernelGGL(k_border<2>, dim3(btiles(pool.ncells)), dim3(MB), 0, st, job.pts,
                       job.pset, pool.cells.as<Cell>(), pool.ncells, G,
                       owner.as<uint32_t>(), R, out.emitm.as<unsigned long long>(),
                       out.hashm.as<unsigned long long>(), vbflag.as<uint32_t>(),
                       nb.as<unsigned long long>(), pflags.as<uint32_t>());
  else
    hipLaunchKernelGGL(k_border<3>, dim3(btiles(pool.ncells)), dim3(MB), 0, st, job.pts,
                       job.pset, pool.cells.as<Cell>(), pool.ncells, G,
                       owner.as<uint32_t>(), R, out.emitm.as<unsigned long long>(),
                       out.hashm.as<unsigned long long>(), vbflag.as<uint32_t>(),
                       nb.as<unsigned long long>(), pflags.as<uint32_t>());
  DT_PROF_END(st);
  hipLaunchKernelGGL(k_degenerate_parts, dim3(mblocks(job.npts)), dim3(MB), 0, st, job.pts,
                     job.pset, job.npts, pool.set_cell0.as<uint32_t>(), vbflag.as<uint32_t>());
  DT_HIP(hipGetLastError());
  unsigned long long hnbs[NB_STRIPES];
  uint32_t hpf = 0;
  DT_HIP(hipMemcpyAsync(hnbs, nb.p, NB_STRIPES * 8, hipMemcpyDeviceToHost, st));
  DT_HIP(hipMemcpyAsync(&hpf, pflags.p, 4, hipMemcpyDeviceToHost, st));
  DT_HIP(hipStreamSynchronize(st));
  if (hpf) return DT_E_INTERNAL;   // the exact predicate ran out of expansion capacity
  unsigned long long hnb = 0;
  for (uint32_t i = 0; i < NB_STRIPES; i++) hnb += hnbs[i];
  out.nb_finite = hnb;
  DT_TRY(compact_indices(vbflag.as<uint32_t>(), n, out.vb, &out.nvb, st));
  return DT_OK;
}

// ------------------------------------------------------------ merge
__device__ __forceinline__ void sorted_keys(const double4* P, uint4 v, int D, uint32_t k[4]) {
  uint32_t vv[4] = {v.x, v.y, v.z, v.w};
  for (int i = 0; i <= D; i++) k[i] = key_of(P, vv[i]);
  for (int i = 1; i <= D; i++)
    for (int j = i; j > 0 && k[j] < k[j - 1]; j--) {
      uint32_t t = k[j]; k[j] = k[j - 1]; k[j - 1] = t;
    }
  if (D == 2) k[3] = 0;
}

__device__ __forceinline__ uint32_t hkey(const uint32_t k[4]) {
  unsigned long long h = ((unsigned long long)k[0] << 32 | k[1]) * 0x9E3779B97F4A7C15ull;
  h ^= ((unsigned long long)k[2] << 32 | k[3]) * 0xC2B2AE3D27D4EB4Full;
  h ^= h >> 29;
  return (uint32_t)(h * 0xBF58476D1CE4E5B9ull >> 32);
}


template <int D>
__device__ __forceinline__ void write_row(int32_t* rows, uint32_t slot, const uint32_t k[4]) {
#pragma unroll
  for (int i = 0; i <= D; i++) rows[(size_t)slot * (D + 1) + i] = (int32_t)k[i];
}

// The merge runs in two passes over each pool, so that the output needs no
// atomic cursor and comes out in cell order: a marking pass (per block:
// the number of cells to output, and the number of finite cells for the
// statistics; local flagged cells go into the table, border cells are
// looked up in it), a scan of the block counts, and a writing pass.  The
// passes work on tiles (above): the local pool's from the border test's
// masks, the border pool's from the forward words and then a mask of its
// own.

// Sum over the lanes of a wavefront.
__device__ __forceinline__ uint32_t wave_total(uint32_t v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Cells to output and finite cells of a block, from its mask words
// (wavefront 0 counts; the others return 0).
__device__ __forceinline__ void block_mask_counts(const unsigned long long* emitm,
                                                  const unsigned long long* finm, uint32_t& ne,
                                                  uint32_t& nf) {
  const uint32_t t = threadIdx.x;
  const size_t wd = (size_t)blockIdx.x * BWORDS + t;
  uint32_t e = 0, f = 0;
  if (t < BWORDS) {
    const unsigned long long em = emitm[wd];
    e = (uint32_t)__popcll(em);
    f = finm ? e + (uint32_t)__popcll(finm[wd]) : 0u;
  }
  ne = t < 64 ? wave_total(e) : 0u;
  nf = t < 64 ? wave_total(f) : 0u;
}

// Local pass 1: the flagged finite cells (B) go into the table; the block
// counts come from the masks.
template <int D>
__global__ void k_merge_mark_local(const double4* P, const Cell* cells,
                                   const unsigned long long* emitm,
                                   const unsigned long long* hashm, uint32_t* occ, uint4* tkeys,
                                   uint32_t tmask, uint32_t* bemit, uint32_t* bfinite,
                                   uint32_t* flags) {
  __shared__ uint32_t s_list[BTILES_PER_BLOCK][BTILE];
  const uint32_t lane = threadIdx.x & 63u, w = threadIdx.x >> 6;
  const uint32_t tile0 = (blockIdx.x * BTILES_PER_BLOCK + w) * BTILE;
  uint32_t* list = s_list[w];
  const uint32_t nh = list_masked(hashm + tile0 / 64, tile0, lane, list);
  for (uint32_t b = lane; b < nh; b += 64) {
    uint32_t k[4];
    sorted_keys(P, cells[list[b]].v, D, k);
    const uint32_t h = hkey(k);
    for (uint32_t pr = 0; pr <= tmask; pr++) {
      const uint32_t s = (h + pr) & tmask;
      if (atomicCAS(&occ[s], 0u, 1u) == 0u) {
        tkeys[s] = make_uint4(k[0], k[1], k[2], k[3]);
        break;
      }
      if (pr == tmask) atomicOr(flags, FAIL_HASH);
    }
  }
  uint32_t ne, nf;
  block_mask_counts(emitm, hashm, ne, nf);
  if (threadIdx.x == 0) {
    bemit[blockIdx.x] = ne;
    bfinite[blockIdx.x] = nf;
  }
}

// Pass 2 of either pool: write the cells of the emit mask, the block's at
// its offset, in cell order.
template <int D>
__global__ void k_merge_write(const double4* P, const Cell* cells,
                              const unsigned long long* emitm, const uint32_t* boff,
                              uint32_t base, int32_t* rows) {
  __shared__ uint32_t s_list[BTILES_PER_BLOCK][BTILE];
  const uint32_t lane = threadIdx.x & 63u, w = threadIdx.x >> 6;
  const uint32_t tile0 = (blockIdx.x * BTILES_PER_BLOCK + w) * BTILE;
  uint32_t* list = s_list[w];
  // rows of the block's earlier tiles
  uint32_t before = 0;
  for (uint32_t x = 0; x < w * BT; x++)
    before += (uint32_t)__popcll(emitm[(size_t)blockIdx.x * BWORDS + x]);
  const uint32_t ne = list_masked(emitm + tile0 / 64, tile0, lane, list);
  const uint32_t at = base + boff[blockIdx.x] + before;
  for (uint32_t b = lane; b < ne; b += 64) {
    uint32_t k[4];
    sorted_keys(P, cells[list[b]].v, D, k);
    write_row<D>(rows, at + b, k);
  }
}

// Border pass 1: a finite cell of T_B is output if it spans several
// partitions or its vertex set is in B; the decision is kept in a mask.
template <int D>
__global__ void k_merge_mark_border(const double4* P, const Cell* cells,
                                    uint32_t ncells, const uint32_t* pid_by_id,
                                    const uint32_t* occ, const uint4* tkeys, uint32_t tmask,
                                    unsigned long long* emitm, uint32_t* bemit,
                                    uint32_t* bfinite, unsigned long long* probe_hist) {
  // probe-length histogram: per block in LDS, one global add per bin
  __shared__ uint32_t s_hist[16];
  __shared__ uint32_t s_list[BTILES_PER_BLOCK][BTILE];
  __shared__ unsigned long long s_em[BTILES_PER_BLOCK][BT];
  __shared__ uint32_t s_fin;
  if (threadIdx.x < 16) s_hist[threadIdx.x] = 0;
  if (threadIdx.x == 0) s_fin = 0;
  const uint32_t lane = threadIdx.x & 63u, w = threadIdx.x >> 6;
  const uint32_t tile0 = (blockIdx.x * BTILES_PER_BLOCK + w) * BTILE;
  if (lane < BT) s_em[w][lane] = 0;
  __syncthreads();
  uint32_t* list = s_list[w];
  const uint32_t nlive = list_live(cells, ncells, tile0, lane, list);
  uint32_t nfin = 0;
  for (uint32_t b = lane; b < nlive; b += 64) {
    const uint32_t c = list[b];
    const uint4 v = cells[c].v;
    if (v.x == INF_V || v.y == INF_V || v.z == INF_V || (D == 3 && v.w == INF_V)) continue;
    nfin++;
    uint32_t k[4];
    sorted_keys(P, v, D, k);
    const uint32_t p0 = pid_by_id[k[0]];
    bool span = false;
#pragma unroll
    for (int i = 1; i <= D; i++)
      if (pid_by_id[k[i]] != p0) span = true;
    bool emit = span;
    if (!span) {
      const uint32_t h = hkey(k);
      uint32_t pr = 0;
      for (; pr <= tmask; pr++) {
        const uint32_t s = (h + pr) & tmask;
        if (occ[s] == 0u) break;
        const uint4 t = tkeys[s];
        if (t.x == k[0] && t.y == k[1] && t.z == k[2] && t.w == k[3]) {
          emit = true;
          break;
        }
      }
      atomicAdd(&s_hist[pr < 15 ? pr : 15], 1u);
    }
    const uint32_t o = c - tile0;
    if (emit) atomicOr(&s_em[w][o >> 6], 1ull << (o & 63u));
  }
  nfin = wave_total(nfin);
  if (lane == 0 && nfin) atomicAdd(&s_fin, nfin);
  __syncthreads();
  if (lane < BT) emitm[tile0 / 64 + lane] = s_em[w][lane];
  uint32_t ne = 0;
  if (threadIdx.x < 64) {
    const uint32_t t = threadIdx.x;
    const uint32_t e = t < BWORDS ? (uint32_t)__popcll(s_em[t / BT][t % BT]) : 0u;
    ne = wave_total(e);
  }
  if (threadIdx.x == 0) {
    bemit[blockIdx.x] = ne;
    bfinite[blockIdx.x] = s_fin;
  }
  if (threadIdx.x < 16 && s_hist[threadIdx.x])
    atomicAdd(&probe_hist[threadIdx.x], (unsigned long long)s_hist[threadIdx.x]);
}

// Sum of n block counts: exclusive offsets into off[0..n], total returned.
static int scan_counts(DevBuf& cnt, DevBuf& off, uint32_t n, uint32_t* total, hipStream_t st) {
  DT_HIP(hipMemsetAsync(cnt.as<uint32_t>() + n, 0, 4, st));
  DT_TRY(exclusive_scan(cnt.as<uint32_t>(), off.as<uint32_t>(), n + 1, st));
  DT_HIP(hipMemcpyAsync(total, off.as<uint32_t>() + n, 4, hipMemcpyDeviceToHost, st));
  DT_HIP(hipStreamSynchronize(st));
  return DT_OK;
}

int merge_output(const LocalJob& job, const CellPool& pool, const BorderOut& b,
                 const LocalJob& bjob, const CellPool& bpool, const uint32_t* pid_by_id, int D,
                 DevBuf& rows, int64_t* m, int64_t* local_finite, int64_t* border_finite,
                 int64_t probe_hist[16], hipStream_t st) {
  uint32_t tsize = 64;
  while (tsize < 2 * b.nb_finite + 16) tsize <<= 1;
  const uint32_t nbl = btiles(pool.ncells), nbb = btiles(bpool.ncells);
  DevBuf occ, tkeys, hist, flags, lemit, lfin, loff, bemit, bfin, boff, bemitm, junk;
  DT_TRY(occ.alloc((size_t)tsize * 4));
  DT_TRY(tkeys.alloc((size_t)tsize * 16));
  DT_TRY(hist.alloc(16 * 8));
  DT_TRY(flags.alloc(4));
  DT_TRY(lemit.alloc((size_t)(nbl + 1) * 4));
  DT_TRY(lfin.alloc((size_t)(nbl + 1) * 4));
  DT_TRY(loff.alloc((size_t)(nbl + 1) * 4));
  DT_TRY(bemit.alloc((size_t)(nbb + 1) * 4));
  DT_TRY(bfin.alloc((size_t)(nbb + 1) * 4));
  DT_TRY(boff.alloc((size_t)(nbb + 1) * 4));
  DT_TRY(bemitm.alloc((size_t)(nbb ? nbb : 1) * BWORDS * 8));
  DT_TRY(junk.alloc((size_t)(((nbl > nbb) ? nbl : nbb) + 1) * 4));
  DT_HIP(hipMemsetAsync(occ.p, 0, (size_t)tsize * 4, st));
  DT_HIP(hipMemsetAsync(hist.p, 0, 16 * 8, st));
  DT_HIP(hipMemsetAsync(flags.p, 0, 4, st));
  DT_PROF_BEGIN(DT_KERN_MERGE, st);
  if (pool.ncells) {
    if (D == 2)
      hipLaunchKernelGGL(k_merge_mark_local<2>, dim3(nbl), dim3(MB), 0, st, job.pts,
                         pool.cells.as<Cell>(), b.emitm.as<unsigned long long>(),
                         b.hashm.as<unsigned long long>(), occ.as<uint32_t>(), tkeys.as<uint4>(),
                         tsize - 1, lemit.as<uint32_t>(), lfin.as<uint32_t>(),
                         flags.as<uint32_t>());
    else
      hipLaunchKernelGGL(k_merge_mark_local<3>, dim3(nbl), dim3(MB), 0, st, job.pts,
                         pool.cells.as<Cell>(), b.emitm.as<unsigned long long>(),
                         b.hashm.as<unsigned long long>(), occ.as<uint32_t>(), tkeys.as<uint4>(),
                         tsize - 1, lemit.as<uint32_t>(), lfin.as<uint32_t>(),
                         flags.as<uint32_t>());
  }
  if (bpool.ncells) {
    if (D == 2)
      hipLaunchKernelGGL(k_merge_mark_border<2>, dim3(nbb), dim3(MB), 0, st, bjob.pts,
                         bpool.cells.as<Cell>(), bpool.ncells,
                         pid_by_id, occ.as<uint32_t>(), tkeys.as<uint4>(), tsize - 1,
                         bemitm.as<unsigned long long>(), bemit.as<uint32_t>(),
                         bfin.as<uint32_t>(), hist.as<unsigned long long>());
    else
      hipLaunchKernelGGL(k_merge_mark_border<3>, dim3(nbb), dim3(MB), 0, st, bjob.pts,
                         bpool.cells.as<Cell>(), bpool.ncells,
                         pid_by_id, occ.as<uint32_t>(), tkeys.as<uint4>(), tsize - 1,
                         bemitm.as<unsigned long long>(), bemit.as<uint32_t>(),
                         bfin.as<uint32_t>(), hist.as<unsigned long long>());
  }
  DT_PROF_END(st);
  DT_HIP(hipGetLastError());
  uint32_t nl = 0, nb = 0, fl = 0, fb = 0;
  if (pool.ncells) {
    DT_TRY(scan_counts(lemit, loff, nbl, &nl, st));
    DT_TRY(scan_counts(lfin, junk, nbl, &fl, st));
  }
  if (bpool.ncells) {
    DT_TRY(scan_counts(bemit, boff, nbb, &nb, st));
    DT_TRY(scan_counts(bfin, junk, nbb, &fb, st));
  }
  const uint64_t total = (uint64_t)nl + nb;
  DT_TRY(rows.alloc_plain((size_t)(total ? total : 1) * (D + 1) * 4));
  DT_PROF_BEGIN(DT_KERN_MERGE, st);
  if (nl) {
    if (D == 2)
      hipLaunchKernelGGL(k_merge_write<2>, dim3(nbl), dim3(MB), 0, st, job.pts,
                         pool.cells.as<Cell>(), b.emitm.as<unsigned long long>(),
                         loff.as<uint32_t>(), 0u, rows.as<int32_t>());
    else
      hipLaunchKernelGGL(k_merge_write<3>, dim3(nbl), dim3(MB), 0, st, job.pts,
                         pool.cells.as<Cell>(), b.emitm.as<unsigned long long>(),
                         loff.as<uint32_t>(), 0u, rows.as<int32_t>());
  }
  if (nb) {
    if (D == 2)
      hipLaunchKernelGGL(k_merge_write<2>, dim3(nbb), dim3(MB), 0, st, bjob.pts,
                         bpool.cells.as<Cell>(), bemitm.as<unsigned long long>(),
                         boff.as<uint32_t>(), nl, rows.as<int32_t>());
    else
      hipLaunchKernelGGL(k_merge_write<3>, dim3(nbb), dim3(MB), 0, st, bjob.pts,
                         bpool.cells.as<Cell>(), bemitm.as<unsigned long long>(),
                         boff.as<uint32_t>(), nl, rows.as<int32_t>());
  }
  DT_PROF_END(st);
  DT_HIP(hipGetLastError());
  uint32_t hf = 0;
  unsigned long long hh[16];
  DT_HIP(hipMemcpyAsync(&hf, flags.p, 4, hipMemcpyDeviceToHost, st));
  DT_HIP(hipMemcpyAsync(hh, hist.p, 16 * 8, hipMemcpyDeviceToHost, st));
  DT_HIP(hipStreamSynchronize(st));
  if (hf) return DT_E_INTERNAL;
  *m = (int64_t)total;
  *local_finite = fl;
  *border_finite = fb;
  for (int i = 0; i < 16; i++) probe_hist[i] = (int64_t)hh[i];
  return DT_OK;
}

}  // namespace dtk
