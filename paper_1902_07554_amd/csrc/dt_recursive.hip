// Recursive bisection (Section "Recursive Bisection"): log2 k levels of
// 2-way division, then k-1 merges bottom-up.  This is the scheme of the
// original divide-and-conquer triangulation (cyclic median split) and its
// sample-based variant (a new sample per block and level); the one-shot
// k-way division of Algorithm 1 is in dt_dc.hip.
//
// Division: every level splits every block in two; the leaf index of a
// point spells its path from the root (bit 1 = upper half), so its block
// at the level with 2^l blocks is leaf >> (log2 k - l).
//   kd:     the cyclic median split (kd_divide);
//   sample: Algorithm 2 with k = 2 in every block: the eta(|block|) points
//           of smallest random key form the block's sample; the samples of
//           all blocks are triangulated in one batched run; each block's
//           sample graph (its Delaunay edges, weighted as in Table
//           "weights") is cut in two by the partitioner (a median split of
//           the sample along its widest axis, refined by label
//           propagation under the balance bound); every point of the block
//           takes the side of its nearest sample of the block, under the
//           key (fl(d^2), id).
// Merging (level by level, all parents of a level in one batched run):
// the triangulations of the two children of a parent are known as simplex
// lists; a simplex is a border simplex when its ball may reach the
// sibling's region (the region test: the sibling's Voronoi cells of the
// level's sample, or the sibling's kd box; or, on request, the grid test
// against cells holding points of the sibling); the hull facets of each
// child add their vertices; the border vertices of every parent are
// triangulated together; the parent keeps the children's other simplices
// and the border triangulation's simplices that span both children or are
// border simplices themselves (the merge of Algorithm 1 with k = 2).
#include <math.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "dt_common.hpp"
#include "dt_geom.hpp"
#include "dt_internal.hpp"
#include "dt_pipeline.hpp"
#include "dt_prep.hpp"
#include "dt_prims.hpp"
#include "dt_stages.hpp"
#include "dt_region.hpp"

namespace dtk {

namespace {

constexpr int RB = 256;
constexpr uint32_t OWN_EMPTY = 0xFFFFFFFFu;
constexpr uint32_t OWN_MIXED = 0xFFFFFFFEu;

inline uint32_t rblocks(uint64_t n) { return (uint32_t)((n + RB - 1) / RB); }

__device__ __forceinline__ uint64_t mix64r(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// set of item i: the s with off[s] <= i < off[s+1]
__device__ __forceinline__ uint32_t seg_of(const uint32_t* off, uint32_t nseg, uint32_t i) {
  uint32_t lo = 0, hi = nseg;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (off[mid] <= i) lo = mid;
    else hi = mid;
  }
  return lo;
}

// ---- sample bisection
// key: block, then a random key of the point (the sample of a block is a
// prefix of its segment after sorting)
__global__ void k_rb_sample_keys(uint32_t n, const uint32_t* pid, uint64_t salt,
                                 unsigned long long* keys, uint32_t* vals) {
  const uint32_t i = blockIdx.x * RB + threadIdx.x;
  if (i >= n) return;
  keys[i] = ((unsigned long long)pid[i] << 40) | (mix64r(salt ^ (uint64_t)i) >> 24);
  vals[i] = i;
}

// nearest sample of the point's own block (grid over this level's samples;
// samples of other blocks are skipped; exact argmin of (fl(d^2), id))
__global__ void k_rb_assign(const double4* P, uint32_t n, const double4* S, const uint32_t* sblock,
                            const uint32_t* slabel, const uint32_t* start, const uint32_t* items,
                            Grid G, uint32_t* pid, uint32_t* nearest) {
  const uint32_t i = blockIdx.x * RB + threadIdx.x;
  if (i >= n) return;
  const double4 p = P[i];
  const uint32_t me = pid[i];
  int c[3] = {cell_coord(p.x, G.lo[0], G.h, G.g[0]), cell_coord(p.y, G.lo[1], G.h, G.g[1]),
              cell_coord(p.z, G.lo[2], G.h, G.g[2])};
  const double pc[3] = {p.x, p.y, p.z};
  double best = INFINITY;
  long long bestid = 0x7FFFFFFFFFFFFFFFll;
  uint32_t bests = 0xFFFFFFFFu;
  const int gmax = max(G.g[0], max(G.g[1], G.g[2]));
  for (int r = 0; r <= gmax; r++) {
    int lo[3], hi[3];
    for (int k = 0; k < 3; k++) {
      lo[k] = max(c[k] - r, 0);
      hi[k] = min(c[k] + r, G.g[k] - 1);
    }
    for (int z = lo[2]; z <= hi[2]; z++)
      for (int y = lo[1]; y <= hi[1]; y++) {
        const bool edge = (z == c[2] - r) || (z == c[2] + r) || (y == c[1] - r) || (y == c[1] + r);
        for (int x = lo[0]; x <= hi[0]; x++) {
          if (!edge && x != c[0] - r && x != c[0] + r) {
            if (x < c[0] + r) x = c[0] + r - 1;
            continue;
          }
          const uint32_t cell = ((uint32_t)z * G.g[1] + y) * G.g[0] + x;
          for (uint32_t j = start[cell]; j < start[cell + 1]; j++) {
            const uint32_t s = items[j];
            if (sblock[s] != me) continue;
            const double4 q = S[s];
            const double dx = p.x - q.x, dy = p.y - q.y, dz = p.z - q.z;
            const double d2 = (dx * dx + dy * dy) + dz * dz;
            const long long sid = __double_as_longlong(q.w);
            if (d2 < best || (d2 == best && sid < bestid)) {
              best = d2;
              bestid = sid;
              bests = s;
            }
          }
        }
      }
    bool all = true;
    double dmin = INFINITY;
    for (int k = 0; k < 3; k++) {
      if (c[k] - r > 0) {
        all = false;
        dmin = fmin(dmin, pc[k] - (G.lo[k] + (c[k] - r) * G.h));
      }
      if (c[k] + r < G.g[k] - 1) {
        all = false;
        dmin = fmin(dmin, (G.lo[k] + (c[k] + r + 1) * G.h) - pc[k]);
      }
    }
    if (all) break;
    if (best < INFINITY) {
      const double dm = fmax(dmin, 0.0) * (1.0 - 1e-9);
      if (dm * dm > best * (1.0 + 1e-9)) break;
    }
  }
  pid[i] = 2 * me + (bests == 0xFFFFFFFFu ? 0u : (slabel[bests] & 1u));
  nearest[i] = bests;
}

// the samples of every block: slot j of block b takes the (j - soff[b])-th
// point of b's segment of the (block, random key) order
__global__ void k_rb_take(const uint32_t* sorted, const uint32_t* seg, const uint32_t* soff,
                          uint32_t nb, uint32_t ns, uint32_t* sidx, uint32_t* sblk) {
  const uint32_t j = blockIdx.x * RB + threadIdx.x;
  if (j >= ns) return;
  const uint32_t b = seg_of(soff, nb, j);
  sidx[j] = sorted[seg[b] + (j - soff[b])];
  sblk[j] = b;
}

// order-preserving unsigned image of a double
__device__ __forceinline__ unsigned long long ord_of(double x) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(x);
  return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}

// bounding box of every block's sample (ordered images, atomic min / max)
__global__ void k_rb_sbox(const double4* S, const uint32_t* sblk, uint32_t ns, int D,
                          unsigned long long* bmin, unsigned long long* bmax) {
  const uint32_t j = blockIdx.x * RB + threadIdx.x;
  if (j >= ns) return;
  const double4 q = S[j];
  const double c[3] = {q.x, q.y, q.z};
  const uint32_t b = sblk[j];
  for (int a = 0; a < D; a++) {
    atomicMin(&bmin[(size_t)b * 3 + a], ord_of(c[a]));
    atomicMax(&bmax[(size_t)b * 3 + a], ord_of(c[a]));
  }
}

__device__ __forceinline__ double dbl_of(unsigned long long o) {
  const unsigned long long u = (o >> 63) ? (o & 0x7FFFFFFFFFFFFFFFull) : ~o;
  return __longlong_as_double((long long)u);
}

// sort key of a sample: its block, then its coordinate along the block
// sample's widest axis (the median split of the partitioner's initial cut)
__global__ void k_rb_axis_keys(const double4* S, const uint32_t* sblk, uint32_t ns, int D,
                               int lbits, const unsigned long long* bmin,
                               const unsigned long long* bmax, unsigned long long* keys,
                               uint32_t* vals) {
  const uint32_t j = blockIdx.x * RB + threadIdx.x;
  if (j >= ns) return;
  const uint32_t b = sblk[j];
  int ax = 0;
  double wmax = -1.0;
  for (int a = 0; a < D; a++) {
    const double w = dbl_of(bmax[(size_t)b * 3 + a]) - dbl_of(bmin[(size_t)b * 3 + a]);
    if (w > wmax) { wmax = w; ax = a; }
  }
  const double4 q = S[j];
  const double c = ax == 0 ? q.x : (ax == 1 ? q.y : q.z);
  keys[j] = ((unsigned long long)b << (64 - lbits)) | (ord_of(c) >> lbits);
  vals[j] = j;
}

// first cut: the lower half (floor) of every block's sample along its axis
// is side 0; label = 2 * block + side
__global__ void k_rb_first_side(const uint32_t* vals, const uint32_t* sblk, const uint32_t* off,
                                uint32_t ns, uint32_t* label) {
  const uint32_t q = blockIdx.x * RB + threadIdx.x;
  if (q >= ns) return;
  const uint32_t j = vals[q];
  const uint32_t b = sblk[j];
  const uint32_t m = off[b + 1] - off[b];
  label[j] = 2 * b + ((q - off[b]) < m / 2 ? 0u : 1u);
}

__global__ void k_rb_grid_count(const double4* S, uint32_t m, Grid G, uint32_t* cnt,
                                uint32_t* cellof) {
  const uint32_t i = blockIdx.x * RB + threadIdx.x;
  if (i >= m) return;
  const double4 q = S[i];
  const uint32_t c = ((uint32_t)cell_coord(q.z, G.lo[2], G.h, G.g[2]) * G.g[1] +
                      cell_coord(q.y, G.lo[1], G.h, G.g[1])) * G.g[0] +
                     cell_coord(q.x, G.lo[0], G.h, G.g[0]);
  cellof[i] = c;
  atomicAdd(&cnt[c], 1u);
}
__global__ void k_rb_grid_fill(uint32_t m, const uint32_t* cellof, const uint32_t* start,
                               uint32_t* cur, uint32_t* items) {
  const uint32_t i = blockIdx.x * RB + threadIdx.x;
  if (i >= m) return;
  const uint32_t c = cellof[i];
  items[start[c] + atomicAdd(&cur[c], 1u)] = i;
}

// ---- merging
// tag of every row (its block at the current level) from the row offsets
__global__ void k_rb_row_tags(const uint32_t* off, uint32_t nseg, uint32_t m, uint32_t* tag) {
  const uint32_t i = blockIdx.x * RB + threadIdx.x;
  if (i < m) tag[i] = seg_of(off, nseg, i);
}

__global__ void k_rb_occupancy(const double4* P, uint32_t n, const uint32_t* leaf, int shift,
                               BGrid G, uint32_t* owner) {
  const uint32_t i = blockIdx.x * RB + threadIdx.x;
  if (i >= n) return;
  const double4 p = P[i];
  const uint32_t c = ((uint32_t)bcoord(p.z, G, 2) * G.g[1] + bcoord(p.y, G, 1)) * G.g[0] +
                     bcoord(p.x, G, 0);
  const uint32_t me = leaf[i] >> shift;
  const uint32_t cur = owner[c];
  if (cur == me || cur == OWN_MIXED) return;
  const uint32_t old = atomicCAS(&owner[c], OWN_EMPTY, me);
  if (old != OWN_EMPTY && old != me) atomicExch(&owner[c], OWN_MIXED);
}

// border simplices of the children: the ball reaches a grid cell holding
// points of the sibling (or of several blocks); hull facets of a child add
// their vertices.
template <int D>
__global__ void k_rb_border(const double4* P, const int32_t* rows, uint32_t m,
                            const uint32_t* tag, const int32_t* nbr, BGrid G,
                            const uint32_t* owner, uint8_t* flag, uint32_t* vbflag,
                            unsigned long long* nb) {
  const uint32_t i = blockIdx.x * RB + threadIdx.x;
  bool f = false;
  if (i < m) {
    uint32_t v[4] = {0, 0, 0, 0};
    for (int j = 0; j <= D; j++) v[j] = (uint32_t)rows[(size_t)i * (D + 1) + j];
    const uint32_t me = tag[i];
    double ctr[3], r = 0.0;
    if (!circumball<D>(P[v[0]], P[v[1]], P[v[2]], P[v[D == 3 ? 3 : 2]], ctr, &r)) {
      f = true;
    } else {
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
        f = true;
      } else {
        const double r2 = r * r;
        for (int z = lo[2]; z <= hi[2] && !f; z++)
          for (int y = lo[1]; y <= hi[1] && !f; y++)
            for (int x = lo[0]; x <= hi[0] && !f; x++) {
              const uint32_t own = owner[((uint32_t)z * G.g[1] + y) * G.g[0] + x];
              if (own == OWN_EMPTY || own == me) continue;
              if (own != OWN_MIXED && (own >> 1) != (me >> 1)) continue;   // not the sibling
              const int cc[3] = {x, y, z};
              double d2 = 0.0;
              for (int k = 0; k < D; k++) {
                double bl = G.lo[k] + cc[k] * G.h, bh = bl + G.h;
                if (cc[k] == 0) bl = -INFINITY;
                if (cc[k] == G.g[k] - 1) bh = INFINITY;
                const double t = ctr[k] < bl ? bl - ctr[k] : (ctr[k] > bh ? ctr[k] - bh : 0.0);
                d2 += t * t;
              }
              if (d2 <= r2) f = true;
            }
      }
    }
    if (f)
      for (int j = 0; j <= D; j++) vbflag[v[j]] = 1u;
    // hull facets of the child
    for (int j = 0; j <= D; j++)
      if (nbr[(size_t)i * (D + 1) + j] < 0)
        for (int t = 0; t <= D; t++)
          if (t != j) vbflag[v[t]] = 1u;
    flag[i] = f ? 1 : 0;
  }
  const unsigned long long b = __ballot(f);
  if ((threadIdx.x & 63) == 0 && b) atomicAdd(nb, (unsigned long long)__popcll(b));
}

// border simplices of the children by the region test: the ball reaches
// the sibling's Voronoi cells of the level's sample (a walk over the
// sample's Delaunay graph from the vertices' nearest sample), or leaves the
// child's kd box; hull facets of a child add their vertices.
template <int D>
__global__ __launch_bounds__(RB) void k_rb_border_region(
    const double4* P, const int32_t* rows, uint32_t m, const uint32_t* tag, const int32_t* nbr,
    Region R, const uint32_t* nearest, const double* cbox, uint8_t* flag, uint32_t* vbflag,
    unsigned long long* nb) {
  __shared__ uint32_t s_vis[VW_CAP * RB];
  const uint32_t i = blockIdx.x * RB + threadIdx.x;
  bool f = false;
  if (i < m) {
    uint32_t v[4] = {0, 0, 0, 0};
    for (int j = 0; j <= D; j++) v[j] = (uint32_t)rows[(size_t)i * (D + 1) + j];
    const uint32_t me = tag[i];
    double ctr[3], r = 0.0;
    if (!circumball<D>(P[v[0]], P[v[1]], P[v[2]], P[v[D == 3 ? 3 : 2]], ctr, &r)) {
      f = true;
    } else if (cbox) {
      const double* b = cbox + (size_t)me * 6;
      for (int k = 0; k < D; k++)
        if (ctr[k] - r <= b[k] || ctr[k] + r >= b[3 + k]) f = true;
    } else {
      // the own sample nearest the centre among the vertices' samples
      uint32_t t = nearest[v[0]];
      double best = INFINITY;
      const double cz = D == 3 ? ctr[2] : 0.0;
      for (int j = 0; j <= D; j++) {
        const uint32_t sj = nearest[v[j]];
        const double4 q = R.S[sj];
        const double dx = ctr[0] - q.x, dy = ctr[1] - q.y, dz = cz - q.z;
        const double d2 = (dx * dx + dy * dy) + dz * dz;
        if (d2 < best) { best = d2; t = sj; }
      }
      // a sample without Delaunay neighbours belongs to a block whose
      // sample has no full-dimensional triangulation: no walk, flagged
      f = R.goff[t + 1] == R.goff[t] ||
          voronoi_walk_hit<D, RB>(R, me, ctr, r, t, s_vis + threadIdx.x);
    }
    if (f)
      for (int j = 0; j <= D; j++) vbflag[v[j]] = 1u;
    for (int j = 0; j <= D; j++)
      if (nbr[(size_t)i * (D + 1) + j] < 0)
        for (int t = 0; t <= D; t++)
          if (t != j) vbflag[v[t]] = 1u;
    flag[i] = f ? 1 : 0;
  }
  const unsigned long long b = __ballot(f);
  if ((threadIdx.x & 63) == 0 && b) atomicAdd(nb, (unsigned long long)__popcll(b));
}

__global__ void k_rb_parent_keys(const uint32_t* vb, uint32_t nvb, const uint32_t* leaf,
                                 int shift, unsigned long long* keys, uint32_t* vals) {
  const uint32_t i = blockIdx.x * RB + threadIdx.x;
  if (i >= nvb) return;
  keys[i] = leaf[vb[i]] >> shift;
  vals[i] = vb[i];
}

__device__ __forceinline__ uint32_t hkey4(const uint32_t k[4]) {
  unsigned long long h = ((unsigned long long)k[0] << 32 | k[1]) * 0x9E3779B97F4A7C15ull;
  h ^= ((unsigned long long)k[2] << 32 | k[3]) * 0xC2B2AE3D27D4EB4Full;
  h ^= h >> 29;
  return (uint32_t)(h * 0xBF58476D1CE4E5B9ull >> 32);
}

// flagged rows into the table of B (keys: sorted ids, unique over all parents)
template <int D>
__global__ void k_rb_table(const int32_t* rows, uint32_t m, const uint8_t* flag, uint32_t* occ,
                           uint4* tkeys, uint32_t tmask, uint32_t* fail) {
  const uint32_t i = blockIdx.x * RB + threadIdx.x;
  if (i >= m || !flag[i]) return;
  uint32_t k[4] = {0, 0, 0, 0};
  for (int j = 0; j <= D; j++) k[j] = (uint32_t)rows[(size_t)i * (D + 1) + j];
  const uint32_t h = hkey4(k);
  for (uint32_t pr = 0; pr <= tmask; pr++) {
    const uint32_t s = (h + pr) & tmask;
    if (atomicCAS(&occ[s], 0u, 1u) == 0u) {
      tkeys[s] = make_uint4(k[0], k[1], k[2], k[3]);
      return;
    }
  }
  atomicOr(fail, FAIL_HASH);
}

// rows kept per parent: count pass and write pass (parent = tag >> 1 for
// the children's rows, the set for the border triangulation's cells)
template <int D>
__global__ void k_rb_keep_local(const int32_t* rows, uint32_t m, const uint32_t* tag,
                                const uint8_t* flag, const uint32_t* base, uint32_t* cur,
                                int32_t* out) {
  const uint32_t i = blockIdx.x * RB + threadIdx.x;
  if (i >= m || flag[i]) return;
  const uint32_t par = tag[i] >> 1;
  if (!out) {
    atomicAdd(&cur[par], 1u);
    return;
  }
  const uint32_t slot = base[par] + atomicAdd(&cur[par], 1u);
  for (int j = 0; j <= D; j++) out[(size_t)slot * (D + 1) + j] = rows[(size_t)i * (D + 1) + j];
}

template <int D>
__global__ void k_rb_keep_border(const double4* Pb, const uint32_t* bset, const Cell* cells,
                                 uint32_t ncells, const uint32_t* leaf, int shift,
                                 const uint32_t* occ, const uint4* tkeys, uint32_t tmask,
                                 const uint32_t* base, uint32_t* cur, int32_t* out) {
  const uint32_t c = blockIdx.x * RB + threadIdx.x;
  if (c >= ncells || cells[c].fwd != ALIVE) return;
  const uint4 v = cells[c].v;
  const uint32_t vv[4] = {v.x, v.y, v.z, v.w};
  uint32_t k[4] = {0, 0, 0, 0};
  for (int j = 0; j <= D; j++) {
    if (vv[j] == INF_V) return;
    k[j] = (uint32_t)__double_as_longlong(Pb[vv[j]].w);
  }
  for (int a = 1; a <= D; a++)
    for (int b = a; b > 0 && k[b] < k[b - 1]; b--) {
      const uint32_t t = k[b]; k[b] = k[b - 1]; k[b - 1] = t;
    }
  const uint32_t side0 = leaf[k[0]] >> shift;
  bool keep = false;
  for (int j = 1; j <= D; j++)
    if ((leaf[k[j]] >> shift) != side0) keep = true;
  if (!keep) {
    const uint32_t h = hkey4(k);
    for (uint32_t pr = 0; pr <= tmask; pr++) {
      const uint32_t s = (h + pr) & tmask;
      if (occ[s] == 0u) break;
      const uint4 t = tkeys[s];
      if (t.x == k[0] && t.y == k[1] && t.z == k[2] && t.w == k[3]) {
        keep = true;
        break;
      }
    }
  }
  if (!keep) return;
  const uint32_t par = bset[vv[0]];
  if (!out) {
    atomicAdd(&cur[par], 1u);
    return;
  }
  const uint32_t slot = base[par] + atomicAdd(&cur[par], 1u);
  for (int j = 0; j <= D; j++) out[(size_t)slot * (D + 1) + j] = (int32_t)k[j];
}

__global__ void k_rb_leaf_keys(const uint32_t* leaf, uint32_t n, unsigned long long* keys,
                               uint32_t* vals) {
  const uint32_t i = blockIdx.x * RB + threadIdx.x;
  if (i >= n) return;
  keys[i] = leaf[i];
  vals[i] = i;
}

__global__ void k_rb_key_lo(const unsigned long long* keys, uint32_t n, uint32_t* out) {
  const uint32_t i = blockIdx.x * RB + threadIdx.x;
  if (i < n) out[i] = (uint32_t)keys[i];
}

__global__ void k_rb_setof(const uint32_t* off, uint32_t nsets, uint32_t n, uint32_t* pset) {
  const uint32_t i = blockIdx.x * RB + threadIdx.x;
  if (i < n) pset[i] = seg_of(off, nsets, i);
}

uint32_t rb_sample_size(uint32_t m, double rate, int D) {
  double e = (rate == 0.0) ? floor(sqrt((double)m) + 0.5) : floor(rate * (double)m + 0.5);
  if (e < D + 2) e = D + 2;
  if (e > m) e = m;
  return (uint32_t)e;
}

// batch of point sets from per-set point lists: points gathered by index,
// sets in order, spatial order inside each set
int make_job(const DevBuf& P, const uint32_t* idx, uint32_t m, const uint32_t* set_of_item,
             uint32_t nsets, int D, const double lo[3], const double hi[3], bool fp32,
             const dt_options& o, DevBuf& pts, DevBuf& pset, DevBuf& off, LocalJob& job,
             hipStream_t st) {
  DevBuf cnt;
  DT_TRY(pts.alloc((size_t)(m ? m : 1) * sizeof(double4)));
  DT_TRY(gather_points(P.as<double4>(), idx, m, pts.as<double4>(), st));
  DT_TRY(cnt.alloc((size_t)(nsets + 1) * 4));
  DT_TRY(off.alloc((size_t)(nsets + 1) * 4));
  DT_TRY(count_by(set_of_item, m, nsets + 1, cnt.as<uint32_t>(), st));
  DT_TRY(exclusive_scan(cnt.as<uint32_t>(), off.as<uint32_t>(), nsets + 1, st));
  DT_TRY(pset.alloc((size_t)(m ? m : 1) * 4));
  hipLaunchKernelGGL(k_rb_setof, dim3(rblocks(m)), dim3(RB), 0, st, off.as<uint32_t>(), nsets, m,
                     pset.as<uint32_t>());
  int sbits = 0;
  while ((1u << sbits) < nsets) sbits++;
  DT_TRY(spatial_sort(pts, m, D, lo, hi, nsets > 1 ? pset.as<uint32_t>() : nullptr, sbits, st));
  job = LocalJob();
  job.D = D;
  job.npts = m;
  job.nsets = nsets;
  job.pts = pts.as<double4>();
  job.pset = pset.as<uint32_t>();
  job.set_off = off.as<uint32_t>();
  job.fp32 = fp32;
  job.tune(o);
  return DT_OK;
}

// The regions of one level of the sample bisection, kept for its merge:
// the level's samples (a batched job, grouped by block), the label 2 *
// block + side of every sample, the samples' Delaunay graph, and the
// nearest sample (of its own block) of every point.
struct LevelRegion {
  DevBuf pts, pset, off, label, goff, gadj, gw, nearest;
  uint32_t ns = 0;
};

// Leaf index of every point by sample bisection (Algorithm 2 with k = 2 in
// every block of every level).
int sample_bisect(const DevBuf& P, uint32_t n, int D, int levels, double rate,
                  const dt_options& o, const double lo[3], const double hi[3], Ctx& cx,
                  dt_stats& S, DevBuf& pid, std::vector<LevelRegion>& lv, hipStream_t st) {
  const bool fp32 = o.precision == DT_PREC_FP32;
  double dstar = 0.0;
  for (int a = 0; a < 3; a++) dstar += (hi[a] - lo[a]) * (hi[a] - lo[a]);
  dstar = sqrt(dstar);
  DT_TRY(pid.alloc((size_t)n * 4));
  DT_HIP(hipMemsetAsync(pid.p, 0, (size_t)n * 4, st));
  DevBuf keys, vals;
  DT_TRY(keys.alloc((size_t)n * 8));
  DT_TRY(vals.alloc((size_t)n * 4));
  lv.clear();
  lv.resize(levels);
  for (int l = 0; l < levels; l++) {
    LevelRegion& L = lv[l];
    const uint32_t nb = 1u << l;
    // points per block, then every block's points by random key
    DevBuf cnt;
    DT_TRY(cnt.alloc((size_t)nb * 4));
    DT_TRY(count_by(pid.as<uint32_t>(), n, nb, cnt.as<uint32_t>(), st));
    std::vector<uint32_t> hc(nb);
    DT_HIP(hipMemcpyAsync(hc.data(), cnt.p, (size_t)nb * 4, hipMemcpyDeviceToHost, st));
    hipLaunchKernelGGL(k_rb_sample_keys, dim3(rblocks(n)), dim3(RB), 0, st, n,
                       pid.as<uint32_t>(), o.seed ^ (0xD1B54A32D192ED03ull * (uint64_t)(l + 1)),
                       keys.as<unsigned long long>(), vals.as<uint32_t>());
    DT_TRY(radix_sort_pairs(keys.as<unsigned long long>(), vals.as<uint32_t>(), n, 40 + l, st));
    DT_HIP(hipStreamSynchronize(st));
    // sample sizes eta(|block|) and their places
    std::vector<uint32_t> seg(nb + 1, 0), soff(nb + 1, 0);
    std::vector<int> lmax(2 * nb);
    for (uint32_t b = 0; b < nb; b++) {
      const uint32_t eta = hc[b] ? rb_sample_size(hc[b], rate, D) : 0;
      seg[b + 1] = seg[b] + hc[b];
      soff[b + 1] = soff[b] + eta;
      const double half = ceil(eta / 2.0);
      lmax[2 * b] = lmax[2 * b + 1] = (int)floor((1.0 + o.eps) * half + 1e-9);
    }
    const uint32_t ns = soff[nb];
    L.ns = ns;
    DevBuf dseg, dsoff, sidx, sblk, dlmax;
    DT_TRY(dseg.alloc((size_t)(nb + 1) * 4));
    DT_TRY(dsoff.alloc((size_t)(nb + 1) * 4));
    DT_TRY(sidx.alloc((size_t)(ns ? ns : 1) * 4));
    DT_TRY(sblk.alloc((size_t)(ns ? ns : 1) * 4));
    DT_TRY(dlmax.alloc((size_t)2 * nb * 4));
    DT_HIP(hipMemcpyAsync(dseg.p, seg.data(), (size_t)(nb + 1) * 4, hipMemcpyHostToDevice, st));
    DT_HIP(hipMemcpyAsync(dsoff.p, soff.data(), (size_t)(nb + 1) * 4, hipMemcpyHostToDevice, st));
    DT_HIP(hipMemcpyAsync(dlmax.p, lmax.data(), (size_t)2 * nb * 4, hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_rb_take, dim3(rblocks(ns)), dim3(RB), 0, st, vals.as<uint32_t>(),
                       dseg.as<uint32_t>(), dsoff.as<uint32_t>(), nb, ns, sidx.as<uint32_t>(),
                       sblk.as<uint32_t>());
    DT_HIP(hipGetLastError());
    // the samples of all blocks triangulated in one batched run
    LocalJob sjob;
    DT_TRY(make_job(P, sidx.as<uint32_t>(), ns, sblk.as<uint32_t>(), nb, D, lo, hi, fp32, o, L.pts,
                    L.pset, L.off, sjob, st));
    CellPool spool;
    {
      K4Stats ks;
      int s = k4_run(sjob, spool, cx.dc(), cx.hctr, st, ks);
      for (int i = 0; i < 4; i++)
        for (int j = 0; j < 4; j++) S.pred[i][j] += (int64_t)ks.pred[i][j];
      S.rounds += ks.rounds;
      S.large_cavities += ks.giant_rounds;
      if (s != DT_OK) { S.fail = cx.hctr->flags; return s; }
    }
    S.eta += ns;
    // every block's sample graph cut in two: a median split along the
    // widest axis of the block's sample, refined by label propagation
    DT_TRY(sample_graph(L.pts.as<double4>(), ns, D, spool, o.weight, dstar, L.goff, L.gadj, L.gw,
                        st));
    spool = CellPool();
    DevBuf bmin, bmax, ak, av;
    DT_TRY(bmin.alloc((size_t)nb * 3 * 8));
    DT_TRY(bmax.alloc((size_t)nb * 3 * 8));
    DT_TRY(ak.alloc((size_t)(ns ? ns : 1) * 8));
    DT_TRY(av.alloc((size_t)(ns ? ns : 1) * 4));
    DT_TRY(L.label.alloc((size_t)(ns ? ns : 1) * 4));
    DT_HIP(hipMemsetAsync(bmin.p, 0xFF, (size_t)nb * 3 * 8, st));
    DT_HIP(hipMemsetAsync(bmax.p, 0, (size_t)nb * 3 * 8, st));
    hipLaunchKernelGGL(k_rb_sbox, dim3(rblocks(ns)), dim3(RB), 0, st, L.pts.as<double4>(),
                       L.pset.as<uint32_t>(), ns, D, bmin.as<unsigned long long>(),
                       bmax.as<unsigned long long>());
    hipLaunchKernelGGL(k_rb_axis_keys, dim3(rblocks(ns)), dim3(RB), 0, st, L.pts.as<double4>(),
                       L.pset.as<uint32_t>(), ns, D, l ? l : 1, bmin.as<unsigned long long>(),
                       bmax.as<unsigned long long>(), ak.as<unsigned long long>(),
                       av.as<uint32_t>());
    DT_HIP(hipGetLastError());
    DT_TRY(radix_sort_pairs(ak.as<unsigned long long>(), av.as<uint32_t>(), ns, 64, st));
    hipLaunchKernelGGL(k_rb_first_side, dim3(rblocks(ns)), dim3(RB), 0, st, av.as<uint32_t>(),
                       L.pset.as<uint32_t>(), L.off.as<uint32_t>(), ns, L.label.as<uint32_t>());
    DT_HIP(hipGetLastError());
    DT_TRY(refine_partition(ns, L.goff.as<uint32_t>(), L.gadj.as<uint32_t>(), L.gw.as<double>(),
                            L.label.as<uint32_t>(), 2 * nb, 0, dlmax.as<int>(), o.refine_iters,
                            o.refine_swaps == 0, st));
    // every point takes the side of its nearest sample of its own block
    // (grid of about ns/2 cells over the input box)
    Grid G;
    {
      double vol = 1.0;
      int nd = 0;
      for (int a = 0; a < D; a++)
        if (hi[a] > lo[a]) { vol *= hi[a] - lo[a]; nd++; }
      const double target = ns / 2.0 > 1.0 ? ns / 2.0 : 1.0;
      double h = nd ? pow(vol / target, 1.0 / nd) : 1.0;
      if (!(h > 0)) h = 1.0;
      for (int a = 0; a < 3; a++) {
        G.lo[a] = lo[a];
        long g = a < D ? (long)floor((hi[a] - lo[a]) / h) + 1 : 1;
        G.g[a] = (int)std::max(1L, std::min(g, 1024L));
      }
      G.h = h;
    }
    const uint32_t ncell = (uint32_t)G.g[0] * G.g[1] * G.g[2];
    DevBuf gcnt, gstart, gcur, gitems, gcell;
    DT_TRY(gcnt.alloc((size_t)(ncell + 1) * 4));
    DT_TRY(gstart.alloc((size_t)(ncell + 1) * 4));
    DT_TRY(gcur.alloc((size_t)ncell * 4));
    DT_TRY(gitems.alloc((size_t)(ns ? ns : 1) * 4));
    DT_TRY(gcell.alloc((size_t)(ns ? ns : 1) * 4));
    DT_HIP(hipMemsetAsync(gcnt.p, 0, (size_t)(ncell + 1) * 4, st));
    DT_HIP(hipMemsetAsync(gcur.p, 0, (size_t)ncell * 4, st));
    hipLaunchKernelGGL(k_rb_grid_count, dim3(rblocks(ns)), dim3(RB), 0, st, L.pts.as<double4>(),
                       ns, G, gcnt.as<uint32_t>(), gcell.as<uint32_t>());
    DT_TRY(exclusive_scan(gcnt.as<uint32_t>(), gstart.as<uint32_t>(), ncell + 1, st));
    hipLaunchKernelGGL(k_rb_grid_fill, dim3(rblocks(ns)), dim3(RB), 0, st, ns,
                       gcell.as<uint32_t>(), gstart.as<uint32_t>(), gcur.as<uint32_t>(),
                       gitems.as<uint32_t>());
    DT_TRY(L.nearest.alloc((size_t)n * 4));
    hipLaunchKernelGGL(k_rb_assign, dim3(rblocks(n)), dim3(RB), 0, st, P.as<double4>(), n,
                       L.pts.as<double4>(), L.pset.as<uint32_t>(), L.label.as<uint32_t>(),
                       gstart.as<uint32_t>(), gitems.as<uint32_t>(), G, pid.as<uint32_t>(),
                       L.nearest.as<uint32_t>());
    DT_HIP(hipGetLastError());
    DT_HIP(hipStreamSynchronize(st));
  }
  return DT_OK;
}

}  // namespace

int run_recursive(const double* points, int64_t n64, int D, int k, double rate,
                  const dt_options& o, bool on_device, hipStream_t st, dt_result* r) {
  double t0 = now_ms();
  dt_stats& S = r->stats;
  S.n = n64;
  S.D = D;
  S.k = k;
  const uint32_t n = (uint32_t)n64;
  if (k < 2 || (k & (k - 1)) != 0 || (uint32_t)k > n) return DT_E_INVALID_ARG;
  int levels = 0;
  while ((1 << levels) < k) levels++;
  const int divide = o.divide == DT_DIVIDE_KD ? DT_DIVIDE_KD : DT_DIVIDE_SAMPLE;
  S.divide_used = divide;
  const bool fp32 = o.precision == DT_PREC_FP32;
  Ctx cx;
  DT_TRY(cx.init());
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
  din.release();
  scratch.release();
  double lo[3], hi[3];
  DT_TRY(bbox(P.as<double4>(), n, lo, hi, st));
  double t1 = now_ms();
  S.stage_ms[DT_STAGE_VALIDATE] = t1 - t0;

  // ---- division into k leaves
  DevBuf leaf, boxes;
  std::vector<LevelRegion> lv;
  std::vector<double> hbox;
  const bool region = o.border != DT_BORDER_GRID;
  if (divide == DT_DIVIDE_KD) {
    DT_TRY(kd_divide(P.as<double4>(), n, D, (uint32_t)k, leaf, boxes, st));
    hbox.resize((size_t)k * 6);
    DT_HIP(hipMemcpyAsync(hbox.data(), boxes.p, (size_t)k * 6 * 8, hipMemcpyDeviceToHost, st));
    DT_HIP(hipStreamSynchronize(st));
  } else {
    DT_TRY(sample_bisect(P, n, D, levels, rate, o, lo, hi, cx, S, leaf, lv, st));
  }
  double t2 = now_ms();
  S.stage_ms[DT_STAGE_ASSIGN] = t2 - t1;

  // ---- leaf triangulations: points sorted by leaf (stable), one set per leaf
  DevBuf leafjob_pts, leafjob_set, leafjob_off, lkeys, lorder, lsorted;
  DT_TRY(lkeys.alloc((size_t)n * 8));
  DT_TRY(lorder.alloc((size_t)n * 4));
  DT_TRY(lsorted.alloc((size_t)n * 4));
  hipLaunchKernelGGL(k_rb_leaf_keys, dim3(rblocks(n)), dim3(RB), 0, st, leaf.as<uint32_t>(), n,
                     lkeys.as<unsigned long long>(), lorder.as<uint32_t>());
  DT_TRY(radix_sort_pairs(lkeys.as<unsigned long long>(), lorder.as<uint32_t>(), n, levels, st));
  hipLaunchKernelGGL(k_rb_key_lo, dim3(rblocks(n)), dim3(RB), 0, st,
                     lkeys.as<unsigned long long>(), n, lsorted.as<uint32_t>());
  LocalJob job;
  DT_TRY(make_job(P, lorder.as<uint32_t>(), n, lsorted.as<uint32_t>(), (uint32_t)k, D, lo, hi,
                  fp32, o, leafjob_pts, leafjob_set, leafjob_off, job, st));
  lkeys.release();
  CellPool pool;
  {
    K4Stats ks;
    int s = k4_run(job, pool, cx.dc(), cx.hctr, st, ks);
    for (int i = 0; i < 4; i++)
      for (int j = 0; j < 4; j++) S.pred[i][j] += (int64_t)ks.pred[i][j];
    S.rounds += ks.rounds;
    S.large_cavities += ks.giant_rounds;
    if (s != DT_OK) { S.fail = cx.hctr->flags; return s; }
  }
  // rows grouped by leaf
  dt_result cur;
  cur.D = D;
  {
    DevBuf cnt2, base, cursor;
    DT_TRY(cnt2.alloc((size_t)k * 4));
    DT_HIP(hipMemsetAsync(cnt2.p, 0, (size_t)k * 4, st));
    DT_TRY(k4_extract(job, pool, nullptr, cx.dflag.as<uint32_t>(), cnt2.as<uint32_t>(), st));
    std::vector<uint32_t> hc(k);
    DT_HIP(hipMemcpyAsync(hc.data(), cnt2.p, (size_t)k * 4, hipMemcpyDeviceToHost, st));
    DT_HIP(hipStreamSynchronize(st));
    cur.set_offsets.assign(k + 1, 0);
    for (int s = 0; s < k; s++) cur.set_offsets[s + 1] = cur.set_offsets[s] + hc[s];
    cur.m = cur.set_offsets[k];
    S.local_simplices = cur.m;
    DT_TRY(cur.rows.alloc_plain((size_t)(cur.m ? cur.m : 1) * (D + 1) * 4));
    DT_TRY(extract_grouped(job, pool, cur.set_offsets, cur.rows.as<int32_t>(), st));
  }
  pool = CellPool();
  leafjob_pts.release();
  leafjob_set.release();
  leafjob_off.release();
  double t3 = now_ms();
  S.stage_ms[DT_STAGE_LOCAL_DT] = t3 - t2;

  // ---- merges, bottom-up
  double cells = (double)n;
  for (int a = 0; a < D; a++) cells /= o.grid_cell;
  uint64_t gtotal = 1;
  const BGrid G = make_bgrid(lo, hi, D, cells, &gtotal);
  double tb_total = 0.0, tdt_total = 0.0;
  for (int l = levels - 1; l >= 0; l--) {
    const uint32_t nchild = 1u << (l + 1), npar = 1u << l;
    const int cshift = levels - (l + 1);   // leaf >> cshift = child at this level
    const uint32_t m = (uint32_t)cur.m;
    double ta = now_ms();
    // neighbours inside each child (hull facets)
    DevBuf nbr;
    DT_TRY(compute_neighbors(cur, nbr, st));
    DevBuf off32, tag, owner, flag, vbflag, nb;
    std::vector<uint32_t> ho(nchild + 1);
    for (uint32_t s = 0; s <= nchild; s++) ho[s] = (uint32_t)cur.set_offsets[s];
    DT_TRY(off32.alloc((size_t)(nchild + 1) * 4));
    DT_HIP(hipMemcpyAsync(off32.p, ho.data(), (size_t)(nchild + 1) * 4, hipMemcpyHostToDevice, st));
    DT_TRY(tag.alloc((size_t)(m ? m : 1) * 4));
    hipLaunchKernelGGL(k_rb_row_tags, dim3(rblocks(m)), dim3(RB), 0, st, off32.as<uint32_t>(),
                       nchild, m, tag.as<uint32_t>());
    if (!region) {
      DT_TRY(owner.alloc(gtotal * 4));
      DT_HIP(hipMemsetAsync(owner.p, 0xFF, gtotal * 4, st));
      hipLaunchKernelGGL(k_rb_occupancy, dim3(rblocks(n)), dim3(RB), 0, st, P.as<double4>(), n,
                         leaf.as<uint32_t>(), cshift, G, owner.as<uint32_t>());
    }
    DT_TRY(flag.alloc((size_t)(m ? m : 1)));
    DT_TRY(vbflag.alloc((size_t)n * 4));
    DT_TRY(nb.alloc(8));
    DT_HIP(hipMemsetAsync(vbflag.p, 0, (size_t)n * 4, st));
    DT_HIP(hipMemsetAsync(nb.p, 0, 8, st));
    DevBuf cbox;
    Region R;
    if (region && divide == DT_DIVIDE_KD) {
      // the box of every child: the union of its leaves' boxes
      std::vector<double> cb((size_t)nchild * 6);
      for (uint32_t c = 0; c < nchild; c++) {
        double* b = cb.data() + (size_t)c * 6;
        for (int a = 0; a < 3; a++) {
          b[a] = INFINITY;
          b[3 + a] = -INFINITY;
        }
        for (uint32_t f = c << cshift; f < (c + 1) << cshift; f++)
          for (int a = 0; a < 3; a++) {
            b[a] = std::min(b[a], hbox[(size_t)f * 6 + a]);
            b[3 + a] = std::max(b[3 + a], hbox[(size_t)f * 6 + 3 + a]);
          }
      }
      DT_TRY(cbox.alloc(cb.size() * 8));
      DT_HIP(hipMemcpyAsync(cbox.p, cb.data(), cb.size() * 8, hipMemcpyHostToDevice, st));
    } else if (region) {
      R.kind = BORDER_VORONOI;
      R.S = lv[l].pts.as<double4>();
      R.part = lv[l].label.as<uint32_t>();
      R.goff = lv[l].goff.as<uint32_t>();
      R.gadj = lv[l].gadj.as<uint32_t>();
    }
    DT_PROF_BEGIN(DT_KERN_BORDER, st);
    if (region) {
      const uint32_t* near = divide == DT_DIVIDE_KD ? nullptr : lv[l].nearest.as<uint32_t>();
      const double* cbp = divide == DT_DIVIDE_KD ? cbox.as<double>() : nullptr;
      if (D == 2)
        hipLaunchKernelGGL(k_rb_border_region<2>, dim3(rblocks(m)), dim3(RB), 0, st,
                           P.as<double4>(), cur.rows.as<int32_t>(), m, tag.as<uint32_t>(),
                           nbr.as<int32_t>(), R, near, cbp, flag.as<uint8_t>(),
                           vbflag.as<uint32_t>(), nb.as<unsigned long long>());
      else
        hipLaunchKernelGGL(k_rb_border_region<3>, dim3(rblocks(m)), dim3(RB), 0, st,
                           P.as<double4>(), cur.rows.as<int32_t>(), m, tag.as<uint32_t>(),
                           nbr.as<int32_t>(), R, near, cbp, flag.as<uint8_t>(),
                           vbflag.as<uint32_t>(), nb.as<unsigned long long>());
    } else if (D == 2) {
      hipLaunchKernelGGL(k_rb_border<2>, dim3(rblocks(m)), dim3(RB), 0, st, P.as<double4>(),
                         cur.rows.as<int32_t>(), m, tag.as<uint32_t>(), nbr.as<int32_t>(), G,
                         owner.as<uint32_t>(), flag.as<uint8_t>(), vbflag.as<uint32_t>(),
                         nb.as<unsigned long long>());
    } else {
      hipLaunchKernelGGL(k_rb_border<3>, dim3(rblocks(m)), dim3(RB), 0, st, P.as<double4>(),
                         cur.rows.as<int32_t>(), m, tag.as<uint32_t>(), nbr.as<int32_t>(), G,
                         owner.as<uint32_t>(), flag.as<uint8_t>(), vbflag.as<uint32_t>(),
                         nb.as<unsigned long long>());
    }
    DT_PROF_END(st);
    DT_HIP(hipGetLastError());
    unsigned long long hnb = 0;
    DT_HIP(hipMemcpyAsync(&hnb, nb.p, 8, hipMemcpyDeviceToHost, st));
    DevBuf vb;
    uint32_t nvb = 0;
    DT_TRY(compact_indices(vbflag.as<uint32_t>(), n, vb, &nvb, st));
    S.border_simplices += (int64_t)hnb;
    S.border_vertices += nvb;
    owner.release();
    nbr.release();
    // border vertices grouped by parent
    DevBuf pk, pv, pset_sorted;
    DT_TRY(pk.alloc((size_t)(nvb ? nvb : 1) * 8));
    DT_TRY(pv.alloc((size_t)(nvb ? nvb : 1) * 4));
    hipLaunchKernelGGL(k_rb_parent_keys, dim3(rblocks(nvb)), dim3(RB), 0, st, vb.as<uint32_t>(),
                       nvb, leaf.as<uint32_t>(), cshift + 1, pk.as<unsigned long long>(),
                       pv.as<uint32_t>());
    DT_TRY(radix_sort_pairs(pk.as<unsigned long long>(), pv.as<uint32_t>(), nvb,
                            l == 0 ? 1 : l, st));
    DT_TRY(pset_sorted.alloc((size_t)(nvb ? nvb : 1) * 4));
    hipLaunchKernelGGL(k_rb_key_lo, dim3(rblocks(nvb)), dim3(RB), 0, st,
                       pk.as<unsigned long long>(), nvb, pset_sorted.as<uint32_t>());
    double tb = now_ms();
    tb_total += tb - ta;
    // border triangulations of all parents in one batched run
    DevBuf bpts, bset, boff;
    LocalJob bjob;
    CellPool bpool;
    DT_TRY(make_job(P, pv.as<uint32_t>(), nvb, pset_sorted.as<uint32_t>(), npar, D, lo, hi, fp32,
                    o, bpts, bset, boff, bjob, st));
    if (nvb) {
      K4Stats ks;
      int s = k4_run(bjob, bpool, cx.dc(), cx.hctr, st, ks);
      for (int i = 0; i < 4; i++)
        for (int j = 0; j < 4; j++) S.pred[i][j] += (int64_t)ks.pred[i][j];
      S.rounds += ks.rounds;
      S.large_cavities += ks.giant_rounds;
      if (s != DT_OK) { S.fail = cx.hctr->flags; return s; }
    }
    double tc = now_ms();
    tdt_total += tc - tb;
    // merge: kept rows of the children and of the border triangulations
    uint32_t tsize = 64;
    while (tsize < 2 * hnb + 16) tsize <<= 1;
    DevBuf occ, tkeys, fail, pcnt, pbase, pcur;
    DT_TRY(occ.alloc((size_t)tsize * 4));
    DT_TRY(tkeys.alloc((size_t)tsize * 16));
    DT_TRY(fail.alloc(4));
    DT_TRY(pcnt.alloc((size_t)(npar + 1) * 4));
    DT_TRY(pbase.alloc((size_t)(npar + 1) * 4));
    DT_TRY(pcur.alloc((size_t)(npar + 1) * 4));
    DT_HIP(hipMemsetAsync(occ.p, 0, (size_t)tsize * 4, st));
    DT_HIP(hipMemsetAsync(fail.p, 0, 4, st));
    DT_HIP(hipMemsetAsync(pcnt.p, 0, (size_t)(npar + 1) * 4, st));
    DT_PROF_BEGIN(DT_KERN_MERGE, st);
    if (D == 2) {
      hipLaunchKernelGGL(k_rb_table<2>, dim3(rblocks(m)), dim3(RB), 0, st, cur.rows.as<int32_t>(),
                         m, flag.as<uint8_t>(), occ.as<uint32_t>(), tkeys.as<uint4>(), tsize - 1,
                         fail.as<uint32_t>());
      hipLaunchKernelGGL(k_rb_keep_local<2>, dim3(rblocks(m)), dim3(RB), 0, st,
                         cur.rows.as<int32_t>(), m, tag.as<uint32_t>(), flag.as<uint8_t>(),
                         nullptr, pcnt.as<uint32_t>(), nullptr);
      if (bpool.ncells)
        hipLaunchKernelGGL(k_rb_keep_border<2>, dim3(rblocks(bpool.ncells)), dim3(RB), 0, st,
                           bjob.pts, bjob.pset, bpool.cells.as<Cell>(), bpool.ncells,
                           leaf.as<uint32_t>(), cshift, occ.as<uint32_t>(), tkeys.as<uint4>(),
                           tsize - 1, nullptr, pcnt.as<uint32_t>(), nullptr);
    } else {
      hipLaunchKernelGGL(k_rb_table<3>, dim3(rblocks(m)), dim3(RB), 0, st, cur.rows.as<int32_t>(),
                         m, flag.as<uint8_t>(), occ.as<uint32_t>(), tkeys.as<uint4>(), tsize - 1,
                         fail.as<uint32_t>());
      hipLaunchKernelGGL(k_rb_keep_local<3>, dim3(rblocks(m)), dim3(RB), 0, st,
                         cur.rows.as<int32_t>(), m, tag.as<uint32_t>(), flag.as<uint8_t>(),
                         nullptr, pcnt.as<uint32_t>(), nullptr);
      if (bpool.ncells)
        hipLaunchKernelGGL(k_rb_keep_border<3>, dim3(rblocks(bpool.ncells)), dim3(RB), 0, st,
                           bjob.pts, bjob.pset, bpool.cells.as<Cell>(), bpool.ncells,
                           leaf.as<uint32_t>(), cshift, occ.as<uint32_t>(), tkeys.as<uint4>(),
                           tsize - 1, nullptr, pcnt.as<uint32_t>(), nullptr);
    }
    DT_HIP(hipGetLastError());
    std::vector<uint32_t> hpc(npar);
    DT_HIP(hipMemcpyAsync(hpc.data(), pcnt.p, (size_t)npar * 4, hipMemcpyDeviceToHost, st));
    uint32_t hfail = 0;
    DT_HIP(hipMemcpyAsync(&hfail, fail.p, 4, hipMemcpyDeviceToHost, st));
    DT_HIP(hipStreamSynchronize(st));
    if (hfail) return DT_E_INTERNAL;
    dt_result nxt;
    nxt.D = D;
    nxt.set_offsets.assign(npar + 1, 0);
    std::vector<uint32_t> hbase(npar);
    for (uint32_t s = 0; s < npar; s++) {
      hbase[s] = (uint32_t)nxt.set_offsets[s];
      nxt.set_offsets[s + 1] = nxt.set_offsets[s] + hpc[s];
    }
    nxt.m = nxt.set_offsets[npar];
    DT_TRY(nxt.rows.alloc_plain((size_t)(nxt.m ? nxt.m : 1) * (D + 1) * 4));
    DT_HIP(hipMemcpyAsync(pbase.p, hbase.data(), (size_t)npar * 4, hipMemcpyHostToDevice, st));
    DT_HIP(hipMemsetAsync(pcur.p, 0, (size_t)(npar + 1) * 4, st));
    if (D == 2) {
      hipLaunchKernelGGL(k_rb_keep_local<2>, dim3(rblocks(m)), dim3(RB), 0, st,
                         cur.rows.as<int32_t>(), m, tag.as<uint32_t>(), flag.as<uint8_t>(),
                         pbase.as<uint32_t>(), pcur.as<uint32_t>(), nxt.rows.as<int32_t>());
      if (bpool.ncells)
        hipLaunchKernelGGL(k_rb_keep_border<2>, dim3(rblocks(bpool.ncells)), dim3(RB), 0, st,
                           bjob.pts, bjob.pset, bpool.cells.as<Cell>(), bpool.ncells,
                           leaf.as<uint32_t>(), cshift, occ.as<uint32_t>(), tkeys.as<uint4>(),
                           tsize - 1, pbase.as<uint32_t>(), pcur.as<uint32_t>(),
                           nxt.rows.as<int32_t>());
    } else {
      hipLaunchKernelGGL(k_rb_keep_local<3>, dim3(rblocks(m)), dim3(RB), 0, st,
                         cur.rows.as<int32_t>(), m, tag.as<uint32_t>(), flag.as<uint8_t>(),
                         pbase.as<uint32_t>(), pcur.as<uint32_t>(), nxt.rows.as<int32_t>());
      if (bpool.ncells)
        hipLaunchKernelGGL(k_rb_keep_border<3>, dim3(rblocks(bpool.ncells)), dim3(RB), 0, st,
                           bjob.pts, bjob.pset, bpool.cells.as<Cell>(), bpool.ncells,
                           leaf.as<uint32_t>(), cshift, occ.as<uint32_t>(), tkeys.as<uint4>(),
                           tsize - 1, pbase.as<uint32_t>(), pcur.as<uint32_t>(),
                           nxt.rows.as<int32_t>());
    }
    DT_PROF_END(st);
    DT_HIP(hipGetLastError());
    DT_HIP(hipStreamSynchronize(st));
    cur.rows = std::move(nxt.rows);
    cur.m = nxt.m;
    cur.set_offsets = nxt.set_offsets;
    cur.nbr_ready = false;
  }
  S.stage_ms[DT_STAGE_BORDER] = tb_total;
  S.stage_ms[DT_STAGE_BORDER_DT] = tdt_total;
  double t4 = now_ms();
  S.stage_ms[DT_STAGE_MERGE] = t4 - t3 - tb_total - tdt_total;
  if (o.keep_stages) {
    r->stage[DT_ARR_PID].resize((size_t)n * 4);
    DT_HIP(hipMemcpyAsync(r->stage[DT_ARR_PID].data(), leaf.p, (size_t)n * 4,
                          hipMemcpyDeviceToHost, st));
    DT_HIP(hipStreamSynchronize(st));
  }
  r->rows = std::move(cur.rows);
  r->m = cur.m;
  r->set_offsets = {0, r->m};
  S.num_simplices = r->m;
  S.stage_ms[DT_STAGE_TOTAL] = now_ms() - t0;
  S.o_dt = ((double)n + S.eta + S.border_vertices) / (double)n;
  return DT_OK;
}

}  // namespace dtk
