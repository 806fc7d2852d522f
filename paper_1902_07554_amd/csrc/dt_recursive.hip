// Recursive bisection (Section "Recursive Bisection"): log2 k levels of
// 2-way division, then k-1 merges bottom-up.  This is the scheme of the
// original divide-and-conquer triangulation (cyclic median split) and its
// sample-based variant (a new sample per level); the one-shot k-way
// division of Algorithm 1 is in dt_dc.hip.
//
// Division: every level splits every block in two; the leaf index of a
// point spells its path from the root (bit 1 = upper half), so its block
// at the level with 2^l blocks is leaf >> (log2 k - l).
//   kd:     the cyclic median split (kd_divide);
//   sample: in every block, the eta(|block|) points of smallest random key
//           form the block's sample; the sample is split at its median
//           along its widest axis (the graph partitioner's initial cut for
//           two parts), and every point of the block takes the side of its
//           nearest sample of the block, under the key (fl(d^2), id).
// Merging (level by level, all parents of a level in one batched run):
// the triangulations of the two children of a parent are known as simplex
// lists; a simplex is a border simplex when its ball may reach a grid cell
// holding points of the sibling (the grid test), the hull facets of each
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
                            const uint8_t* sside, const uint32_t* start, const uint32_t* items,
                            Grid G, uint32_t* pid) {
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
  pid[i] = 2 * me + (bests == 0xFFFFFFFFu ? 0u : (uint32_t)sside[bests]);
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

// leaf index of every point by sample bisection
int sample_bisect(const DevBuf& P, uint32_t n, int D, int levels, double rate, uint64_t seed,
                  const double lo[3], const double hi[3], DevBuf& pid, hipStream_t st) {
  DT_TRY(pid.alloc((size_t)n * 4));
  DT_HIP(hipMemsetAsync(pid.p, 0, (size_t)n * 4, st));
  DevBuf keys, vals, cnt;
  DT_TRY(keys.alloc((size_t)n * 8));
  DT_TRY(vals.alloc((size_t)n * 4));
  std::vector<double4> hp;
  for (int l = 0; l < levels; l++) {
    const uint32_t nb = 1u << l;
    DT_TRY(cnt.alloc((size_t)nb * 4));
    DT_TRY(count_by(pid.as<uint32_t>(), n, nb, cnt.as<uint32_t>(), st));
    std::vector<uint32_t> hc(nb);
    DT_HIP(hipMemcpyAsync(hc.data(), cnt.p, (size_t)nb * 4, hipMemcpyDeviceToHost, st));
    hipLaunchKernelGGL(k_rb_sample_keys, dim3(rblocks(n)), dim3(RB), 0, st, n,
                       pid.as<uint32_t>(), seed ^ (0xD1B54A32D192ED03ull * (uint64_t)(l + 1)),
                       keys.as<unsigned long long>(), vals.as<uint32_t>());
    DT_TRY(radix_sort_pairs(keys.as<unsigned long long>(), vals.as<uint32_t>(), n, 40 + l, st));
    std::vector<uint32_t> order(n);
    DT_HIP(hipMemcpyAsync(order.data(), vals.p, (size_t)n * 4, hipMemcpyDeviceToHost, st));
    if (hp.empty()) {
      hp.resize(n);
      DT_HIP(hipMemcpyAsync(hp.data(), P.p, (size_t)n * sizeof(double4), hipMemcpyDeviceToHost,
                            st));
    }
    DT_HIP(hipStreamSynchronize(st));
    // samples of every block, split at the median of the widest axis
    std::vector<double4> S;
    std::vector<uint32_t> sblock;
    std::vector<uint8_t> sside;
    uint32_t seg = 0;
    for (uint32_t b = 0; b < nb; b++) {
      const uint32_t m = hc[b];
      const uint32_t eta = m ? rb_sample_size(m, rate, D) : 0;
      std::vector<uint32_t> smp(order.begin() + seg, order.begin() + seg + eta);
      seg += m;
      if (eta == 0) continue;
      double blo[3] = {INFINITY, INFINITY, INFINITY}, bhi[3] = {-INFINITY, -INFINITY, -INFINITY};
      for (uint32_t s : smp) {
        const double c[3] = {hp[s].x, hp[s].y, hp[s].z};
        for (int a = 0; a < 3; a++) {
          blo[a] = std::min(blo[a], c[a]);
          bhi[a] = std::max(bhi[a], c[a]);
        }
      }
      int ax = 0;
      for (int a = 1; a < D; a++)
        if (bhi[a] - blo[a] > bhi[ax] - blo[ax]) ax = a;
      auto coord = [&](uint32_t s) { return ax == 0 ? hp[s].x : (ax == 1 ? hp[s].y : hp[s].z); };
      std::sort(smp.begin(), smp.end(), [&](uint32_t a2, uint32_t b2) {
        const double ca = coord(a2), cb = coord(b2);
        return ca < cb || (ca == cb && a2 < b2);
      });
      for (uint32_t j = 0; j < eta; j++) {
        S.push_back(hp[smp[j]]);
        sblock.push_back(b);
        sside.push_back(j < eta / 2 ? 0 : 1);
      }
    }
    const uint32_t ns = (uint32_t)S.size();
    DevBuf dS, dsb, dss, gcnt, gstart, gcur, gitems, gcell;
    DT_TRY(dS.alloc((size_t)ns * sizeof(double4)));
    DT_TRY(dsb.alloc((size_t)ns * 4));
    DT_TRY(dss.alloc((size_t)ns));
    DT_HIP(hipMemcpyAsync(dS.p, S.data(), (size_t)ns * sizeof(double4), hipMemcpyHostToDevice, st));
    DT_HIP(hipMemcpyAsync(dsb.p, sblock.data(), (size_t)ns * 4, hipMemcpyHostToDevice, st));
    DT_HIP(hipMemcpyAsync(dss.p, sside.data(), (size_t)ns, hipMemcpyHostToDevice, st));
    // grid of about ns/2 cells over the input box
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
    DT_TRY(gcnt.alloc((size_t)(ncell + 1) * 4));
    DT_TRY(gstart.alloc((size_t)(ncell + 1) * 4));
    DT_TRY(gcur.alloc((size_t)ncell * 4));
    DT_TRY(gitems.alloc((size_t)ns * 4));
    DT_TRY(gcell.alloc((size_t)ns * 4));
    DT_HIP(hipMemsetAsync(gcnt.p, 0, (size_t)(ncell + 1) * 4, st));
    DT_HIP(hipMemsetAsync(gcur.p, 0, (size_t)ncell * 4, st));
    hipLaunchKernelGGL(k_rb_grid_count, dim3(rblocks(ns)), dim3(RB), 0, st, dS.as<double4>(), ns, G,
                       gcnt.as<uint32_t>(), gcell.as<uint32_t>());
    DT_TRY(exclusive_scan(gcnt.as<uint32_t>(), gstart.as<uint32_t>(), ncell + 1, st));
    hipLaunchKernelGGL(k_rb_grid_fill, dim3(rblocks(ns)), dim3(RB), 0, st, ns,
                       gcell.as<uint32_t>(), gstart.as<uint32_t>(), gcur.as<uint32_t>(),
                       gitems.as<uint32_t>());
    hipLaunchKernelGGL(k_rb_assign, dim3(rblocks(n)), dim3(RB), 0, st, P.as<double4>(), n,
                       dS.as<double4>(), dsb.as<uint32_t>(), dss.as<uint8_t>(),
                       gstart.as<uint32_t>(), gitems.as<uint32_t>(), G, pid.as<uint32_t>());
    DT_HIP(hipGetLastError());
    DT_HIP(hipStreamSynchronize(st));
  }
  return DT_OK;
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
  if (divide == DT_DIVIDE_KD) {
    DT_TRY(kd_divide(P.as<double4>(), n, D, (uint32_t)k, leaf, boxes, st));
  } else {
    DT_TRY(sample_bisect(P, n, D, levels, rate, o.seed, lo, hi, leaf, st));
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
    DT_TRY(owner.alloc(gtotal * 4));
    DT_HIP(hipMemsetAsync(owner.p, 0xFF, gtotal * 4, st));
    hipLaunchKernelGGL(k_rb_occupancy, dim3(rblocks(n)), dim3(RB), 0, st, P.as<double4>(), n,
                       leaf.as<uint32_t>(), cshift, G, owner.as<uint32_t>());
    DT_TRY(flag.alloc((size_t)(m ? m : 1)));
    DT_TRY(vbflag.alloc((size_t)n * 4));
    DT_TRY(nb.alloc(8));
    DT_HIP(hipMemsetAsync(vbflag.p, 0, (size_t)n * 4, st));
    DT_HIP(hipMemsetAsync(nb.p, 0, 8, st));
    DT_PROF_BEGIN(DT_KERN_BORDER, st);
    if (D == 2)
      hipLaunchKernelGGL(k_rb_border<2>, dim3(rblocks(m)), dim3(RB), 0, st, P.as<double4>(),
                         cur.rows.as<int32_t>(), m, tag.as<uint32_t>(), nbr.as<int32_t>(), G,
                         owner.as<uint32_t>(), flag.as<uint8_t>(), vbflag.as<uint32_t>(),
                         nb.as<unsigned long long>());
    else
      hipLaunchKernelGGL(k_rb_border<3>, dim3(rblocks(m)), dim3(RB), 0, st, P.as<double4>(),
                         cur.rows.as<int32_t>(), m, tag.as<uint32_t>(), nbr.as<int32_t>(), G,
                         owner.as<uint32_t>(), flag.as<uint8_t>(), vbflag.as<uint32_t>(),
                         nb.as<unsigned long long>());
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
  r->rows = std::move(cur.rows);
  r->m = cur.m;
  r->set_offsets = {0, r->m};
  S.num_simplices = r->m;
  S.stage_ms[DT_STAGE_TOTAL] = now_ms() - t0;
  S.o_dt = ((double)n + S.border_vertices) / (double)n;
  return DT_OK;
}

}  // namespace dtk
