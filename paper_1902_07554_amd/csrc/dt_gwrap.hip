// Delaunay triangulation of small point sets by gift wrapping: the sample
// triangulation of Algorithm 2 (eta(n) = sqrt(n) points by default, Section
// "Sample Size"), and the seeds of the parallel insertion (the first points
// of every large set, see dt_k4.hip).  Several independent sets are wrapped
// together: each facet searches only the points of its own set, and the
// levels of all sets run in the same launches.
//
// Parallel insertion spends about a hundred rounds on the start-up of a
// small single set (while the triangulation has few cells, the cavities of
// the candidates overlap and one or two points are inserted per round), and
// every round is a chain of dependent gathers.  Gift wrapping inserts
// nothing: from one Delaunay simplex, each facet finds the simplex on its
// other side directly, and the facets of the simplices found are searched
// in the next level.  The simplex beyond an oriented facet f is (f, p) for
// the point p strictly beyond f whose sphere through f holds no other such
// point: of two candidates p and q, q comes first when it lies inside the
// sphere through f and p (spheres through f form a pencil, and the
// in-sphere test orders the candidates along it).  Because f is a facet of
// a Delaunay simplex on its near side, the balls of the pencil beyond that
// simplex's ball hold no point on the near side either, so (f, p) is
// Delaunay.  A facet with no point strictly beyond it lies on the hull.
// Points on f's own hyperplane can never complete it (the simplex would be
// flat).
//
// Exactness: orientation and the perturbed in-sphere test are the
// library's predicates (FP64 filter, then exact), so the simplices
// found are the finite cells of the same perturbed Delaunay triangulation
// that parallel insertion builds.  The seed of a set is a simplex through
// its first point and D of that point's 16 nearest whose circumsphere holds
// no point of the set, checked against every one.  When some set has no
// such simplex among them, or a capacity runs out, the caller triangulates
// the sets by parallel insertion instead.
//
// The FP64 filter comes first here whatever the run's precision: the
// tests that decide a facet compare nearly cospherical candidates, where the
// FP32 filter often cannot decide and the out-of-line stages would run.
//
// Cost: one wavefront per facet search.  A small single set is copied into
// every block's LDS and each search reads all of it; larger sets, and every
// set of a multi-set wrap, are searched through a uniform grid of their
// points (the cells around the facet for a first candidate, then the cells
// under the ball through the facet and that candidate).  A search is then
// a chain of dependent loads and FP64 predicates of some tens of
// microseconds.  A level is one launch; the number of levels is the depth
// of the simplices' adjacency graph from the seed (tens for a few thousand
// points).
#include "dt_common.hpp"
#include "dt_geom.hpp"
#include "dt_internal.hpp"
#include "dt_pred.hpp"
#include "dt_gwrap.hpp"
#include "dt_prims.hpp"

#include <stdio.h>
#include <stdlib.h>

#include <vector>

namespace dtk {

namespace {

constexpr uint32_t GW_NN = 16;              // nearest points tried for the seed
constexpr uint32_t GW_BASES = 4;            // start points tried per set for the seed
constexpr uint32_t GW_NONE = 0xFFFFFFFFu;
constexpr uint32_t GW_MAX_LEVELS = 4096;
constexpr uint32_t GW_THREADS = 256;        // level kernel: four facets per block
constexpr uint32_t GW_LEVEL_BLOCKS = 1024;  // grid of the level kernel (a grid-stride loop)
constexpr uint32_t GW_GROUP = 8;            // levels launched between two reads of the counters
constexpr uint32_t GW_CHUNK = 64;           // facets per block between two allocations (at most)
constexpr uint32_t GW_LDS_POINTS = 2048;    // a single set this small is copied into LDS (64 KB)
constexpr int GW_LOCAL_BITS = 13;           // set-local point index in simplex keys (8192 points)

// device failure bits of the wrap (any: the caller falls back)
enum : uint32_t { GW_FAIL_SEED = 1u, GW_FAIL_CAP = 2u, GW_FAIL_HASH = 4u };

__device__ __forceinline__ uint32_t vget(const uint4& v, int i) {
  return i == 0 ? v.x : (i == 1 ? v.y : (i == 2 ? v.z : v.w));
}
__device__ __forceinline__ void vput(uint4& v, int i, uint32_t x) {
  if (i == 0) v.x = x;
  else if (i == 1) v.y = x;
  else if (i == 2) v.z = x;
  else v.w = x;
}

__device__ __forceinline__ void gw_load(const double4* P, uint32_t i, double* p,
                                        unsigned long long& key) {
  const double4 t = P[i];
  p[0] = t.x;
  p[1] = t.y;
  p[2] = t.z;
  key = (unsigned long long)__double_as_longlong(t.w);
}

// Point (p, key) into slot i of X, i known only at run time: an unrolled
// select, so that X stays in registers.
template <int D>
__device__ __forceinline__ void put_slot(PtsX& X, uint32_t i, const double* p,
                                         unsigned long long key) {
#pragma unroll
  for (int k = 0; k <= D; k++)
    if ((uint32_t)k == i) {
      X.p[k][0] = p[0];
      X.p[k][1] = p[1];
      X.p[k][2] = p[2];
      X.key[k] = key;
    }
}

// The facet's circumcentre cf and squared circumradius r2 (in the facet's
// hyperplane) and a normal nrm pointing away from the point v on its near
// side, in FP64.  A sphere through the facet has its centre at cf + s nrm;
// a point x beyond the facet lies on the one with
//   s(x) = (|x - cf|^2 - r2) / (2 (x - cf) . nrm),
// so ordering the points beyond the facet by s(x) orders them along the
// pencil.  Used only to guess a good first candidate.  False when the
// facet is too flat to say.
template <int D>
__device__ __forceinline__ bool facet_frame(const PtsX& F, uint32_t i, const double4& v,
                                            double cf[3], double* r2, double nrm[3]) {
  // the facet's points in slot order (selects, so that they stay in
  // registers)
  double a[3], b[3], c[3];
#pragma unroll
  for (int x = 0; x < 3; x++) {
    const int ka = i == 0 ? 1 : 0;
    const int kb = i <= 1 ? 2 : 1;
    const int kc = i <= 2 ? 3 : 2;
    a[x] = ka == 0 ? F.p[0][x] : F.p[1][x];
    b[x] = kb == 1 ? F.p[1][x] : F.p[2][x];
    c[x] = D == 3 ? (kc == 2 ? F.p[2][x] : F.p[3][x]) : 0.0;
  }
  if (D == 2) {
    const double ex = b[0] - a[0], ey = b[1] - a[1];
    cf[0] = 0.5 * (a[0] + b[0]);
    cf[1] = 0.5 * (a[1] + b[1]);
    cf[2] = 0.0;
    *r2 = 0.25 * (ex * ex + ey * ey);
    nrm[0] = -ey;
    nrm[1] = ex;
    nrm[2] = 0.0;
  } else {
    const double e1[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
    const double e2[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
    const double nv[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                          e1[0] * e2[1] - e1[1] * e2[0]};
    const double l1 = e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2];
    const double l2 = e2[0] * e2[0] + e2[1] * e2[1] + e2[2] * e2[2];
    const double nn = nv[0] * nv[0] + nv[1] * nv[1] + nv[2] * nv[2];
    if (!(nn > 1e-20 * l1 * l2)) return false;
    const double u[3] = {l1 * e2[0] - l2 * e1[0], l1 * e2[1] - l2 * e1[1],
                         l1 * e2[2] - l2 * e1[2]};
    const double inv = 0.5 / nn;
    const double o[3] = {(u[1] * nv[2] - u[2] * nv[1]) * inv, (u[2] * nv[0] - u[0] * nv[2]) * inv,
                         (u[0] * nv[1] - u[1] * nv[0]) * inv};
    cf[0] = a[0] + o[0];
    cf[1] = a[1] + o[1];
    cf[2] = a[2] + o[2];
    *r2 = o[0] * o[0] + o[1] * o[1] + o[2] * o[2];
    nrm[0] = nv[0];
    nrm[1] = nv[1];
    nrm[2] = nv[2];
  }
  const double side = (v.x - cf[0]) * nrm[0] + (v.y - cf[1]) * nrm[1] +
                      (D == 3 ? (v.z - cf[2]) * nrm[2] : 0.0);
  if (side == 0.0) return false;
  if (side > 0.0) {
    nrm[0] = -nrm[0];
    nrm[1] = -nrm[1];
    nrm[2] = -nrm[2];
  }
  return true;
}

// The simplex's set and its sorted set-local vertex indices (13 bits each)
// packed into one key.
template <int D>
__device__ __forceinline__ unsigned long long simplex_key(const uint4& v, uint32_t set,
                                                          uint32_t base, int bits) {
  uint32_t k[4] = {v.x - base, v.y - base, v.z - base, D == 3 ? v.w - base : 0u};
#pragma unroll
  for (int i = 1; i <= D; i++)
#pragma unroll
    for (int j = i; j > 0; j--)
      if (k[j] < k[j - 1]) {
        const uint32_t t = k[j];
        k[j] = k[j - 1];
        k[j - 1] = t;
      }
  unsigned long long key = (unsigned long long)set;
#pragma unroll
  for (int i = 0; i <= D; i++) key = (key << bits) | (unsigned long long)k[i];
  return key;
}

__device__ __forceinline__ uint32_t key_hash(unsigned long long k) {
  k *= 0x9E3779B97F4A7C15ull;
  return (uint32_t)(k >> 32) ^ (uint32_t)k;
}

// Sign of the orientation of the simplex v (D+1 vertex indices).
template <int D>
__device__ __forceinline__ int simplex_orient(const double4* P, PredT<false>& pr, const uint4& v) {
  PtsX X;
#pragma unroll
  for (int i = 0; i <= D; i++) gw_load(P, vget(v, i), X.p[i], X.key[i]);
  return pr.template orient<D>(X);
}

// Is point q strictly inside the circumsphere of the positively oriented
// simplex v (perturbed)?
template <int D>
__device__ __forceinline__ bool in_sphere(const double4* P, PredT<false>& pr, const uint4& v,
                                          uint32_t q) {
  PtsX X;
#pragma unroll
  for (int i = 0; i <= D; i++) gw_load(P, vget(v, i), X.p[i], X.key[i]);
  gw_load(P, q, X.p[D + 1], X.key[D + 1]);
  return pr.template insphere<D>(X) > 0;
}

// Start point b of a set (b < GW_BASES): spread over the set's points.
__device__ __forceinline__ uint32_t gw_base(uint32_t lo, uint32_t hi, uint32_t b) {
  return lo + b * ((hi - lo) / GW_BASES);
}

// GW_NN points near each start point of each set, one block per (set,
// start): the nearest point of each thread's share (by squared distance
// rounded to FP32, then index), and of those the GW_NN smallest by rank.
// Any near points do: they only propose seeds, each checked exactly.  The
// list of (set s, start b) is nn[(s * GW_BASES + b) * (GW_NN + 1) ...], its
// length last.
__global__ void k_gw_nearest(const double4* P, const uint32_t* soff, uint32_t* nn_all) {
  __shared__ unsigned long long s_key[GW_THREADS];
  const uint32_t set = blockIdx.x / GW_BASES, lo = soff[set], hi = soff[set + 1];
  const uint32_t ob = gw_base(lo, hi, blockIdx.x % GW_BASES);
  uint32_t* nn = nn_all + (size_t)blockIdx.x * (GW_NN + 1);
  if (hi - lo < 2) {
    if (threadIdx.x == 0) nn[GW_NN] = 0;
    return;
  }
  const double4 o = P[ob];
  unsigned long long best = ~0ull;
  for (uint32_t j = lo + threadIdx.x; j < hi; j += GW_THREADS) {
    if (j == ob) continue;
    const double4 q = P[j];
    const double dx = q.x - o.x, dy = q.y - o.y, dz = q.z - o.z;
    const float d2 = (float)(dx * dx + dy * dy + dz * dz);
    const unsigned long long k = ((unsigned long long)__float_as_uint(d2) << 32) | j;
    best = k < best ? k : best;
  }
  s_key[threadIdx.x] = best;
  __syncthreads();
  uint32_t rank = 0, real = 0;
  for (uint32_t t = 0; t < GW_THREADS; t++) {
    const unsigned long long x = s_key[t];
    rank += x < best ? 1u : 0u;
    real += x != ~0ull ? 1u : 0u;
  }
  if (best != ~0ull && rank < GW_NN) nn[rank] = (uint32_t)(best & 0xFFFFFFFFull);
  if (threadIdx.x == 0) nn[GW_NN] = real < GW_NN ? real : GW_NN;
}

// Candidate seed simplex c: the set's first point o and D of the near
// points (combination number c in lexicographic order), positively
// oriented; false when flat.
template <int D>
__device__ bool seed_candidate(const double4* P, PredT<false>& pr, const uint32_t* nn,
                               uint32_t m, uint32_t c, uint32_t o, uint4& v) {
  uint32_t idx[3] = {0, 0, 0};
  uint32_t left = c;
  bool found = false;
  if (D == 2) {
    for (uint32_t a = 0; a < m && !found; a++)
      for (uint32_t b = a + 1; b < m && !found; b++) {
        if (left == 0) { idx[0] = a; idx[1] = b; found = true; }
        else left--;
      }
  } else {
    for (uint32_t a = 0; a < m && !found; a++)
      for (uint32_t b = a + 1; b < m && !found; b++)
        for (uint32_t e = b + 1; e < m && !found; e++) {
          if (left == 0) { idx[0] = a; idx[1] = b; idx[2] = e; found = true; }
          else left--;
        }
  }
  if (!found) return false;
  v = make_uint4(o, nn[idx[0]], nn[idx[1]], D == 3 ? nn[idx[2]] : NOSLOT);
  const int sg = simplex_orient<D>(P, pr, v);
  if (sg == 0) return false;
  if (sg < 0) {
    const uint32_t t = v.y;
    v.y = v.z;
    v.z = t;
  }
  return true;
}

// Seed candidates of a set with m near points.
template <int D>
__host__ __device__ __forceinline__ uint32_t seed_combos(uint32_t m) {
  return D == 2 ? m * (m - 1) / 2 : m * (m - 1) * (m - 2) / 6;
}

// One wavefront per candidate seed of each (set, start) for the starts
// b0 .. b0 + nb - 1 (ncomb each): is its circumsphere empty of every point
// of the set?  The smallest empty candidate's number is kept per (set,
// start).  Later starts are searched only for the sets where the first
// found nothing (a second launch; its other wavefronts return at once).
template <int D>
__global__ void k_gw_seed(const double4* P, const uint32_t* soff, uint32_t nsets,
                          const uint32_t* nn_all, uint32_t ncomb, uint32_t b0, uint32_t nb,
                          uint32_t* best_all, uint32_t* flags) {
  PredT<false> pr;
  pr.init(flags);
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t w = (blockIdx.x * blockDim.x + threadIdx.x) / 64;
  const uint32_t c = w % ncomb, set = w / ncomb / nb;
  if (set >= nsets) return;
  const uint32_t sb = set * GW_BASES + b0 + (w / ncomb) % nb;
  if (b0 > 0 && best_all[set * GW_BASES] != GW_NONE) return;
  const uint32_t* nn = nn_all + (size_t)sb * (GW_NN + 1);
  const uint32_t m = nn[GW_NN];
  if (m < (uint32_t)D || c >= seed_combos<D>(m)) return;
  const uint32_t lo = soff[set], hi = soff[set + 1];
  uint4 v;
  if (!seed_candidate<D>(P, pr, nn, m, c, gw_base(lo, hi, sb % GW_BASES), v)) return;
  // only points inside the conservatively enlarged circumball can be
  // strictly inside the sphere (a nearly flat candidate tests them all)
  double sc[3] = {0.0, 0.0, 0.0}, sr = 0.0;
  const bool ball = circumball<D>(P[v.x], P[v.y], P[v.z], P[D == 3 ? v.w : v.z], sc, &sr);
  const double sr2 = sr * sr;
  bool hit = false;
  for (uint32_t q = lo + lane; q < hi && !hit; q += 64) {
    if (ball) {
      const double4 t = P[q];
      const double dx = t.x - sc[0], dy = t.y - sc[1], dz = t.z - sc[2];
      if (dx * dx + dy * dy + dz * dz > sr2) continue;
    }
    bool vert = false;
#pragma unroll
    for (int i = 0; i <= D; i++) vert |= (vget(v, i) == q);
    if (!vert && in_sphere<D>(P, pr, v, q)) hit = true;
  }
  if (__ballot(hit) == 0ull && lane == 0) atomicMin(best_all + sb, c);
}

// The seed simplex of a set: the empty candidate of its first start point
// that has one.  False when none has.
template <int D>
__device__ bool gw_pick_seed(const double4* P, PredT<false>& pr, const uint32_t* soff,
                             uint32_t set, const uint32_t* nn_all, const uint32_t* best_all,
                             uint4& v) {
  const uint32_t lo = soff[set], hi = soff[set + 1];
  for (uint32_t b = 0; b < GW_BASES; b++) {
    const uint32_t sb = set * GW_BASES + b;
    const uint32_t* nn = nn_all + (size_t)sb * (GW_NN + 1);
    if (best_all[sb] != GW_NONE &&
        seed_candidate<D>(P, pr, nn, nn[GW_NN], best_all[sb], gw_base(lo, hi, b), v))
      return true;
  }
  return false;
}

// Uniform grid over each set's points, the points sorted by cell: for set
// s, meta[4s ..] = its lower corner and the inverse cell edge, dims[4s ..]
// = the cells per axis and the index of its first cell; cell c holds the
// points cstart[c] .. cstart[c+1].
struct GwGrid {
  const double* meta;
  const int* dims;
  const uint32_t* cstart;
};
// Hash set of the simplices found (keys only) and the cell list.
struct GwState {
  const double4* P;
  uint32_t n;
  const uint32_t* soff;   // set s: points soff[s] .. soff[s+1]
  const uint32_t* sof;    // set of every point
  Cell* cells;
  uint32_t cap;
  uint32_t* ncells;
  unsigned long long* table;
  uint32_t tmask;
  uint32_t* flags;
  int kbits;              // bits of a set-local index in the simplex keys
  GwGrid grid;            // used when has_grid
  bool has_grid;
};

// Claim simplex v (of set `set`) in the hash set: 1 when it is new, 0 when
// it is known, -1 when the table is full.
template <int D>
__device__ int gw_claim(const GwState& g, const uint4& v, uint32_t set) {
  const unsigned long long key = simplex_key<D>(v, set, g.soff[set], g.kbits);
  const uint32_t h = key_hash(key);
  for (uint32_t pr = 0; pr <= g.tmask; pr++) {
    const uint32_t s = (h + pr) & g.tmask;
    const unsigned long long old = atomicCAS(&g.table[s], ~0ull, key);
    if (old == key) return 0;
    if (old == ~0ull) return 1;
  }
  atomicOr(g.flags, (uint32_t)GW_FAIL_HASH);
  return -1;
}

__device__ __forceinline__ void gw_cell(Cell& x, const uint4& v) {
  x.v = v;
  x.n = make_uint4(0u, 0u, 0u, 0u);
  x.spare = 0;
  x.cav = NOKEY;
  x.shell = NOKEY;
  x.fwd = ALIVE;
  x.pos = 0;
}

// Record simplex v unless it is known; true when it is new (then *idx is
// its cell, taken from the one counter of the pool).
template <int D>
__device__ bool gw_record(const GwState& g, const uint4& v, uint32_t set, uint32_t* idx) {
  if (gw_claim<D>(g, v, set) != 1) return false;
  const uint32_t c = atomicAdd(g.ncells, 1u);
  if (c >= g.cap) {
    atomicOr(g.flags, (uint32_t)GW_FAIL_CAP);
    return false;
  }
  gw_cell(g.cells[c], v);
  *idx = c;
  return true;
}

// The seed simplex of every set (one thread per set) becomes a cell; its
// D+1 facets join the first level.  An empty set is skipped.
template <int D>
__global__ void k_gw_start(GwState g, uint32_t nsets, const uint32_t* nn_all,
                           const uint32_t* best_all, uint32_t* front, uint32_t* cnt,
                           uint32_t* first) {
  const uint32_t set = blockIdx.x * blockDim.x + threadIdx.x;
  if (set >= nsets || g.soff[set] == g.soff[set + 1]) return;
  PredT<false> pr;
  pr.init(g.flags);
  uint4 v;
  if (!gw_pick_seed<D>(g.P, pr, g.soff, set, nn_all, best_all, v)) {
    atomicOr(g.flags, (uint32_t)GW_FAIL_SEED);
    return;
  }
  uint32_t c = 0;
  if (!gw_record<D>(g, v, set, &c)) {
    atomicOr(g.flags, (uint32_t)GW_FAIL_SEED);
    return;
  }
  const uint32_t at = atomicAdd(cnt, (uint32_t)D + 1);
  for (uint32_t i = 0; i <= (uint32_t)D; i++) front[at + i] = (c << 2) | i;
  if (first) first[set] = c;
}

constexpr uint32_t GW_BALL_CELLS = 512;     // larger balls scan the whole set

// The conservative circumball of the facet's points (slots other than i of
// F) and the candidate c in slot i, from the coordinates in registers (the
// same values as the points' records, so the same ball).
template <int D>
__device__ __forceinline__ bool gw_ball(const PtsX& F, uint32_t i, const double* c, double sc[3],
                                        double* r) {
  double4 Q[D + 1];
#pragma unroll
  for (int k = 0; k <= D; k++)
    Q[k] = (uint32_t)k == i ? make_double4(c[0], c[1], c[2], 0.0)
                            : make_double4(F.p[k][0], F.p[k][1], F.p[k][2], 0.0);
  return circumball<D>(Q[0], Q[1], Q[2], Q[D], sc, r);
}

__device__ __forceinline__ int gw_coord(double x, double lo, double inv, int g) {
  const double f = (x - lo) * inv;
  if (!(f >= 0.0)) return 0;
  return f >= (double)g ? g - 1 : (int)f;
}

// The search of one facet by one wavefront: facet i of the simplex t (two
// of its vertices already swapped, so that (facet, x) is positively
// oriented exactly for x strictly beyond it) among the points lo .. hi of
// set `set`; point x is PP[x - pb].  Returns the point beyond the facet
// whose sphere through it holds no other such point, or GW_NONE (a hull
// facet); the same in every lane.  With a grid, the first candidate comes
// from the cells around the facet's circumcentre and the exact pass reads
// only the cells under the ball through the facet and that candidate (any
// point that comes before it lies strictly inside that sphere); without
// one, or when the ball covers too many cells, every point is read.
template <int D>
__device__ uint32_t gw_search(PredT<false>& pr, const double4* PP, uint32_t pb, uint32_t lo,
                              uint32_t hi, const uint4& t, uint32_t i, uint32_t lane,
                              const GwGrid& G, bool grid, uint32_t set) {
  // facet points in their slots (slot i takes the candidate)
  PtsX F;
#pragma unroll
  for (int k = 0; k <= D; k++) {
    F.p[k][0] = F.p[k][1] = F.p[k][2] = 0.0;
    F.key[k] = 0;
    if (k != (int)i) gw_load(PP, vget(t, k) - pb, F.p[k], F.key[k]);
  }
  double gl[3] = {0.0, 0.0, 0.0}, ginv = 0.0;
  int gd[3] = {1, 1, 1}, gbase = 0;
  if (grid) {
    gl[0] = G.meta[4 * set];
    gl[1] = G.meta[4 * set + 1];
    gl[2] = G.meta[4 * set + 2];
    ginv = G.meta[4 * set + 3];
    gd[0] = G.dims[4 * set];
    gd[1] = G.dims[4 * set + 1];
    gd[2] = G.dims[4 * set + 2];
    gbase = G.dims[4 * set + 3];
  }
  // A first candidate: the least pencil parameter in FP64 over the points
  // beyond the facet (a guess; the exact order decides below).
  uint32_t guess = GW_NONE;
  double gp[3] = {0.0, 0.0, 0.0};   // the guess's coordinates and key, carried along
  unsigned long long gk = 0;
  {
    double cf[3], r2, nrm[3];
    if (facet_frame<D>(F, i, PP[vget(t, (int)i) - pb], cf, &r2, nrm)) {
      double bnum = 0.0, bden = 1.0;
      auto consider = [&](uint32_t q, const double4& cp) {
        const double wx = cp.x - cf[0], wy = cp.y - cf[1], wz = cp.z - cf[2];
        const double h = wx * nrm[0] + wy * nrm[1] + (D == 3 ? wz * nrm[2] : 0.0);
        if (!(h > 0.0)) return;
        // the facet's own points lie on its hyperplane (h is rounding)
        bool vert = false;
#pragma unroll
        for (int k = 0; k <= D; k++) vert |= (k != (int)i && vget(t, k) == q);
        if (vert) return;
        const double num = (wx * wx + wy * wy + (D == 3 ? wz * wz : 0.0)) - r2;
        if (guess == GW_NONE || num * bden < bnum * h) {
          guess = q;
          bnum = num;
          bden = h;
          gp[0] = cp.x;
          gp[1] = cp.y;
          gp[2] = cp.z;
          gk = (unsigned long long)__double_as_longlong(cp.w);
        }
      };
      auto reduce = [&]() {
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
          const uint32_t oq = __shfl_xor(guess, off, 64);
          const double on = __shfl_xor(bnum, off, 64), od = __shfl_xor(bden, off, 64);
          const double ox = __shfl_xor(gp[0], off, 64), oy = __shfl_xor(gp[1], off, 64),
                       oz = __shfl_xor(gp[2], off, 64);
          const unsigned long long ok = __shfl_xor(gk, off, 64);
          if (oq != GW_NONE && (guess == GW_NONE || on * bden < bnum * od)) {
            guess = oq;
            bnum = on;
            bden = od;
            gp[0] = ox;
            gp[1] = oy;
            gp[2] = oz;
            gk = ok;
          }
        }
        guess = __shfl(guess, 0, 64);
        gp[0] = __shfl(gp[0], 0, 64);
        gp[1] = __shfl(gp[1], 0, 64);
        gp[2] = __shfl(gp[2], 0, 64);
        gk = __shfl(gk, 0, 64);
      };
      if (grid) {
        // the cells around the facet's circumcentre
        const int cx = gw_coord(cf[0], gl[0], ginv, gd[0]);
        const int cy = gw_coord(cf[1], gl[1], ginv, gd[1]);
        const int cz = D == 3 ? gw_coord(cf[2], gl[2], ginv, gd[2]) : 0;
        const int x0 = max(cx - 1, 0), x1 = min(cx + 1, gd[0] - 1);
        for (int z = max(cz - 1, 0); z <= min(cz + 1, gd[2] - 1); z++)
          for (int y = max(cy - 1, 0); y <= min(cy + 1, gd[1] - 1); y++) {
            const int row = gbase + (z * gd[1] + y) * gd[0];
            const uint32_t a = G.cstart[row + x0], b = G.cstart[row + x1 + 1];
            for (uint32_t q = a + lane; q < b; q += 64) consider(q, PP[q - pb]);
          }
        reduce();
      }
      if (guess == GW_NONE) {
        for (uint32_t q0 = lo + lane; q0 < hi; q0 += 4 * 64) {
          double4 cp[4];
#pragma unroll
          for (int u = 0; u < 4; u++) {
            const uint32_t q = q0 + 64u * (uint32_t)u;
            cp[u] = PP[(q < hi ? q : lo) - pb];
          }
#pragma unroll
          for (int u = 0; u < 4; u++) {
            const uint32_t q = q0 + 64u * (uint32_t)u;
            if (q < hi) consider(q, cp[u]);
          }
        }
        reduce();
      }
    }
  }
  // The exact scan starts from the guess when it lies strictly beyond the
  // facet: a point outside the conservatively enlarged ball through the
  // facet and the current candidate cannot come before it (it is not
  // strictly inside the sphere), so only points inside the ball are
  // tested.
  uint32_t best = GW_NONE;
  double bp[3] = {0.0, 0.0, 0.0};
  unsigned long long bk = 0;
  bool ball = false;
  double sc[3] = {0.0, 0.0, 0.0}, sr2 = 0.0, sr = 0.0;
  if (guess != GW_NONE) {
    PtsX X = F;
    put_slot<D>(X, i, gp, gk);
    if (pr.template orient<D>(X) > 0) {
      best = guess;
      bp[0] = gp[0]; bp[1] = gp[1]; bp[2] = gp[2];
      bk = gk;
      ball = gw_ball<D>(F, i, gp, sc, &sr);
      sr2 = sr * sr;
    }
  }
  auto test = [&](uint32_t q, const double4& cp) {
    if (q == best) return;
    if (ball) {
      const double dx = cp.x - sc[0], dy = cp.y - sc[1], dz = cp.z - sc[2];
      if (dx * dx + dy * dy + dz * dz > sr2) return;
    }
    bool vert = false;
#pragma unroll
    for (int k = 0; k <= D; k++) vert |= (k != (int)i && vget(t, k) == q);
    if (vert) return;
    const double qp[3] = {cp.x, cp.y, cp.z};
    const unsigned long long qk = (unsigned long long)__double_as_longlong(cp.w);
    PtsX X = F;
    put_slot<D>(X, i, qp, qk);
    if (pr.template orient<D>(X) <= 0) return;
    bool take = best == GW_NONE;
    if (!take) {
      put_slot<D>(X, i, bp, bk);
      X.p[D + 1][0] = qp[0]; X.p[D + 1][1] = qp[1]; X.p[D + 1][2] = qp[2];
      X.key[D + 1] = qk;
      take = pr.template insphere<D>(X) > 0;
    }
    if (take) {
      best = q;
      bp[0] = qp[0]; bp[1] = qp[1]; bp[2] = qp[2];
      bk = qk;
      double r = 0.0;
      ball = gw_ball<D>(F, i, qp, sc, &r);
      sr2 = r * r;
    }
  };
  // the cells under the guess's ball, when there are few of them
  bool local = false;
  if (grid && ball) {
    int c0[3] = {0, 0, 0}, c1[3] = {0, 0, 0};
    long long ncell = 1;
#pragma unroll
    for (int k = 0; k < 3; k++) {
      if (k < D) {
        c0[k] = gw_coord(sc[k] - sr, gl[k], ginv, gd[k]);
        c1[k] = gw_coord(sc[k] + sr, gl[k], ginv, gd[k]);
      }
      ncell *= c1[k] - c0[k] + 1;
    }
    if (ncell <= (long long)GW_BALL_CELLS) {
      local = true;
      for (int z = c0[2]; z <= c1[2]; z++)
        for (int y = c0[1]; y <= c1[1]; y++) {
          const int row = gbase + (z * gd[1] + y) * gd[0];
          const uint32_t a = G.cstart[row + c0[0]], b = G.cstart[row + c1[0] + 1];
          for (uint32_t q = a + lane; q < b; q += 64) test(q, PP[q - pb]);
        }
    }
  }
  if (!local) {
    // every point, loaded four at a time ahead of the tests
    for (uint32_t q0 = lo + lane; q0 < hi; q0 += 4 * 64) {
      double4 cp[4];
#pragma unroll
      for (int u = 0; u < 4; u++) {
        const uint32_t q = q0 + 64u * (uint32_t)u;
        cp[u] = PP[(q < hi ? q : lo) - pb];
      }
#pragma unroll
      for (int u = 0; u < 4; u++) {
        const uint32_t q = q0 + 64u * (uint32_t)u;
        if (q < hi) test(q, cp[u]);
      }
    }
  }
  // the wavefront's first candidate: a minimum over the lanes under the
  // same order (a strict total order, so every lane ends with it)
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t o = __shfl_xor(best, off, 64);
    const double op[3] = {__shfl_xor(bp[0], off, 64), __shfl_xor(bp[1], off, 64),
                          __shfl_xor(bp[2], off, 64)};
    const unsigned long long ok = __shfl_xor(bk, off, 64);
    if (o == GW_NONE || o == best) continue;
    bool take = best == GW_NONE;
    if (!take) {
      PtsX X = F;
      put_slot<D>(X, i, bp, bk);
      X.p[D + 1][0] = op[0]; X.p[D + 1][1] = op[1]; X.p[D + 1][2] = op[2];
      X.key[D + 1] = ok;
      take = pr.template insphere<D>(X) > 0;
    }
    if (take) {
      best = o;
      bp[0] = op[0]; bp[1] = op[1]; bp[2] = op[2];
      bk = ok;
    }
  }
  return best;
}

// One level: every facet of the input list, one wavefront each, finds the
// simplex beyond it; a simplex not found before is recorded and its other
// D facets go to the output list.  Facet (c, i) is the facet of cell c
// opposite its vertex i, searched away from that vertex, among the points
// of its own set (through the sets' grid).
template <int D>
__global__ __launch_bounds__(GW_THREADS) void k_gw_level(GwState g, const uint32_t* fin,
                                                         const uint32_t* cnt_in, uint32_t* fout,
                                                         uint32_t* cnt_out, uint32_t fcap) {
  // new simplices of the block's chunk of facets: one allocation of cells
  // and of next-level facets per chunk (counters that every new simplex
  // hit alone would serialise a large level); the chunk is one facet per
  // wavefront on small levels, so that they spread over the device
  __shared__ uint4 s_new[GW_CHUNK];
  __shared__ uint32_t s_opp[GW_CHUNK];
  __shared__ uint32_t s_nnew, s_cbase, s_fbase, s_ok;
  const uint32_t nin = *cnt_in;
  if (nin == 0 || *g.flags) return;
  const uint32_t wpb = GW_THREADS / 64;
  uint32_t ch = (nin + gridDim.x - 1) / gridDim.x;
  ch = (ch + wpb - 1) / wpb * wpb;
  ch = ch < wpb ? wpb : (ch > GW_CHUNK ? GW_CHUNK : ch);
  if (blockIdx.x * ch >= nin) return;
  const double4* PP = g.P;
  PredT<false> pr;
  pr.init(g.flags);
  const uint32_t lane = threadIdx.x & 63u;
  for (uint32_t c0 = blockIdx.x * ch; c0 < nin; c0 += gridDim.x * ch) {
    if (threadIdx.x == 0) s_nnew = 0;
    __syncthreads();
    const uint32_t c1 = min(c0 + ch, nin);
    for (uint32_t e = c0 + threadIdx.x / 64; e < c1; e += wpb) {
      const uint32_t ent = fin[e];
      const uint32_t c = ent >> 2, i = ent & 3u;
      // the facet's vertices with two of them swapped: (facet, x) is then
      // positively oriented exactly for x strictly beyond the facet
      uint4 t = g.cells[c].v;
      const int a = i == 0 ? 1 : 0, b = i <= 1 ? 2 : 1;
      // the points of the facet's set
      const uint32_t set = g.sof[vget(t, a)];
      const uint32_t lo = g.soff[set], hi = g.soff[set + 1];
      {
        const uint32_t x = vget(t, a);
        vput(t, a, vget(t, b));
        vput(t, b, x);
      }
      const uint32_t best = gw_search<D>(pr, PP, 0, lo, hi, t, i, lane, g.grid, g.has_grid, set);
      if (lane == 0 && best != GW_NONE) {
        vput(t, (int)i, best);
        if (gw_claim<D>(g, t, set) == 1) {
          const uint32_t k = atomicAdd(&s_nnew, 1u);
          s_new[k] = t;
          s_opp[k] = i;
        }
      }
    }
    __syncthreads();
    const uint32_t nn = s_nnew;
    if (threadIdx.x == 0) {
      s_ok = 0;
      if (nn) {
        const uint32_t cb = atomicAdd(g.ncells, nn);
        const uint32_t fb = atomicAdd(cnt_out, nn * (uint32_t)D);
        if ((uint64_t)cb + nn > g.cap || (uint64_t)fb + (uint64_t)nn * D > fcap) {
          atomicOr(g.flags, (uint32_t)GW_FAIL_CAP);
        } else {
          s_cbase = cb;
          s_fbase = fb;
          s_ok = 1;
        }
      }
    }
    __syncthreads();
    if (s_ok) {
      for (uint32_t k = threadIdx.x; k < nn; k += GW_THREADS) {
        const uint32_t nc = s_cbase + k;
        gw_cell(g.cells[nc], s_new[k]);
        uint32_t w = s_fbase + k * (uint32_t)D;
        for (uint32_t f = 0; f <= (uint32_t)D; f++)
          if (f != s_opp[k]) fout[w++] = (nc << 2) | f;
      }
    }
    __syncthreads();
  }
}

// The same level for a single set copied into LDS by every block (sets of
// at most GW_LDS_POINTS points): a facet search is then a chain of LDS
// reads rather than of L2 loads; such sets have few facets per level, so
// each new simplex takes its cell and facets from the counters directly.
template <int D>
__global__ __launch_bounds__(GW_THREADS) void k_gw_level_lds(GwState g, const uint32_t* fin,
                                                             const uint32_t* cnt_in,
                                                             uint32_t* fout, uint32_t* cnt_out,
                                                             uint32_t fcap) {
  extern __shared__ double4 s_pts[];
  const uint32_t nin = *cnt_in;
  if (nin == 0 || *g.flags) return;
  const uint32_t wpb = GW_THREADS / 64;
  if (blockIdx.x * wpb >= nin) return;
  for (uint32_t j = threadIdx.x; j < g.n; j += GW_THREADS) s_pts[j] = g.P[j];
  __syncthreads();
  PredT<false> pr;
  pr.init(g.flags);
  const uint32_t lane = threadIdx.x & 63u;
  for (uint32_t e = blockIdx.x * wpb + threadIdx.x / 64; e < nin; e += gridDim.x * wpb) {
    const uint32_t ent = fin[e];
    const uint32_t c = ent >> 2, i = ent & 3u;
    uint4 t = g.cells[c].v;
    const int a = i == 0 ? 1 : 0, b = i <= 1 ? 2 : 1;
    {
      const uint32_t x = vget(t, a);
      vput(t, a, vget(t, b));
      vput(t, b, x);
    }
    const uint32_t best = gw_search<D>(pr, s_pts, 0, 0, g.n, t, i, lane, g.grid, false, 0);
    if (lane == 0 && best != GW_NONE) {
      vput(t, (int)i, best);
      uint32_t nc = 0;
      if (gw_record<D>(g, t, 0, &nc)) {
        const uint32_t at = atomicAdd(cnt_out, (uint32_t)D);
        if (at + D > fcap) {
          atomicOr(g.flags, (uint32_t)GW_FAIL_CAP);
        } else {
          uint32_t w = at;
          for (uint32_t k = 0; k <= (uint32_t)D; k++)
            if (k != i) fout[w++] = (nc << 2) | k;
        }
      }
    }
  }
}

// The set of every point.
__global__ void k_gw_setof(const uint32_t* soff, uint32_t* sof) {
  const uint32_t set = blockIdx.x, lo = soff[set], hi = soff[set + 1];
  for (uint32_t j = lo + threadIdx.x; j < hi; j += blockDim.x) sof[j] = set;
}

// Grid of each set (one block per set): its bounding box, about two
// points per cell, at most GW_GRID_AXIS cells per axis.  dims[4s + 3]
// receives the set's cell count (the host turns it into the first cell).
constexpr int GW_GRID_AXIS = 256;
__global__ void k_gw_grid_dims(const double4* P, const uint32_t* soff, int D, double* meta,
                               int* dims) {
  __shared__ double s_lo[3][GW_THREADS], s_hi[3][GW_THREADS];
  const uint32_t set = blockIdx.x, lo = soff[set], hi = soff[set + 1];
  double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (uint32_t j = lo + threadIdx.x; j < hi; j += GW_THREADS) {
    const double4 q = P[j];
    const double c[3] = {q.x, q.y, q.z};
    for (int k = 0; k < 3; k++) {
      mn[k] = fmin(mn[k], c[k]);
      mx[k] = fmax(mx[k], c[k]);
    }
  }
  for (int k = 0; k < 3; k++) {
    s_lo[k][threadIdx.x] = mn[k];
    s_hi[k][threadIdx.x] = mx[k];
  }
  __syncthreads();
  for (uint32_t w = GW_THREADS / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w)
      for (int k = 0; k < 3; k++) {
        s_lo[k][threadIdx.x] = fmin(s_lo[k][threadIdx.x], s_lo[k][threadIdx.x + w]);
        s_hi[k][threadIdx.x] = fmax(s_hi[k][threadIdx.x], s_hi[k][threadIdx.x + w]);
      }
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  const uint32_t n = hi - lo;
  double e[3], vol = 1.0;
  int nd = 0;
  for (int k = 0; k < 3; k++) {
    e[k] = (k < D && n) ? s_hi[k][0] - s_lo[k][0] : 0.0;
    if (e[k] > 0.0) {
      vol *= e[k];
      nd++;
    }
  }
  const double target = n > 2 ? 0.5 * n : 1.0;
  double h = nd ? pow(vol / target, 1.0 / nd) : 1.0;
  if (!(h > 0.0)) h = 1.0;
  int g[3];
  // a flat set would get far more cells than points: coarser until at
  // most about four cells per point
  for (int it = 0; it < 64; it++) {
    for (int k = 0; k < 3; k++) {
      const double c = e[k] > 0.0 ? floor(e[k] / h) + 1.0 : 1.0;
      g[k] = c > GW_GRID_AXIS ? GW_GRID_AXIS : (int)c;
    }
    if ((double)g[0] * g[1] * g[2] <= 4.0 * n + 64.0) break;
    h *= 1.25;
  }
  for (int k = 0; k < 3; k++) meta[4 * set + k] = n ? s_lo[k][0] : 0.0;
  meta[4 * set + 3] = 1.0 / h;
  dims[4 * set] = g[0];
  dims[4 * set + 1] = g[1];
  dims[4 * set + 2] = g[2];
  dims[4 * set + 3] = g[0] * g[1] * g[2];
}

// Cell of every point (one thread per point), counted per cell.
__global__ void k_gw_grid_cell(const double4* P, uint32_t n, const uint32_t* sof,
                               const double* meta, const int* dims, int D, uint32_t* cellof,
                               uint32_t* cnt) {
  const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const uint32_t s = sof[j];
  const double4 q = P[j];
  const double inv = meta[4 * s + 3];
  const int cx = gw_coord(q.x, meta[4 * s], inv, dims[4 * s]);
  const int cy = gw_coord(q.y, meta[4 * s + 1], inv, dims[4 * s + 1]);
  const int cz = D == 3 ? gw_coord(q.z, meta[4 * s + 2], inv, dims[4 * s + 2]) : 0;
  const uint32_t c = (uint32_t)dims[4 * s + 3] + ((uint32_t)cz * dims[4 * s + 1] + cy) * dims[4 * s] + cx;
  cellof[j] = c;
  atomicAdd(&cnt[c], 1u);
}

// The points in cell order (each set keeps its range); perm[new] = old.
__global__ void k_gw_grid_fill(const double4* P, uint32_t n, const uint32_t* cellof,
                               const uint32_t* cstart, uint32_t* cur, double4* out,
                               uint32_t* perm) {
  const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const uint32_t c = cellof[j];
  const uint32_t at = cstart[c] + atomicAdd(&cur[c], 1u);
  out[at] = P[j];
  perm[at] = j;
}

// Cell vertices back to the caller's point indices.
__global__ void k_gw_unperm(Cell* cells, uint32_t nc, const uint32_t* perm, int D) {
  const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nc) return;
  uint4 v = cells[c].v;
  v.x = perm[v.x];
  v.y = perm[v.y];
  v.z = perm[v.z];
  if (D == 3) v.w = perm[v.w];
  cells[c].v = v;
}

}  // namespace

int gift_wrap_sets(const double4* P, uint32_t n, const uint32_t* soff, uint32_t nsets,
                   uint32_t max_set, int D, CellPool& pool, uint32_t* levels, hipStream_t st,
                   uint32_t* first) {
  *levels = 0;
  if ((D != 2 && D != 3) || nsets == 0 || n < (uint32_t)D + 2) return DT_E_NOT_READY;
  // the set's number and D+1 set-local indices share one 64-bit key: 16
  // bits per index for a single set, 13 for several
  const int kbits = nsets == 1 ? 16 : GW_LOCAL_BITS;
  if (max_set > (nsets == 1 ? GW_MAX_POINTS : GW_MAX_SET_POINTS)) return DT_E_NOT_READY;
  if ((uint64_t)nsets > (1ull << (64 - (D + 1) * kbits))) return DT_E_NOT_READY;
  // about 6.8 n simplices in 3D and 2 n in 2D; room for far more
  const size_t cap = (size_t)n * (D == 3 ? 12 : 4) + (size_t)64 * nsets;
  if (cap >= (1ull << 30)) return DT_E_NOT_READY;
  size_t tsize = 64;
  while (tsize < 2 * cap) tsize <<= 1;
  const size_t fcap = cap * (size_t)D + 8;
  DevBuf nn, best, flags, table, fa, fb, cnt, sof;
  DT_TRY(pool.cells.alloc(cap * sizeof(Cell)));
  DT_TRY(pool.set_cell0.alloc(16));
  DT_TRY(nn.alloc((size_t)nsets * GW_BASES * (GW_NN + 1) * 4));
  DT_TRY(best.alloc((size_t)nsets * GW_BASES * 4));
  DT_TRY(flags.alloc(16));
  DT_TRY(table.alloc(tsize * 8));
  DT_TRY(fa.alloc(fcap * 4));
  DT_TRY(fb.alloc(fcap * 4));
  DT_TRY(cnt.alloc((size_t)(GW_MAX_LEVELS + 1) * 4 + 4));
  DT_TRY(sof.alloc((size_t)n * 4));
  uint32_t* ncells = cnt.as<uint32_t>() + GW_MAX_LEVELS + 1;
  DT_HIP(hipMemsetAsync(best.p, 0xFF, (size_t)nsets * GW_BASES * 4, st));
  DT_HIP(hipMemsetAsync(flags.p, 0, 4, st));
  DT_HIP(hipMemsetAsync(table.p, 0xFF, tsize * 8, st));
  DT_HIP(hipMemsetAsync(cnt.p, 0, (size_t)(GW_MAX_LEVELS + 2) * 4, st));
  DT_HIP(hipMemsetAsync(pool.set_cell0.p, 0, 4, st));
  hipLaunchKernelGGL(k_gw_setof, dim3(nsets), dim3(GW_THREADS), 0, st, soff, sof.as<uint32_t>());
  const bool lds = nsets == 1 && n <= GW_LDS_POINTS;
  // the grid (not for a single set small enough for LDS): the points
  // sorted by cell within each set
  DevBuf gmeta, gdims, gcnt, gstart, gcur, cellof, P2, perm;
  GwGrid grid{nullptr, nullptr, nullptr};
  if (!lds) {
    DT_TRY(gmeta.alloc((size_t)nsets * 4 * sizeof(double)));
    DT_TRY(gdims.alloc((size_t)nsets * 4 * sizeof(int)));
    hipLaunchKernelGGL(k_gw_grid_dims, dim3(nsets), dim3(GW_THREADS), 0, st, P, soff, D,
                       gmeta.as<double>(), gdims.as<int>());
    DT_HIP(hipGetLastError());
    std::vector<int> hd((size_t)nsets * 4);
    DT_HIP(hipMemcpyAsync(hd.data(), gdims.p, hd.size() * sizeof(int), hipMemcpyDeviceToHost, st));
    DT_HIP(hipStreamSynchronize(st));
    uint64_t ncell = 0;
    for (uint32_t i = 0; i < nsets; i++) {
      const uint64_t c = (uint64_t)hd[4 * i + 3];
      hd[4 * i + 3] = (int)ncell;
      ncell += c;
    }
    if (ncell >= (1ull << 31)) return DT_E_NOT_READY;
    DT_HIP(hipMemcpyAsync(gdims.p, hd.data(), hd.size() * sizeof(int), hipMemcpyHostToDevice, st));
    DT_TRY(gcnt.alloc((size_t)(ncell + 1) * 4));
    DT_TRY(gstart.alloc((size_t)(ncell + 1) * 4));
    DT_TRY(gcur.alloc((size_t)ncell * 4));
    DT_TRY(cellof.alloc((size_t)n * 4));
    DT_TRY(P2.alloc((size_t)n * sizeof(double4)));
    DT_TRY(perm.alloc((size_t)n * 4));
    DT_HIP(hipMemsetAsync(gcnt.p, 0, (size_t)(ncell + 1) * 4, st));
    DT_HIP(hipMemsetAsync(gcur.p, 0, (size_t)ncell * 4, st));
    const uint32_t nb = (n + GW_THREADS - 1) / GW_THREADS;
    hipLaunchKernelGGL(k_gw_grid_cell, dim3(nb), dim3(GW_THREADS), 0, st, P, n, sof.as<uint32_t>(),
                       gmeta.as<double>(), gdims.as<int>(), D, cellof.as<uint32_t>(),
                       gcnt.as<uint32_t>());
    DT_TRY(exclusive_scan(gcnt.as<uint32_t>(), gstart.as<uint32_t>(), (uint32_t)ncell + 1, st));
    hipLaunchKernelGGL(k_gw_grid_fill, dim3(nb), dim3(GW_THREADS), 0, st, P, n,
                       cellof.as<uint32_t>(), gstart.as<uint32_t>(), gcur.as<uint32_t>(),
                       P2.as<double4>(), perm.as<uint32_t>());
    DT_HIP(hipGetLastError());
    grid = GwGrid{gmeta.as<double>(), gdims.as<int>(), gstart.as<uint32_t>()};
    P = P2.as<double4>();
  }
  GwState g{P, n, soff, sof.as<uint32_t>(), pool.cells.as<Cell>(), (uint32_t)cap, ncells,
            table.as<unsigned long long>(), (uint32_t)(tsize - 1), flags.as<uint32_t>(),
            kbits, grid, !lds};
  const uint32_t ncomb = D == 2 ? seed_combos<2>(GW_NN) : seed_combos<3>(GW_NN);
  hipLaunchKernelGGL(k_gw_nearest, dim3(nsets * GW_BASES), dim3(GW_THREADS), 0, st, P, soff,
                     nn.as<uint32_t>());
  const uint64_t sw0 = (uint64_t)nsets * ncomb, sw1 = sw0 * (GW_BASES - 1);
  const uint32_t sb0 = (uint32_t)((sw0 * 64 + GW_THREADS - 1) / GW_THREADS);
  const uint32_t sb1 = (uint32_t)((sw1 * 64 + GW_THREADS - 1) / GW_THREADS);
#define GW_LAUNCH(K, ...)                                                                 \
  do {                                                                                    \
    if (D == 2) hipLaunchKernelGGL((K<2>), __VA_ARGS__);                                  \
    else hipLaunchKernelGGL((K<3>), __VA_ARGS__);                                         \
  } while (0)
  GW_LAUNCH(k_gw_seed, dim3(sb0), dim3(GW_THREADS), 0, st, P, soff, nsets, nn.as<uint32_t>(),
            ncomb, 0u, 1u, best.as<uint32_t>(), flags.as<uint32_t>());
  GW_LAUNCH(k_gw_seed, dim3(sb1), dim3(GW_THREADS), 0, st, P, soff, nsets, nn.as<uint32_t>(),
            ncomb, 1u, GW_BASES - 1, best.as<uint32_t>(), flags.as<uint32_t>());
  GW_LAUNCH(k_gw_start, dim3((nsets + 63) / 64), dim3(64), 0, st, g, nsets, nn.as<uint32_t>(),
            best.as<uint32_t>(), fa.as<uint32_t>(), cnt.as<uint32_t>(), first);
  DT_HIP(hipGetLastError());
  uint32_t lev = 0;
  for (;;) {
    for (uint32_t r = 0; r < GW_GROUP && lev < GW_MAX_LEVELS; r++, lev++) {
      const uint32_t* fin = (lev & 1u) ? fb.as<uint32_t>() : fa.as<uint32_t>();
      uint32_t* fout = (lev & 1u) ? fa.as<uint32_t>() : fb.as<uint32_t>();
      if (lds)
        GW_LAUNCH(k_gw_level_lds, dim3(GW_LEVEL_BLOCKS), dim3(GW_THREADS),
                  (size_t)n * sizeof(double4), st, g, fin, cnt.as<uint32_t>() + lev, fout,
                  cnt.as<uint32_t>() + lev + 1, (uint32_t)fcap);
      else
        GW_LAUNCH(k_gw_level, dim3(GW_LEVEL_BLOCKS), dim3(GW_THREADS), 0, st, g, fin,
                  cnt.as<uint32_t>() + lev, fout, cnt.as<uint32_t>() + lev + 1, (uint32_t)fcap);
    }
    DT_HIP(hipGetLastError());
    uint32_t h[2] = {0, 0};
    DT_HIP(hipMemcpyAsync(&h[0], cnt.as<uint32_t>() + lev, 4, hipMemcpyDeviceToHost, st));
    DT_HIP(hipMemcpyAsync(&h[1], flags.p, 4, hipMemcpyDeviceToHost, st));
    DT_HIP(hipStreamSynchronize(st));
    if (h[1]) {                               // no seed, or a capacity: fall back
      if (getenv("DT_DEBUG")) fprintf(stderr, "[gwrap] failure bits %x at level %u\n", h[1], lev);
      return DT_E_NOT_READY;
    }
    if (h[0] == 0) break;
    if (lev >= GW_MAX_LEVELS) return DT_E_NOT_READY;
  }
#undef GW_LAUNCH
  uint32_t nc = 0;
  std::vector<uint32_t> hc(lev + 1);
  DT_HIP(hipMemcpyAsync(&nc, ncells, 4, hipMemcpyDeviceToHost, st));
  DT_HIP(hipMemcpyAsync(hc.data(), cnt.p, (size_t)(lev + 1) * 4, hipMemcpyDeviceToHost, st));
  DT_HIP(hipStreamSynchronize(st));
  if (!lds && nc) {
    hipLaunchKernelGGL(k_gw_unperm, dim3((nc + GW_THREADS - 1) / GW_THREADS), dim3(GW_THREADS), 0,
                       st, pool.cells.as<Cell>(), nc, perm.as<uint32_t>(), D);
    DT_HIP(hipGetLastError());
    DT_HIP(hipStreamSynchronize(st));
  }
  pool.cap = (uint32_t)cap;
  pool.ncells = nc;
  // levels that had facets to search
  uint32_t nl = 0;
  for (uint32_t x = 0; x <= lev; x++) nl += hc[x] ? 1u : 0u;
  *levels = nl;
  return DT_OK;
}

int gift_wrap(const double4* P, uint32_t n, int D, CellPool& pool, uint32_t* levels,
              hipStream_t st) {
  *levels = 0;
  if (n < (uint32_t)D + 2 || n > GW_MAX_POINTS || (D != 2 && D != 3)) return DT_E_NOT_READY;
  DevBuf soff;
  DT_TRY(soff.alloc(8));
  const uint32_t h[2] = {0u, n};
  DT_HIP(hipMemcpyAsync(soff.p, h, 8, hipMemcpyHostToDevice, st));
  // (h outlives the copy: gift_wrap_sets synchronises the stream)
  return gift_wrap_sets(P, n, soff.as<uint32_t>(), 1, n, D, pool, levels, st);
}

}  // namespace dtk
