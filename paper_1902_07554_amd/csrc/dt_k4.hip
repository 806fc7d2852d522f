// Batched local Delaunay triangulations on gfx950 (the "parallel
// triangulation" step of Algorithm 1, and the sample and border
// triangulations, which reuse it).
//
// Every set of a job is triangulated at once, in synchronous rounds of
// parallel Bowyer-Watson insertion over all sets together:
//   pick     every active uninserted point bids for the cell it lies in;
//            each cell keeps its lowest random key;
//   select   a point that holds its cell's bid becomes a candidate unless a
//            cell within three facet-hops holds a smaller one;
//   cavity   each candidate grows its conflict region (cells whose
//            circumsphere strictly contains it, or hull cells whose facet it
//            sees) and claims those cells and the cells around them with
//            its key (atomic minimum);
//   insert   a candidate whose cavity cells and surrounding cells carry no
//            smaller key wins: no other winner touches its cavity or its
//            shell, so winners retriangulate independently, exactly as a
//            sequential insertion would;
//   relocate (lazily, at the next pick) active points whose cell was
//            destroyed follow forward pointers and walk to their new cell.
// Points become active in levels of growing priority threshold, so a point
// is located when its turn approaches rather than after every round.
// The globally smallest key always wins, so every round makes progress.
// Because the result of each round equals a sequence of ordinary
// insertions, the final triangulation is the unique (perturbed) Delaunay
// triangulation of each set.
//
// Why cavities rather than flips: a batch of simultaneous 1-to-4 splits
// followed by parallel flipping can stall in 3D on configurations no flip
// repairs; cavity insertion with priority claims always terminates.
//
// Data layout (HBM): one 64-byte record per cell (uint4 vertices, uint4
// neighbours = cell << 2 | facet index in the neighbour, the 64-bit cavity
// and shell claims, the forward pointer and the cavity position), and the
// cells' bids in an array of their own.  New cells are always appended
// (old slots are never reused within a job), so a destroyed cell keeps its
// data and a forward pointer for the walk; the cells of one star are
// contiguous.
#include "dt_common.hpp"
#include "dt_internal.hpp"
#include "dt_pred.hpp"
#include "dt_block.hpp"
#include "dt_prims.hpp"
#include "dt_gwrap.hpp"

#include <stdio.h>
#include <stdlib.h>

#include <vector>

namespace dtk {

constexpr int BLOCK = 256;
// ploc flag: the stored cell is only a start for the walk (dormant point)
constexpr uint32_t NEEDWALK = 0x80000000u;
constexpr uint32_t NEAR_WIN = 4;   // neighbours on each side searched for a walk start
// ploc flag: the point's bid is in place on its (live) cell
constexpr uint32_t BIDDED = 0x40000000u;
constexpr uint32_t LOCMASK = 0x3FFFFFFFu;   // cell indices stay below 2^30

struct K4Args {
  const double4* pts;
  const uint32_t* pset;
  const uint32_t* set_off;
  uint32_t* ploc;
  Cell* cells;
  uint32_t* set_cell0;
  uint32_t* cand_pt;
  uint32_t* cand_n;
  uint32_t* cav;
  uint32_t* cavinfo;
  uint32_t* cand_ext;   // extension chunk of a candidate's cavity list, or DONE
  uint32_t* extcell;    // [MAXEXT * EXTCAP]
  uint32_t* extinfo;
  Counters* ctr;
  // striped statistics (many blocks add to them at once; NSTRIPE copies
  // keep the atomics from serialising on one address)
  struct Stripes* sx;
  uint32_t npts;
  uint32_t nsets;
  uint32_t cap;
  uint32_t maxcand;
  uint32_t cavcap;
  uint32_t round;
  uint32_t* act;        // active point list (a superset of the pending points);
                        // its length and the level's threshold live in ctr
  uint32_t grow_div;
  uint32_t grow_num;    // threshold growth per level, in eighths
  uint32_t* vcell;      // a cell incident to each inserted point (start of later walks)
  // smallest bid of a pending point inside each cell: an array of its own,
  // so that the selection's ring checks read 8 bytes per cell from lines
  // shared by the cells of one star (allocated together)
  unsigned long long* bid;
  uint32_t rings;       // bid rings checked by the selection (0 to 3)
  int fp32;
  // pool-sized cavity list for the one candidate per round whose cavity
  // outgrew the regular list (allocated on the first such request)
  uint32_t* gcell;
  uint32_t* ginfo;
  uint32_t gcap;
};

// Large cavities spill from the fixed per-candidate list into extension
// chunks taken from a small pool (reset every round).
constexpr uint32_t MAXEXT = 256;
constexpr uint32_t NSTRIPE = 64;
struct Stripes {
  unsigned long long pred[NSTRIPE][16];   // [orient2, orient3, in2, in3][calls, fp32, fp64, exact]
  unsigned long long cavcells[NSTRIPE];   // cells placed in cavities
  uint32_t pend[NSTRIPE];                 // pending points this round
  uint32_t ins[NSTRIPE];                  // points inserted this round
  uint32_t maxcav[NSTRIPE];               // largest cavity
  unsigned long long verified[NSTRIPE];   // candidates whose search completed
};
constexpr uint32_t EXTCAP = 8192;
// cand_ext value of the candidate that uses the pool-sized list
constexpr uint32_t GIANT = 0xFFFFFFFEu;

struct CavList {
  uint32_t* a;
  uint32_t* ia;
  uint32_t* b;
  uint32_t* ib;
  uint32_t cap;
  __device__ __forceinline__ uint32_t& cell(uint32_t h) { return h < cap ? a[h] : b[h - cap]; }
  __device__ __forceinline__ uint32_t& info(uint32_t h) { return h < cap ? ia[h] : ib[h - cap]; }
};

// ------------------------------------------------------------ helpers
__device__ __forceinline__ uint32_t vat(const uint4& v, int i) {
  return i == 0 ? v.x : (i == 1 ? v.y : (i == 2 ? v.z : v.w));
}
// A new cell: vertices, no bid, no claims, alive (neighbours are written
// apart).
template <class A>
__device__ __forceinline__ void init_cell(A& a, uint32_t x, const uint4& v) {
  Cell& c = a.cells[x];
  a.bid[x] = NOKEY;
  c.v = v;
  c.spare = 0;
  c.cav = NOKEY;
  c.shell = NOKEY;
  c.fwd = ALIVE;
  c.pos = 0;
}
// Neighbour slot s of cell x, for single-slot updates.
__device__ __forceinline__ uint32_t* nslot(Cell* cells, uint32_t x, uint32_t s) {
  return reinterpret_cast<uint32_t*>(&cells[x].n) + s;
}
__device__ __forceinline__ void vset(uint4& v, int i, uint32_t x) {
  if (i == 0) v.x = x;
  else if (i == 1) v.y = x;
  else if (i == 2) v.z = x;
  else v.w = x;
}

__device__ __forceinline__ void load_pt(const double4* pts, uint32_t v, double* p,
                                        unsigned long long& key) {
  double4 t = pts[v];
  p[0] = t.x;
  p[1] = t.y;
  p[2] = t.z;
  key = (unsigned long long)__double_as_longlong(t.w);
}

__device__ __forceinline__ uint32_t hash32(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7FEB352Du;
  x ^= x >> 15;
  x *= 0x846CA68Bu;
  x ^= x >> 16;
  return x;
}

// Fixed random priority of a point (20 bits): the insertion order follows
// it, as in randomised incremental construction, and points become active
// in levels of growing priority threshold.
__device__ __forceinline__ uint32_t prio_of(uint32_t p) {
  return hash32(p * 0x9E3779B9u + 0x632BE5ABu) >> 12;
}

// Candidate key of the cavity and shell claims: newer rounds compare
// smaller (12-bit round stamp, so stale claims never win; those claim words
// are reset every 4096 rounds), then the priority, then the point index
// (unique).
__device__ __forceinline__ unsigned long long make_key(uint32_t round, uint32_t p) {
  return ((unsigned long long)((~round) & 0xFFFu) << 52) |
         ((unsigned long long)prio_of(p) << 32) | (unsigned long long)p;
}

// Bid of a point for the cell it lies in (no round stamp: a bid on a live
// cell stays valid, since the cell dies as soon as its bidder is inserted
// or moves on); ordered like the candidate keys of one round.
__device__ __forceinline__ unsigned long long bid_key(uint32_t p) {
  return ((unsigned long long)prio_of(p) << 32) | (unsigned long long)p;
}

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// One slot per lane that asks for one; a single atomic per wave.
__device__ __forceinline__ uint32_t wave_alloc(bool want, uint32_t* ctr) {
  unsigned long long m = __ballot(want);
  if (m == 0) return 0xFFFFFFFFu;
  int leader = __ffsll((long long)m) - 1;
  uint32_t base = 0;
  if ((int)lane_id() == leader) base = atomicAdd(ctr, (uint32_t)__popcll(m));
  base = __shfl(base, leader);
  uint32_t below = (uint32_t)__popcll(m & ((1ull << lane_id()) - 1ull));
  return want ? base + below : 0xFFFFFFFFu;
}

// n slots per lane (n may be 0); a single atomic per wave.
__device__ __forceinline__ uint32_t wave_alloc_n(uint32_t n, uint32_t* ctr) {
  uint32_t lane = lane_id();
  uint32_t x = n;
  for (int off = 1; off < warpSize; off <<= 1) {
    uint32_t y = __shfl_up(x, off);
    if ((int)lane >= off) x += y;
  }
  uint32_t total = __shfl(x, warpSize - 1);
  uint32_t base = 0;
  if ((int)lane == warpSize - 1 && total) base = atomicAdd(ctr, total);
  base = __shfl(base, warpSize - 1);
  return base + x - n;
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
  for (int off = warpSize / 2; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// Predicate counters, flushed once per wave at kernel end.
template <int D>
__device__ __forceinline__ void flush_pred(Stripes* sx, const PredStats& s) {
  const int io = (D == 2) ? 0 : 1, ii = (D == 2) ? 2 : 3;
  uint32_t v[6] = {s.calls[0], s.f32ok[0], s.exact[0], s.calls[1], s.f32ok[1], s.exact[1]};
#pragma unroll
  for (int j = 0; j < 6; j++) v[j] = wave_sum(v[j]);
  if (lane_id() == 0) {
    unsigned long long* st = sx->pred[blockIdx.x % NSTRIPE];
    if (v[0]) {
      atomicAdd(&st[io * 4 + 0], (unsigned long long)v[0]);
      atomicAdd(&st[io * 4 + 1], (unsigned long long)v[1]);
      atomicAdd(&st[io * 4 + 2], (unsigned long long)(v[0] - v[1] - v[2]));
      atomicAdd(&st[io * 4 + 3], (unsigned long long)v[2]);
    }
    if (v[3]) {
      atomicAdd(&st[ii * 4 + 0], (unsigned long long)v[3]);
      atomicAdd(&st[ii * 4 + 1], (unsigned long long)v[4]);
      atomicAdd(&st[ii * 4 + 2], (unsigned long long)(v[3] - v[4] - v[5]));
      atomicAdd(&st[ii * 4 + 3], (unsigned long long)v[5]);
    }
  }
}

// ------------------------------------------------------------ conflict
// q lies in the hyperplane of a hull facet: decide with the facet's own
// (D-1)-dimensional circumsphere under the same perturbed lifting.  With an
// auxiliary point e off the hyperplane, the sphere through the facet and e
// meets the hyperplane exactly in the facet's circumsphere, so q is inside
// it iff In_pert(facet, e, q) has the sign of Orient1(facet, e); e carries
// no perturbation and the answer does not depend on which e is used.
template <int D, bool F32>
__device__ __noinline__ int conflict_coplanar(const double4* pts, uint32_t* flags, uint4 v,
                                              int inf, uint32_t q) {
  PredT<F32> pr;
  pr.init(flags);
  PtsX X;
  double F[3][3];
  unsigned long long fk[3];
  int nf = 0;
#pragma unroll
  for (int i = 0; i <= D; i++)
    if (i != inf) {
      load_pt(pts, vat(v, i), F[nf], fk[nf]);
      nf++;
    }
  int axis = 0;
  if (D == 2) {
    axis = (F[0][1] != F[1][1]) ? 0 : 1;
  } else {
    axis = -1;
    for (int ax = 0; ax < 3 && axis < 0; ax++) {
      PtsX Y;
      for (int j = 0; j < 3; j++) {
        int t = 0;
        for (int k = 0; k < 3; k++)
          if (k != ax) Y.p[j][t++] = F[j][k];
        Y.p[j][2] = 0.0;
      }
      if (pr.template orient<2>(Y) != 0) axis = ax;
    }
    if (axis < 0) return 0;
  }
  double e[3] = {F[0][0], F[0][1], D == 3 ? F[0][2] : 0.0};
  double a0 = F[0][axis];
  e[axis] = (a0 == 0.0) ? 1.0 : (fabs(a0) < 1e300 ? 2.0 * a0 : 0.5 * a0);
  int t = 0;
  for (int i = 0; i <= D; i++) {
    if (i == inf) {
      X.p[i][0] = e[0]; X.p[i][1] = e[1]; X.p[i][2] = e[2];
      X.key[i] = NOKEY;
    } else {
      X.p[i][0] = F[t][0]; X.p[i][1] = F[t][1]; X.p[i][2] = F[t][2];
      X.key[i] = fk[t];
      t++;
    }
  }
  int oe = pr.template orient<D>(X);
  load_pt(pts, q, X.p[D + 1], X.key[D + 1]);
  int s = pr.template insphere<D>(X);
  return (s != 0 && s == oe) ? 1 : 0;
}

// Is point q (coordinates qp, key qk) in conflict with the cell with
// vertices v?
template <int D, bool F32>
__device__ __forceinline__ bool conflict(const K4Args& a, PredT<F32>& pr, uint4 v, uint32_t q,
                                         const double* qp, unsigned long long qk) {
  int inf = -1;
#pragma unroll
  for (int i = 0; i <= D; i++)
    if (vat(v, i) == INF_V) inf = i;
  PtsX X;
  if (inf < 0) {
#pragma unroll
    for (int i = 0; i <= D; i++) load_pt(a.pts, vat(v, i), X.p[i], X.key[i]);
    X.p[D + 1][0] = qp[0]; X.p[D + 1][1] = qp[1]; X.p[D + 1][2] = qp[2];
    X.key[D + 1] = qk;
    return pr.template insphere<D>(X) > 0;
  }
#pragma unroll
  for (int i = 0; i <= D; i++) {
    if (i == inf) {
      X.p[i][0] = qp[0]; X.p[i][1] = qp[1]; X.p[i][2] = qp[2];
      X.key[i] = qk;
    } else {
      load_pt(a.pts, vat(v, i), X.p[i], X.key[i]);
    }
  }
  int o = pr.template orient<D>(X);
  if (o != 0) return o > 0;
  return conflict_coplanar<D, F32>(a.pts, &a.ctr->flags, v, inf, q) != 0;
}

// Visibility walk from cell c to a cell in conflict with q: inside a
// finite cell (closed), or a hull cell whose facet q sees.
template <int D, bool F32>
__device__ uint32_t walk(const K4Args& a, PredT<F32>& pr, uint32_t c, uint32_t q, const double* qp,
                         unsigned long long qk) {
  for (int step = 0; step < (1 << 16); step++) {
    if (c >= a.cap) break;
    // vertices and neighbours together: the next step needs no further load
    const uint4 v = a.cells[c].v, nb = a.cells[c].n;
    int inf = -1;
    bool bad = false;
#pragma unroll
    for (int i = 0; i <= D; i++) {
      uint32_t w = vat(v, i);
      if (w == INF_V) inf = i;
      else if (w >= a.npts) bad = true;
    }
    if (bad) break;
    if (inf >= 0) {
      if (conflict<D, F32>(a, pr, v, q, qp, qk)) return c;
      c = vat(nb, inf) >> 2;
      continue;
    }
    PtsX X;
    double P[D + 1][3];
    unsigned long long kk;
#pragma unroll
    for (int j = 0; j <= D; j++) load_pt(a.pts, vat(v, j), P[j], kk);
    int exitf = -1;
#pragma unroll
    for (int i = 0; i <= D; i++) {
      if (exitf >= 0) break;
#pragma unroll
      for (int j = 0; j <= D; j++) {
        const double* s = (j == i) ? qp : P[j];
        X.p[j][0] = s[0]; X.p[j][1] = s[1]; X.p[j][2] = s[2];
      }
      if (pr.template orient<D>(X) < 0) exitf = i;
    }
    if (exitf < 0) return c;
    c = vat(nb, exitf) >> 2;
  }
  atomicOr(&a.ctr->flags, FAIL_WALK);
  return 0;
}

// ------------------------------------------------------------ set setup
// One thread per set: the first D+1 affinely independent points (in index
// order) form the initial cell, plus one hull cell per facet.
template <int D>
__global__ void k4_init_sets(K4Args a, const uint32_t* seeded0) {
  uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= a.nsets) return;
  // a set started from a seed (its first cell given)
  if (seeded0 && seeded0[s] != DONE) {
    a.set_cell0[s] = seeded0[s];
    return;
  }
  PredT<false> pr;
  pr.init(&a.ctr->flags);
  uint32_t lo = a.set_off[s], hi = a.set_off[s + 1];
  uint32_t iv[4] = {0, 0, 0, NOSLOT};
  int ni = 0;
  double P[4][3];
  unsigned long long K[4];
  if (hi - lo >= (uint32_t)(D + 1)) {
    iv[0] = lo;
    load_pt(a.pts, lo, P[0], K[0]);
    ni = 1;
    for (uint32_t p = lo + 1; p < hi && ni < D + 1; p++) {
      double c[3];
      unsigned long long kc;
      load_pt(a.pts, p, c, kc);
      bool ok = false;
      if (ni == 1) {
        ok = true;
      } else if (ni == 2 && D == 3) {
        for (int ax = 0; ax < 3 && !ok; ax++) {
          PtsX Y;
          const double* src[3] = {P[0], P[1], c};
          for (int j = 0; j < 3; j++) {
            int t = 0;
            for (int k = 0; k < 3; k++)
              if (k != ax) Y.p[j][t++] = src[j][k];
            Y.p[j][2] = 0.0;
          }
          ok = pr.template orient<2>(Y) != 0;
        }
      } else {
        PtsX Y;
        for (int j = 0; j < ni; j++)
          for (int k = 0; k < 3; k++) Y.p[j][k] = P[j][k];
        for (int k = 0; k < 3; k++) Y.p[ni][k] = c[k];
        ok = pr.template orient<D>(Y) != 0;
      }
      if (ok) {
        iv[ni] = p;
        for (int k = 0; k < 3; k++) P[ni][k] = c[k];
        K[ni] = kc;
        ni++;
      }
    }
  }
  if (ni < D + 1) {
    a.set_cell0[s] = DONE;
    return;
  }
  {
    PtsX Y;
    for (int j = 0; j <= D; j++)
      for (int k = 0; k < 3; k++) Y.p[j][k] = P[j][k];
    if (pr.template orient<D>(Y) < 0) {
      uint32_t t = iv[0]; iv[0] = iv[1]; iv[1] = t;
    }
  }
  uint32_t base = atomicAdd(&a.ctr->cells, (uint32_t)(D + 2));
  if (base + D + 2 > a.cap) {
    atomicOr(&a.ctr->flags, FAIL_CELL_POOL);
    a.set_cell0[s] = DONE;
    return;
  }
  uint4 cells[5];
  cells[0] = make_uint4(iv[0], iv[1], iv[2], D == 3 ? iv[3] : NOSLOT);
  for (int i = 0; i <= D; i++) {
    uint4 w = cells[0];
    vset(w, i, INF_V);
    int x = (i == 0) ? 1 : 0, y = (i <= 1) ? 2 : 1;   // two finite slots
    uint32_t t = vat(w, x);
    vset(w, x, vat(w, y));
    vset(w, y, t);
    cells[i + 1] = w;
  }
  // adjacency by facet matching among the D+2 cells
  for (int x = 0; x < D + 2; x++) {
    uint4 nb = make_uint4(0, 0, 0, 0);
    for (int sl = 0; sl <= D; sl++) {
      for (int y = 0; y < D + 2; y++) {
        if (y == x) continue;
        int shared = 0, other = -1;
        for (int r = 0; r <= D; r++) {
          uint32_t vy = vat(cells[y], r);
          bool in = false;
          for (int l = 0; l <= D; l++)
            if (l != sl && vat(cells[x], l) == vy) in = true;
          if (in) shared++;
          else other = r;
        }
        if (shared == D) vset(nb, sl, ((base + y) << 2) | (uint32_t)other);
      }
    }
    if (D == 2) nb.w = NOSLOT;
    init_cell(a, base + x, cells[x]);
    a.cells[base + x].n = nb;
  }
  for (int j = 0; j <= D; j++) {
    a.ploc[iv[j]] = DONE;
    a.vcell[iv[j]] = base;
  }
  a.set_cell0[s] = base;
}

// One thread per point: every point starts in the initial cell of its set;
// it is located (walked) only when it becomes active.
__global__ void k4_place_init(K4Args a) {
  uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  bool act = false;
  if (p < a.npts) {
    uint32_t c0 = a.set_cell0[a.pset[p]];
    if (c0 == DONE) {
      a.ploc[p] = DONE;
    } else if (a.ploc[p] != DONE) {
      a.ploc[p] = c0 | NEEDWALK;   // a start cell, not yet a location
      act = true;
    }
  }
  uint32_t c = wave_sum(act ? 1u : 0u);
  if (lane_id() == 0 && c) atomicAdd(&a.ctr->active, c);
}

// Active list: the points not yet inserted whose priority is below the
// threshold (rebuilt when the threshold grows or the list thins out; the
// round's control step decides).  Grid-stride, whole waves per step.
__global__ void k4_build_active(K4Args a) {
  if (!a.ctr->rebuild || a.ctr->skip) return;
  const uint32_t thresh = a.ctr->thresh;
  // a contiguous chunk per block: count, one allocation, then write in order
  const uint32_t chunk = ((a.npts + gridDim.x - 1) / gridDim.x + BLOCK - 1) / BLOCK * BLOCK;
  const uint32_t lo = blockIdx.x * chunk;
  const uint32_t hi = min(a.npts, lo + chunk);
  uint32_t mine = 0;
  for (uint32_t p = lo + threadIdx.x; p < hi; p += BLOCK)
    mine += (a.ploc[p] != DONE && prio_of(p) < thresh) ? 1u : 0u;
  __shared__ uint32_t s_base;
  uint32_t tot;
  block_exclusive<BLOCK>(mine, &tot);
  if (threadIdx.x == 0) s_base = tot ? atomicAdd(&a.ctr->nact, tot) : 0u;
  __syncthreads();
  uint32_t run = s_base;
  for (uint32_t b = lo; b < hi; b += BLOCK) {
    const uint32_t p = b + threadIdx.x;
    const bool take = p < hi && a.ploc[p] != DONE && prio_of(p) < thresh;
    const uint32_t pre = block_exclusive<BLOCK>(take ? 1u : 0u, &tot);
    if (take) a.act[run + pre] = p;
    run += tot;
  }
}

// Round control (one thread).  Initial state: every located point is
// pending, the first level's threshold is thresh0.
__global__ void k4_ctl_init(K4Args a, uint32_t thresh0) {
  Counters* c = a.ctr;
  c->remaining = c->active;
  c->done = 0;
  c->ins_since = 0;
  c->thresh = thresh0;
  c->stall = 0;
  c->rounds = 0;
  c->skip = (c->active == 0 || c->flags) ? 1u : 0u;
  c->ncand = c->inserted = c->overflow = c->extused = c->pending = 0;
  for (uint32_t i = 0; i < NSTRIPE; i++) a.sx->pend[i] = a.sx->ins[i] = 0;
  c->rebuild = 1;
  c->nact = 0;
  c->built_thresh = thresh0;
  c->giant_req = NOKEY;
  c->giant_owner = DONE;
  c->giant_need = 0;
  c->giant_rounds = 0;
}

// Continue after the host has allocated the pool-sized cavity list.
__global__ void k4_resume(K4Args a) {
  Counters* c = a.ctr;
  c->giant_need = 0;
  c->stall = 0;
  c->skip = (c->remaining == 0 || c->flags) ? 1u : 0u;
}

// End of a round: account the insertions, move to the next level when
// fewer points are pending than 1/grow_div of those inserted, detect a
// stall, then prepare the next round (counters, active-list rebuild).
__global__ void k4_ctl_end(K4Args a) {
  Counters* c = a.ctr;
  if (c->skip) return;
  const uint32_t PMAX = 1u << 20;
  uint32_t pending = 0, ins = 0;
  for (uint32_t i = 0; i < NSTRIPE; i++) {
    pending += a.sx->pend[i];
    ins += a.sx->ins[i];
    a.sx->pend[i] = 0;
    a.sx->ins[i] = 0;
  }
  c->inserted = ins;
  c->pending = pending;
  c->rounds++;
  c->cand_total += c->ncand;
  c->last_ins = ins;
  c->last_cand = c->ncand;
  c->remaining -= ins;
  c->done += ins;
  c->ins_since += ins;
  const unsigned long long left = c->pending >= ins ? c->pending - ins : 0;
  const unsigned long long lim = c->done / a.grow_div;
  if (c->thresh < PMAX && left < (lim > 256 ? lim : 256)) {
    unsigned long long nt = (unsigned long long)c->thresh * a.grow_num / 8;
    if (nt <= c->thresh) nt = c->thresh + 1;
    c->thresh = nt > PMAX ? PMAX : (uint32_t)nt;
  } else if (ins == 0) {
    if (++c->stall > 8) c->flags |= FAIL_NO_PROGRESS;
  }
  if (ins) c->stall = 0;
  // the smallest candidate whose cavity outgrew its list gets the
  // pool-sized list next round; if that list does not exist yet, pause
  // (skip) until the host has allocated it
  c->giant_owner = c->giant_req != NOKEY ? (uint32_t)(c->giant_req & 0xFFFFFFFFull) : DONE;
  c->giant_req = NOKEY;
  if (c->giant_owner != DONE) c->giant_rounds++;
  if (c->giant_owner != DONE && a.gcap == 0) {
    c->giant_need = 1;
    c->stall = 0;
    c->skip = 1;
  }
  if (c->remaining == 0 || c->flags) c->skip = 1;
  c->ncand = c->inserted = c->overflow = c->extused = c->pending = 0;
  if (c->thresh != c->built_thresh || c->ins_since * 2 > c->nact) {
    c->rebuild = 1;
    c->nact = 0;
    c->built_thresh = c->thresh;
    c->ins_since = 0;
  } else {
    c->rebuild = 0;
  }
}

// ------------------------------------------------------------ rounds
// Active points whose cell was destroyed follow the forward pointers of
// destroyed cells (each points into the star that replaced it) to a live
// cell near them and walk from there; then every active point bids for its
// cell.  Dormant points are not touched.
template <int D, bool F32>
__global__ void k4_pick(K4Args a) {
  if (a.ctr->skip) return;
  const uint32_t nact = a.ctr->nact, thresh = a.ctr->thresh;
  PredT<F32> pr;
  pr.init(&a.ctr->flags);
  uint32_t npend = 0;
  for (uint32_t ia = blockIdx.x * blockDim.x + threadIdx.x; ia < nact;
       ia += gridDim.x * blockDim.x) {
    const uint32_t p = a.act[ia];
    const uint32_t raw = a.ploc[p];
    if (raw != DONE && prio_of(p) < thresh) {
      npend++;
      const bool need = (raw & NEEDWALK) != 0;
      bool bid = (raw & BIDDED) != 0;
      uint32_t L = raw & LOCMASK;
      if (need) {
        // First location of a newly active point: start at a cell of an
        // inserted point next to it in the (spatially sorted) point order
        // instead of the set's first cell, whose forward pointers lead far.
        const uint32_t s = a.pset[p], lo = a.set_off[s], hi = a.set_off[s + 1];
        uint32_t nb[2 * NEAR_WIN];
#pragma unroll
        for (uint32_t d = 1; d <= NEAR_WIN; d++) {
          nb[2 * d - 2] = p >= lo + d ? a.ploc[p - d] : 0u;
          nb[2 * d - 1] = p + d < hi ? a.ploc[p + d] : 0u;
        }
        uint32_t q = DONE;
#pragma unroll
        for (uint32_t j = 0; j < 2 * NEAR_WIN; j++)
          if (q == DONE && nb[j] == DONE) q = (j & 1u) ? p + (j / 2 + 1) : p - (j / 2 + 1);
        if (q != DONE) L = a.vcell[q];
      }
      if (need || a.cells[L].fwd != ALIVE) {
        for (int h = 0; h < (1 << 16); h++) {
          uint32_t f = a.cells[L].fwd;
          if (f == ALIVE) break;
          L = f;
        }
        double qp[3];
        unsigned long long qk;
        load_pt(a.pts, p, qp, qk);
        L = walk<D, F32>(a, pr, L, p, qp, qk);
        bid = false;
      }
      if (!bid) {
        atomicMin(&a.bid[L], bid_key(p));
        a.ploc[p] = L | BIDDED;
      }
    }
  }
  uint32_t c = wave_sum(npend);
  if (lane_id() == 0 && c) atomicAdd(&a.sx->pend[blockIdx.x % NSTRIPE], c);
  flush_pred<D>(a.sx, pr.st);
}

// Candidate selection (one thread per active point): a located point
// whose bid won its cell becomes a candidate unless a neighbouring cell
// holds a smaller bid -- that bidder's cavity holds its own cell, which
// touches this point's cell, so it would always win against this one.
template <int D>
__global__ void k4_select(K4Args a) {
  if (a.ctr->skip) return;
  const uint32_t nact = a.ctr->nact, thresh = a.ctr->thresh;
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t base = blockIdx.x * blockDim.x; base < nact; base += stride) {
  const uint32_t ia = base + threadIdx.x;
  bool want = false;
  uint32_t p = 0;
  if (ia < nact) {
    p = a.act[ia];
    const uint32_t raw = a.ploc[p];
    if (raw != DONE && (raw & NEEDWALK) == 0 && prio_of(p) < thresh) {
      const uint32_t L = raw & LOCMASK;
      const unsigned long long K = bid_key(p);
      want = (a.bid[L] == K);
      if (want && a.rings > 0) {
        // Each ring's loads are issued together (one dependent step for the
        // links, one for the bids): a link that leads back is redirected to
        // a cell of an inner ring, whose bid is known not to be smaller, so
        // no load waits on a branch.
        const uint4 nb = a.cells[L].n;
        uint32_t c1[D + 1];
#pragma unroll
        for (int i = 0; i <= D; i++) c1[i] = vat(nb, i);
        unsigned long long m = NOKEY;
#pragma unroll
        for (int i = 0; i <= D; i++) m = min(m, a.bid[c1[i] >> 2]);
        if (m < K) want = false;
        // Second and third rings: a smaller bid two or three cells away
        // almost always claims a cell next to this cavity.  Skipping such
        // candidates now (they would lose) saves their searches; the
        // smallest bid of all is never skipped, so every round still
        // inserts a point.
        // (a link's low two bits are the index of the facet leading back)
        if (want && a.rings > 1) {
          uint4 n2[D + 1];
#pragma unroll
          for (int i = 0; i <= D; i++) n2[i] = a.cells[c1[i] >> 2].n;
          uint32_t c2[D + 1][D + 1];
#pragma unroll
          for (int i = 0; i <= D; i++)
#pragma unroll
            for (int j = 0; j <= D; j++)
              c2[i][j] = (j == (int)(c1[i] & 3u)) ? c1[i] : vat(n2[i], j);
          m = NOKEY;
#pragma unroll
          for (int i = 0; i <= D; i++)
#pragma unroll
            for (int j = 0; j <= D; j++) m = min(m, a.bid[c2[i][j] >> 2]);
          if (m < K) want = false;
          if (want && a.rings > 2) {
            m = NOKEY;
#pragma unroll
            for (int i = 0; i <= D; i++) {
              uint4 n3[D + 1];
#pragma unroll
              for (int j = 0; j <= D; j++) n3[j] = a.cells[c2[i][j] >> 2].n;
#pragma unroll
              for (int j = 0; j <= D; j++)
#pragma unroll
                for (int l = 0; l <= D; l++) {
                  const uint32_t x =
                      (l == (int)(c2[i][j] & 3u)) ? c2[i][j] : vat(n3[j], l);
                  m = min(m, a.bid[x >> 2]);
                }
            }
            if (m < K) want = false;
          }
        }
      }
    }
  }
  // one allocation per block and iteration
  __shared__ uint32_t s_base;
  uint32_t tot;
  const uint32_t pre = block_exclusive<BLOCK>(want ? 1u : 0u, &tot);
  if (threadIdx.x == 0) s_base = tot ? atomicAdd(&a.ctr->ncand, tot) : 0u;
  __syncthreads();
  const uint32_t slot = s_base + pre;
  __syncthreads();
  if (want && slot < a.maxcand) {
    a.cand_pt[slot] = p;
    // Claim the candidate's own cell now: it lies in the candidate's
    // cavity whatever else does, so any larger candidate whose search
    // reaches it loses (it would fail verification anyway) and can stop
    // at once instead of finishing its search.
    atomicMin(&a.cells[a.ploc[p] & LOCMASK].cav, make_key(a.round, p));
  }
  }
}

// Cavity search: four candidates per wavefront, sixteen lanes each, in
// lockstep levels.  Each candidate runs a level-synchronous breadth-first
// search over its conflict region, the lanes of its group testing the
// neighbours of the current frontier in parallel; the four groups' memory
// accesses overlap, which is what bounds this search (a few dependent
// gathers per level).  Each cell found in conflict is claimed with the
// candidate's key (atomic minimum; the previous value also detects a cell
// found twice); each neighbour found not in conflict gets a shell claim.
// A smaller claim anywhere means this candidate cannot win: its search
// stops.  All control state is per group in LDS; the barriers are outside
// every group-dependent branch.  Three waves per SIMD: the working set of
// the filters stays in registers (no spills), which pays more than a
// fourth wave.
constexpr uint32_t CAV_GROUPS = 4;
constexpr uint32_t CAV_LANES = 64 / CAV_GROUPS;
constexpr uint32_t CAV_STASH = 64;

template <int D, bool F32>
__global__ __launch_bounds__(64, 3) void k4_cavity(K4Args a) {
  constexpr uint32_t G = CAV_GROUPS, GL = CAV_LANES;
  constexpr uint32_t IDLE = 0, BUSY = 1, EXHAUSTED = 2;
  __shared__ uint32_t s_n[G], s_flo[G], s_fhi[G], s_abort[G], s_gave[G], s_ext[G], s_slot[G],
      s_state[G];
  // Links of recently found cavity cells, by cavity position modulo CAV_STASH
  // (tagged with the position): the next level reads a frontier cell's
  // neighbours here instead of from its list entry and cell record.
  __shared__ uint32_t s_tag[G][CAV_STASH];
  __shared__ uint4 s_lnk[G][CAV_STASH];
  PredT<F32> pr;
  pr.init(&a.ctr->flags);
  const uint32_t lane = threadIdx.x, g = lane / GL, gl = lane % GL;
  const uint32_t ncand = min(a.ctr->ncand, a.maxcand);
  const uint32_t stride = gridDim.x * G;
  uint32_t mx = 0, gave = 0;
  unsigned long long cells = 0;
  if (gl == 0) {
    s_slot[g] = blockIdx.x * G + g;
    s_state[g] = IDLE;
  }
  // candidate of this lane's group, as loaded by this lane
  uint32_t cur = 0xFFFFFFFFu, p = 0;
  unsigned long long K = 0, qk = 0;
  double qp[3] = {0.0, 0.0, 0.0};
  __syncthreads();
  for (;;) {
    // leaders start a candidate in every idle group
    if (gl == 0 && s_state[g] == IDLE) {
      const uint32_t slot = s_slot[g];
      if (slot >= ncand) {
        s_state[g] = EXHAUSTED;
      } else {
        const uint32_t q = a.cand_pt[slot];
        const unsigned long long Kq = make_key(a.round, q);
        const uint32_t L = a.ploc[q] & LOCMASK;
        const bool giant = a.gcap != 0 && q == a.ctr->giant_owner;
        a.cand_ext[slot] = giant ? GIANT : DONE;
        // the own cell was claimed at selection; a smaller claim means a
        // smaller candidate's cavity holds it already
        const bool ok = atomicMin(&a.cells[L].cav, Kq) >= Kq;
        if (ok) {
          if (giant) a.gcell[0] = L;
          else a.cav[(size_t)slot * a.cavcap] = L;
        }
        s_ext[g] = giant ? GIANT : DONE;
        s_abort[g] = ok ? 0u : 1u;
        s_gave[g] = 0;
        s_n[g] = ok ? 1u : 0u;
        s_flo[g] = 0;
        s_fhi[g] = ok ? 1u : 0u;
        s_state[g] = BUSY;
      }
    }
    __syncthreads();
    bool any = false;
#pragma unroll
    for (uint32_t h = 0; h < G; h++) any |= (s_state[h] == BUSY);
    if (!any) break;
    const bool busy = s_state[g] == BUSY;
    const uint32_t slot = s_slot[g];
    if (busy && slot != cur) {
      cur = slot;
      p = a.cand_pt[slot];
      K = make_key(a.round, p);
      load_pt(a.pts, p, qp, qk);
      for (uint32_t j = gl; j < CAV_STASH; j += GL) s_tag[g][j] = DONE;
    }
    // leaders make room for the level's appends
    if (gl == 0 && busy && !s_abort[g] && s_flo[g] < s_fhi[g] && s_ext[g] != GIANT) {
      const uint32_t items = (s_fhi[g] - s_flo[g]) * (D + 1);
      if (s_n[g] + items > a.cavcap) {
        if (s_n[g] + items > a.cavcap + EXTCAP) {
          s_abort[g] = 1;
          s_gave[g] = 1;
        } else if (s_ext[g] == DONE) {
          const uint32_t e = atomicAdd(&a.ctr->extused, 1u);
          if (e >= MAXEXT) {
            s_abort[g] = 1;
            s_gave[g] = 1;
          } else {
            s_ext[g] = e;
            a.cand_ext[slot] = e;
          }
        }
      }
      // a cavity too large for the regular list asks for the pool-sized
      // one (the smallest such candidate of the round gets it next round)
      if (s_gave[g]) atomicMin(&a.ctr->giant_req, bid_key(p));
    }
    __syncthreads();
    const uint32_t flo = s_flo[g], fhi = s_fhi[g];
    if (busy && !s_abort[g] && flo < fhi) {
      const bool giant = s_ext[g] == GIANT;
      uint32_t* la = giant ? a.gcell : a.cav + (size_t)slot * a.cavcap;
      const uint32_t lcap = giant ? a.gcap : a.cavcap;
      uint32_t* lb = (giant || s_ext[g] == DONE) ? nullptr
                                                 : a.extcell + (size_t)s_ext[g] * EXTCAP;
      const uint32_t items = (fhi - flo) * (D + 1);
      for (uint32_t it = gl; it < items; it += GL) {
        if (s_abort[g]) break;
        const uint32_t h = flo + it / (D + 1);
        const int i = (int)(it % (D + 1));
        const uint32_t si = h % CAV_STASH;
        uint32_t t;
        if (s_tag[g][si] == h) {
          t = vat(s_lnk[g][si], i) >> 2;
        } else {
          const uint32_t c = h < lcap ? la[h] : lb[h - lcap];
          t = vat(a.cells[c].n, i) >> 2;
        }
        if (t >= a.cap) {
          atomicOr(&a.ctr->flags, FAIL_INVARIANT);
          s_abort[g] = 1;
          break;
        }
        const uint4 tv = a.cells[t].v, tn = a.cells[t].n;
        bool badv = false;
#pragma unroll
        for (int r = 0; r <= D; r++)
          if (vat(tv, r) != INF_V && vat(tv, r) >= a.npts) badv = true;
        if (badv) {
          atomicOr(&a.ctr->flags, FAIL_INVARIANT);
          s_abort[g] = 1;
          break;
        }
        // both claims in one step (same cell record)
        const unsigned long long cc = __atomic_load_n(&a.cells[t].cav, __ATOMIC_RELAXED);
        const unsigned long long sh = __atomic_load_n(&a.cells[t].shell, __ATOMIC_RELAXED);
        if (cc == K) continue;
        if (cc < K) { s_abort[g] = 1; break; }
        if (sh == K) continue;
        if (conflict<D, F32>(a, pr, tv, p, qp, qk)) {
          // a cavity cell in a smaller candidate's shell fails verification
          if (sh < K) { s_abort[g] = 1; break; }
          const unsigned long long old = atomicMin(&a.cells[t].cav, K);
          if (old < K) { s_abort[g] = 1; break; }
          if (old == K) continue;
          const uint32_t pos = atomicAdd(&s_n[g], 1u);
          if (pos < lcap) {
            la[pos] = t;
          } else if (lb && pos - lcap < EXTCAP) {
            lb[pos - lcap] = t;
          } else {
            // only the pool-sized list can get here: more cavity cells
            // than cells in the pool
            atomicOr(&a.ctr->flags, FAIL_INVARIANT);
            s_abort[g] = 1;
            break;
          }
          // the slot's previous entry is from an earlier level (no reader
          // of this level can hold its tag)
          if (pos < flo + CAV_STASH) {
            s_tag[g][pos % CAV_STASH] = pos;
            s_lnk[g][pos % CAV_STASH] = tn;
          }
        } else {
          atomicMin(&a.cells[t].shell, K);
        }
      }
    }
    __syncthreads();
    // leaders advance to the next level, or finish the candidate
    if (gl == 0 && busy) {
      s_flo[g] = fhi;
      s_fhi[g] = s_n[g];
      if (s_abort[g] || s_flo[g] >= s_fhi[g]) {
        a.cand_n[slot] = s_abort[g] ? 0u : s_n[g];
        mx = max(mx, s_n[g]);
        cells += s_n[g];
        gave += s_gave[g];
        s_slot[g] = slot + stride;
        s_state[g] = IDLE;
      }
    }
    __syncthreads();
  }
  if (gl == 0) {
    if (gave) atomicAdd(&a.ctr->overflow, gave);
    if (mx) atomicMax(&a.sx->maxcav[blockIdx.x % NSTRIPE], mx);
    if (cells) atomicAdd(&a.sx->cavcells[blockIdx.x % NSTRIPE], cells);
  }
  flush_pred<D>(a.sx, pr.st);
}

// New cell index of boundary facet (cavity position h, facet f).
__device__ __forceinline__ uint32_t facet_cell(uint32_t info, int f, uint32_t base) {
  uint32_t mask = info & 0xFFu, pre = info >> 8;
  return base + pre + (uint32_t)__popc(mask & ((1u << f) - 1u));
}

// Verification and retriangulation, one wavefront per candidate.  A
// candidate wins if its cavity cells carry its cavity claim and no smaller
// shell claim, and no cell around the cavity carries a smaller cavity
// claim: then no other winner's cavity overlaps or touches its own, and
// it can replace its cavity by the cone of new cells from the point to the
// cavity boundary exactly as a sequential insertion would.  The lanes take
// the cavity cells; the new cell on a boundary facet links to its
// neighbours across the facets through the point by rotating around the
// shared ridge inside the cavity.
// Boundary facets listed in LDS for the facet-parallel build (a cavity
// with more falls back to one lane per cavity cell).
constexpr uint32_t FTAB = 1024;

// The new cell on boundary facet i of cavity cell c (cavity position of c
// encoded in inf): its vertices, and its neighbour across facet i, which
// gets the back link.
template <int D>
__device__ __forceinline__ void new_cell_outer(K4Args& a, uint32_t c, uint32_t inf,
                                               int i, uint32_t base, uint32_t p) {
  const uint32_t x = facet_cell(inf, i, base);
  uint4 nv = a.cells[c].v;
  vset(nv, i, p);
  init_cell(a, x, nv);
  const uint32_t out = vat(a.cells[c].n, i);
  *nslot(a.cells, x, i) = out;
  if (D == 2) *nslot(a.cells, x, 3) = NOSLOT;
  *nslot(a.cells, out >> 2, out & 3u) = (x << 2) | (uint32_t)i;
}

// Neighbour of the new cell on facet i of cavity cell c across its facet
// j (a facet through the new point): rotate around the ridge shared by
// facets i and j inside the cavity until leaving it; the boundary facet
// reached carries that neighbour.  Every step enters another cavity cell
// around the ridge, so a cavity of n cells is left within n steps (a
// thin input can put thousands of cells of one cavity around a ridge).
template <int D>
__device__ __forceinline__ uint32_t new_cell_link(K4Args& a, CavList& cl, uint32_t c, int i, int j,
                                                  uint32_t base, unsigned long long K,
                                                  uint32_t n) {
  uint32_t cur = c;
  int sin = i, sout = j;
  uint4 vcur = a.cells[c].v;
  for (uint32_t step = 0; step <= n; step++) {
    // each step: the current cell's link and position, then the next
    // cell's claim and vertices (each pair from one cell record)
    const uint32_t nbr = vat(a.cells[cur].n, sout);
    const uint32_t cpos = a.cells[cur].pos;
    const uint32_t ncell = nbr >> 2;
    if (ncell >= a.cap) break;
    const unsigned long long ncav = a.cells[ncell].cav;
    const uint4 vn = a.cells[ncell].v;
    if (ncav != K) {
      const uint32_t xp = facet_cell(cl.info(cpos), sout, base);
      return (xp << 2) | (uint32_t)sin;
    }
    const uint32_t av = vat(vcur, sin);
    int nout = 0;
#pragma unroll
    for (int r = 0; r <= D; r++)
      if (vat(vn, r) == av) nout = r;
    cur = ncell;
    sin = (int)(nbr & 3u);
    sout = nout;
    vcur = vn;
  }
  atomicOr(&a.ctr->flags, FAIL_PIVOT);
  return 0xFFFFFFFFu;
}

// Blocks of INS_WAVES wavefronts, one candidate per wavefront at a time:
// each wavefront verifies and numbers its candidate's boundary facets,
// then one thread takes the new cells of all the block's winners with a
// single atomic (a counter that every winner hit alone serialises the
// whole launch), then each wavefront builds its cells.  Eight waves per
// SIMD (at most 64 registers): its chains of dependent gathers gain more
// from the extra waves than they lose to a few spilled bytes (the step's
// insert 62.0 -> 58.5 ms on 4M clustered points; the selection and the
// walk lose at higher occupancy, their spills are larger).
constexpr uint32_t INS_WAVES = 8;

// Barrier of one wavefront (its lanes run in lockstep: only the memory
// ordering of a barrier is needed).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

template <int D>
__global__ __launch_bounds__(64 * INS_WAVES, 8) void k4_insert(K4Args a) {
  __shared__ uint32_t s_failw[INS_WAVES], s_runw[INS_WAVES], s_basew[INS_WAVES];
  __shared__ uint32_t s_ftabw[INS_WAVES][FTAB];   // boundary facet f: cavity position << 2 | facet
  __shared__ uint32_t s_poolfail;
  const uint32_t wv = threadIdx.x / 64, lane = threadIdx.x % 64;
  uint32_t& s_fail = s_failw[wv];
  uint32_t& s_run = s_runw[wv];
  uint32_t* s_ftab = s_ftabw[wv];
  const uint32_t ncand = min(a.ctr->ncand, a.maxcand);
  uint32_t won = 0;
  for (uint32_t first = blockIdx.x * INS_WAVES; first < ncand; first += gridDim.x * INS_WAVES) {
    const uint32_t slot = first + wv;
    const uint32_t n = slot < ncand ? a.cand_n[slot] : 0u;
    const uint32_t p = n ? a.cand_pt[slot] : 0u;
    const unsigned long long K = make_key(a.round, p);
    CavList cl{a.cav + (size_t)slot * a.cavcap, a.cavinfo + (size_t)slot * a.cavcap, nullptr,
               nullptr, a.cavcap};
    if (n) {
      const uint32_t e = a.cand_ext[slot];
      if (e == GIANT) {
        cl.a = a.gcell;
        cl.ia = a.ginfo;
        cl.cap = a.gcap;
      } else if (e != DONE) {
        cl.b = a.extcell + (size_t)e * EXTCAP;
        cl.ib = a.extinfo + (size_t)e * EXTCAP;
      }
    }
    if (lane == 0) {
      s_fail = n ? 0u : 1u;
      s_run = 0;
      if (n) atomicAdd(&a.sx->verified[(blockIdx.x * INS_WAVES + wv) % NSTRIPE], 1ull);
    }
    wave_sync();
    // boundary-facet mask of the lane's first cavity cell, kept for the
    // numbering below
    uint32_t mask0 = 0, c0 = 0;
    for (uint32_t h = lane; h < n; h += 64) {
      const uint32_t c = cl.cell(h);
      // the cell's claims and links in one step, the neighbours' claims in
      // the next
      const unsigned long long cv = a.cells[c].cav, sh = a.cells[c].shell;
      const uint4 nb = a.cells[c].n;
      bool oob = false;
#pragma unroll
      for (int i = 0; i <= D; i++) oob |= (vat(nb, i) >> 2) >= a.cap;
      if (oob) {
        atomicOr(&a.ctr->flags, FAIL_INVARIANT);
        s_fail = 1;
        continue;
      }
      unsigned long long m = NOKEY;
      uint32_t mk = 0;
#pragma unroll
      for (int i = 0; i <= D; i++) {
        const unsigned long long ci = a.cells[vat(nb, i) >> 2].cav;
        m = min(m, ci);
        if (ci != K) mk |= 1u << i;
      }
      if (cv != K || sh <= K || m < K) s_fail = 1;
      if (h == lane) {
        mask0 = mk;
        c0 = c;
      }
    }
    wave_sync();
    const bool win = s_fail == 0;
    // boundary facets of every cavity cell and their new cell numbers
    for (uint32_t start = 0; win && start < n; start += 64) {
      const uint32_t h = start + lane;
      uint32_t mask = 0;
      uint32_t c = 0;
      if (h < n && start == 0) {
        c = c0;
        mask = mask0;
      } else if (h < n) {
        c = cl.cell(h);
        const uint4 nb = a.cells[c].n;
#pragma unroll
        for (int i = 0; i <= D; i++)
          if (a.cells[vat(nb, i) >> 2].cav != K) mask |= 1u << i;
      }
      const uint32_t cnt = (uint32_t)__popc(mask);
      uint32_t incl = cnt;
      for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(incl, off, 64);
        if ((int)lane >= off) incl += y;
      }
      const uint32_t run = s_run;
      if (h < n) {
        const uint32_t pre = run + incl - cnt;
        cl.info(h) = (pre << 8) | mask;
        a.cells[c].pos = h;
        uint32_t f = pre;
#pragma unroll
        for (int i = 0; i <= D; i++)
          if ((mask >> i & 1u) && f < FTAB) s_ftab[f++] = (h << 2) | (uint32_t)i;
      }
      const uint32_t total = __shfl(incl, 63, 64);
      wave_sync();
      if (lane == 0) s_run = run + total;
      wave_sync();
    }
    // one allocation for the block's winners
    __syncthreads();
    if (threadIdx.x == 0) {
      uint32_t tot = 0;
      for (uint32_t w = 0; w < INS_WAVES; w++) {
        const uint32_t m = s_failw[w] ? 0u : s_runw[w];
        s_basew[w] = tot;
        tot += m;
      }
      const uint32_t b = tot ? atomicAdd(&a.ctr->cells, tot) : 0u;
      s_poolfail = 0;
      if ((uint64_t)b + tot > a.cap) {
        atomicOr(&a.ctr->flags, FAIL_CELL_POOL);
        s_poolfail = 1;
      }
      for (uint32_t w = 0; w < INS_WAVES; w++) s_basew[w] += b;
    }
    __syncthreads();
    if (win && !s_poolfail) {
    const uint32_t nbf = s_run;
    const uint32_t base = s_basew[wv];
    if (nbf <= FTAB) {
      // facet-parallel build: one task per (boundary facet, other facet of
      // the new cell); the numbering written by the other lanes is read here
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
      const uint32_t ntask = nbf * D;
      for (uint32_t t = lane; t < ntask; t += 64) {
        const uint32_t f = t / D, jj = t % D;
        const uint32_t hf = s_ftab[f];
        const uint32_t h = hf >> 2;
        const int i = (int)(hf & 3u);
        const int j = (int)jj < i ? (int)jj : (int)jj + 1;
        const uint32_t c = cl.cell(h);
        const uint32_t inf = cl.info(h);
        const uint32_t x = facet_cell(inf, i, base);
        if (jj == 0) new_cell_outer<D>(a, c, inf, i, base, p);
        uint32_t link = new_cell_link<D>(a, cl, c, i, j, base, K, n);
        if (link == 0xFFFFFFFFu) link = (x << 2) | (uint32_t)j;   // in-bounds; the run is abandoned
        *nslot(a.cells, x, j) = link;
      }
    } else {
    // large cavity: one lane per cavity cell builds all its new cells
    for (uint32_t h = lane; h < n; h += 64) {
      const uint32_t c = cl.cell(h);
      const uint32_t inf = cl.info(h);
      const uint32_t mask = inf & 0xFFu;
      if (!mask) continue;
      const uint4 vc = a.cells[c].v;
      const uint4 nc = a.cells[c].n;
#pragma unroll
      for (int i = 0; i <= D; i++) {
        if (!(mask >> i & 1u)) continue;
        const uint32_t x = facet_cell(inf, i, base);
        uint4 nv = vc;
        vset(nv, i, p);
        uint4 nn = make_uint4(0, 0, 0, NOSLOT);
        const uint32_t out = vat(nc, i);
        vset(nn, i, out);
        *nslot(a.cells, out >> 2, out & 3u) = (x << 2) | (uint32_t)i;
#pragma unroll
        for (int j = 0; j <= D; j++) {
          if (j == i) continue;
          uint32_t cur = c;
          int sin = i, sout = j;
          uint4 vcur = vc;
          uint32_t link = 0xFFFFFFFFu;
          for (uint32_t step = 0; step <= n; step++) {
            const uint32_t nbr = vat(a.cells[cur].n, sout);
            const uint32_t ncell = nbr >> 2;
            if (ncell >= a.cap) break;
            if (a.cells[ncell].cav != K) {
              const uint32_t xp = facet_cell(cl.info(a.cells[cur].pos), sout, base);
              link = (xp << 2) | (uint32_t)sin;
              break;
            }
            const uint32_t av = vat(vcur, sin);
            const uint4 vn = a.cells[ncell].v;
            int nout = 0;
#pragma unroll
            for (int r = 0; r <= D; r++)
              if (vat(vn, r) == av) nout = r;
            cur = ncell;
            sin = (int)(nbr & 3u);
            sout = nout;
            vcur = vn;
          }
          if (link == 0xFFFFFFFFu) {
            atomicOr(&a.ctr->flags, FAIL_PIVOT);
            link = (x << 2) | (uint32_t)j;   // in-bounds placeholder; the run is abandoned
          }
          vset(nn, j, link);
        }
        init_cell(a, x, nv);
        a.cells[x].n = nn;
      }
    }
    }
    // destroyed cavity cells point into the star: to the new cell over one
    // of their own boundary facets when they have one (near the points
    // they held), else to the star's first cell
    for (uint32_t h = lane; h < n; h += 64) {
      const uint32_t inf = cl.info(h);
      const uint32_t mask = inf & 0xFFu;
      a.cells[cl.cell(h)].fwd = mask ? facet_cell(inf, __ffs(mask) - 1, base) : base;
    }
    if (lane == 0) {
      a.ploc[p] = DONE;
      a.vcell[p] = base;   // every cell of the star has p as a vertex
      won++;
    }
    }
    // the block's LDS is reused by the next candidates
    __syncthreads();
  }
  if (lane == 0 && won) atomicAdd(&a.sx->ins[(blockIdx.x * INS_WAVES + wv) % NSTRIPE], won);
}

// ------------------------------------------------------------ extraction
// Live finite cells, in cell order: a counting pass (per block of BLOCK
// cells, optionally also per set), a scan of the block counts, and a
// writing pass that puts each block's rows at its offset.
template <int D>
__device__ __forceinline__ bool finite_live_cell(const Cell* cells,
                                                 uint32_t ncells, uint32_t c, uint4& v) {
  v = make_uint4(0, 0, 0, 0);
  if (c >= ncells || cells[c].fwd != ALIVE) return false;
  v = cells[c].v;
#pragma unroll
  for (int i = 0; i <= D; i++)
    if (vat(v, i) == INF_V) return false;
  return true;
}

template <int D>
__global__ void k4_count_rows(const uint32_t* pset, const Cell* cells,
                              uint32_t ncells, uint32_t* bcnt, uint32_t* set_rows) {
  uint4 v;
  const bool take = finite_live_cell<D>(cells, ncells, blockIdx.x * BLOCK + threadIdx.x, v);
  if (take && set_rows) atomicAdd(&set_rows[pset[v.x]], 1u);
  uint32_t tot;
  block_exclusive<BLOCK>(take ? 1u : 0u, &tot);
  if (threadIdx.x == 0) bcnt[blockIdx.x] = tot;
}

template <int D>
__global__ void k4_write_rows(const double4* pts, const Cell* cells,
                              uint32_t ncells, const uint32_t* boff, int32_t* rows) {
  uint4 v;
  const bool take = finite_live_cell<D>(cells, ncells, blockIdx.x * BLOCK + threadIdx.x, v);
  uint32_t tot;
  const uint32_t pre = block_exclusive<BLOCK>(take ? 1u : 0u, &tot);
  if (!take) return;
  const size_t slot = (size_t)boff[blockIdx.x] + pre;
  int32_t k[4];
#pragma unroll
  for (int i = 0; i <= D; i++) k[i] = (int32_t)__double_as_longlong(pts[vat(v, i)].w);
#pragma unroll
  for (int i = 1; i <= D; i++)
#pragma unroll
    for (int j = i; j > 0; j--)
      if (k[j] < k[j - 1]) { int32_t t = k[j]; k[j] = k[j - 1]; k[j - 1] = t; }
#pragma unroll
  for (int i = 0; i <= D; i++) rows[slot * (D + 1) + i] = k[i];
}

// Clear the cavity and shell claims of the cells in use (the round stamp
// of the claim keys wraps every 4096 rounds).
__global__ void k4_reset_claims(Cell* cells, uint32_t used) {
  const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= used) return;
  cells[c].cav = NOKEY;
  cells[c].shell = NOKEY;
}

// ------------------------------------------------------------ seeded start
// A single large set starts from the Delaunay triangulation of its first
// points in priority order, built by gift wrapping (dt_gwrap.hip), instead
// of from one simplex.  Parallel insertion spends its first hundred-odd
// rounds on those points (while the triangulation has few cells, the
// cavities of the candidates overlap and a round inserts a point or two),
// each round a chain of dependent gathers.  The seed's simplices get their
// neighbour links by matching facets, and every hull facet gets a hull cell
// (the infinite vertex and the facet), linked to its neighbours across the
// hull's ridges, exactly as the insertion keeps them.  The seed points are
// then inserted; the rest continue in activation levels above them.
constexpr uint32_t SEED_POINTS = 4096;     // expected seed size
constexpr uint32_t SEED_MIN_SET = 65536;   // smaller single sets start from one simplex
constexpr uint32_t SEED_KEY_BITS = 21;     // facet keys: three seed-point indices of 21 bits

// The points below the priority threshold T, gathered.
__global__ void k_seed_pick(uint32_t npts, uint32_t T, const double4* pts, uint32_t* cnt,
                            uint32_t* sidx, double4* spts, uint32_t cap) {
  const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npts || prio_of(p) >= T) return;
  const uint32_t i = atomicAdd(cnt, 1u);
  if (i < cap) {
    sidx[i] = p;
    spts[i] = pts[p];
  }
}

// The wrapped simplices as cells of the pool (vertex indices of the job),
// their vertices inserted.
template <int D>
__global__ void k_seed_cells(const Cell* wc, uint32_t nf, const uint32_t* sidx, Cell* cells,
                             unsigned long long* bid, uint32_t* vcell, uint32_t* ploc) {
  const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nf) return;
  uint4 v = wc[c].v;
#pragma unroll
  for (int i = 0; i <= D; i++) vset(v, i, sidx[vat(v, i)]);
  if (D == 2) v.w = NOSLOT;
  Cell& x = cells[c];
  x.v = v;
  x.n = make_uint4(0u, 0u, 0u, D == 2 ? NOSLOT : 0u);
  x.spare = 0;
  x.cav = NOKEY;
  x.shell = NOKEY;
  x.fwd = ALIVE;
  x.pos = 0;
  bid[c] = NOKEY;
#pragma unroll
  for (int i = 0; i <= D; i++) {
    vcell[vat(v, i)] = c;
    ploc[vat(v, i)] = DONE;
  }
}

// Facet and ridge tables: a key and the (cell << 2 | slot) of the two cells
// that share it.
struct SeedTab {
  unsigned long long* key;
  uint32_t* e0;
  uint32_t* e1;
  uint32_t mask;
};

__device__ __forceinline__ void seed_tab_put(const SeedTab& t, unsigned long long key,
                                             uint32_t val, uint32_t* flags) {
  uint32_t h = (uint32_t)((key * 0x9E3779B97F4A7C15ull) >> 32);
  for (uint32_t pr = 0; pr <= t.mask; pr++) {
    const uint32_t s = (h + pr) & t.mask;
    const unsigned long long old = atomicCAS(&t.key[s], ~0ull, key);
    if (old == ~0ull) { t.e0[s] = val; return; }
    if (old == key) { t.e1[s] = val; return; }
  }
  atomicOr(flags, FAIL_HASH);
}

// Key of the facet of cell vertices v (indices into the seed's points)
// opposite slot i: the sorted finite indices (the infinite vertex is left
// out; hull ridges have their own table).
template <int D>
__device__ __forceinline__ unsigned long long seed_key(const uint4& v, int i) {
  uint32_t k[3] = {0u, 0u, 0u};
  int m = 0;
#pragma unroll
  for (int j = 0; j <= D; j++)
    if (j != i && vat(v, j) != INF_V) {
      if (m == 0) k[0] = vat(v, j);
      else if (m == 1) k[1] = vat(v, j);
      else k[2] = vat(v, j);
      m++;
    }
  if (m == 1) return (unsigned long long)k[0];
  if (k[1] < k[0]) { const uint32_t t = k[0]; k[0] = k[1]; k[1] = t; }
  if (m == 3) {
    if (k[2] < k[1]) { const uint32_t t = k[1]; k[1] = k[2]; k[2] = t; }
    if (k[1] < k[0]) { const uint32_t t = k[0]; k[0] = k[1]; k[1] = t; }
    return ((unsigned long long)k[0] << (2 * SEED_KEY_BITS)) |
           ((unsigned long long)k[1] << SEED_KEY_BITS) | (unsigned long long)k[2];
  }
  return ((unsigned long long)k[0] << 32) | (unsigned long long)k[1];
}

template <int D>
__global__ void k_seed_facets(const Cell* wc, uint32_t nf, SeedTab t, uint32_t* flags) {
  const uint32_t x = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t c = x / (D + 1), i = x % (D + 1);
  if (c >= nf) return;
  seed_tab_put(t, seed_key<D>(wc[c].v, (int)i), (c << 2) | i, flags);
}

// Twin facets link their cells; a facet without a twin is on the hull and
// gets a hull cell (the facet with the infinite vertex in slot i and two
// other slots swapped, as the first cells of a set are made), whose
// ridges go to the ridge table.
template <int D>
__global__ void k_seed_link(const Cell* wc, const uint32_t* sidx, Cell* cells, SeedTab t,
                            SeedTab r, uint32_t* ncells, uint32_t cap, unsigned long long* bid,
                            uint32_t* flags) {
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s > t.mask || t.key[s] == ~0ull) return;
  const uint32_t a = t.e0[s], b = t.e1[s];
  if (b != DONE) {
    *nslot(cells, a >> 2, a & 3u) = b;
    *nslot(cells, b >> 2, b & 3u) = a;
    return;
  }
  const uint32_t c = a >> 2, i = a & 3u;
  const uint32_t h = atomicAdd(ncells, 1u);
  if (h >= cap) {
    atomicOr(flags, FAIL_CELL_POOL);
    return;
  }
  // in seed indices (for the ridge keys), then in job indices
  uint4 w = wc[c].v;
  vset(w, (int)i, INF_V);
  const int x = (i == 0) ? 1 : 0, y = (i <= 1) ? 2 : 1;
  const uint32_t tv = vat(w, x);
  vset(w, x, vat(w, y));
  vset(w, y, tv);
  uint4 wj = w;
#pragma unroll
  for (int j = 0; j <= D; j++)
    if (vat(w, j) != INF_V) vset(wj, j, sidx[vat(w, j)]);
  if (D == 2) wj.w = NOSLOT;
  Cell& hc = cells[h];
  hc.v = wj;
  hc.n = make_uint4(0u, 0u, 0u, D == 2 ? NOSLOT : 0u);
  hc.spare = 0;
  hc.cav = NOKEY;
  hc.shell = NOKEY;
  hc.fwd = ALIVE;
  hc.pos = 0;
  bid[h] = NOKEY;
  *nslot(cells, h, i) = a;
  *nslot(cells, c, i) = (h << 2) | i;
#pragma unroll
  for (int j = 0; j <= D; j++)
    if (j != (int)i) seed_tab_put(r, seed_key<D>(w, j), (h << 2) | (uint32_t)j, flags);
}

// Hull cells that share a ridge link to each other.
__global__ void k_seed_ridges(Cell* cells, SeedTab r, uint32_t* flags) {
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s > r.mask || r.key[s] == ~0ull) return;
  const uint32_t a = r.e0[s], b = r.e1[s];
  if (b == DONE) {
    atomicOr(flags, FAIL_INVARIANT);
    return;
  }
  *nslot(cells, a >> 2, a & 3u) = b;
  *nslot(cells, b >> 2, b & 3u) = a;
}

static inline uint32_t nblk(uint32_t n);

// The wrapped simplices of the seed points sidx (their indices into the
// job's points) as cells of the pool, with their links and a hull cell on
// every hull facet.  DT_OK: *ncells cells made.
static int seed_link(const LocalJob& job, const K4Args& a, const DevBuf& sidx, CellPool& wp,
                     uint32_t* ncells, hipStream_t st);

// Build the seed of a single set into the pool and the point records
// (ploc, vcell).  DT_OK: *ncells cells made, *thresh the first activation
// threshold above the seed; DT_E_NOT_READY: not seeded (the caller starts
// from one simplex; nothing it uses was written).
static int seed_single_set(const LocalJob& job, const K4Args& a, uint32_t* ncells,
                           uint32_t* thresh, hipStream_t st) {
  const int D = job.D;
  const uint32_t npts = job.npts;
  const uint32_t PMAX = 1u << 20;
  const uint32_t T = (uint32_t)(((uint64_t)PMAX * SEED_POINTS) / npts);
  const uint32_t scap = GW_MAX_POINTS;
  DevBuf cnt, sidx, spts, flags;
  DT_TRY(cnt.alloc(16));
  DT_TRY(sidx.alloc((size_t)scap * 4));
  DT_TRY(spts.alloc((size_t)scap * sizeof(double4)));
  DT_TRY(flags.alloc(16));
  DT_HIP(hipMemsetAsync(cnt.p, 0, 4, st));
  DT_HIP(hipMemsetAsync(flags.p, 0, 4, st));
  hipLaunchKernelGGL(k_seed_pick, dim3(nblk(npts)), dim3(BLOCK), 0, st, npts, T, job.pts,
                     cnt.as<uint32_t>(), sidx.as<uint32_t>(), spts.as<double4>(), scap);
  DT_HIP(hipGetLastError());
  uint32_t m = 0;
  DT_HIP(hipMemcpyAsync(&m, cnt.p, 4, hipMemcpyDeviceToHost, st));
  DT_HIP(hipStreamSynchronize(st));
  if (m > scap || m < (uint32_t)D + 2) return DT_E_NOT_READY;
  CellPool wp;
  uint32_t levels = 0;
  const int g = gift_wrap(spts.as<double4>(), m, D, wp, &levels, st);
  if (g != DT_OK) return g;
  DT_TRY(seed_link(job, a, sidx, wp, ncells, st));
  const uint64_t t1 = (uint64_t)T + T / 2;
  *thresh = (uint32_t)(t1 > PMAX ? PMAX : t1);
  return DT_OK;
}

// Seeds for the sets of a batched run (the local triangulations of the
// divide, a batch of independent sets).  Every set of at least
// SEED_SET_MIN points starts from the triangulation of its points below a
// common priority threshold T, all sets gift-wrapped together; a set whose
// seed would be smaller than SEED_SET_MIN_SEED or larger than a wrapped
// set may be starts from one simplex as before.  The seeds' cells are made
// exactly as for a single set.  A facet search of the wrap is a chain of
// dependent loads and FP64 predicates (about 20 us), so the wrap's cost
// grows with the seeds' total: a set of average size gets
// SEED_SET_POINTS, and fewer when the seeds together would pass the total
// for the dimension (measured on 4M clustered 3D points: 1024 per set
// pays at k = 16 and 64; at k = 256, 256 seeds of 1024 cost more than they
// save, and 128 each about break even; 2D facet searches are cheaper: the
// 4096-set 2D batch runs 389.5 -> 380.9 ms with 805 sets seeded).
constexpr uint32_t SEED_SET_POINTS = 1024;
constexpr uint32_t SEED_TOTAL_3D = 32768;
constexpr uint32_t SEED_TOTAL_2D = 262144;
constexpr uint32_t SEED_SET_MIN = 8192;
constexpr uint32_t SEED_SET_MIN_SEED = 64;

// The points of each set below T (one block per set: a set's points are
// consecutive).
__global__ void k_seed_count(const uint32_t* set_off, uint32_t T, uint32_t* scnt) {
  const uint32_t s = blockIdx.x, lo = set_off[s], hi = set_off[s + 1];
  uint32_t c = 0;
  for (uint32_t p = lo + threadIdx.x; p < hi; p += blockDim.x) c += prio_of(p) < T ? 1u : 0u;
  uint32_t tot;
  block_exclusive<BLOCK>(c, &tot);
  if (threadIdx.x == 0) scnt[s] = tot;
}

// The seed points: below T in a set chosen for a seed.
__global__ void k_seed_flag(uint32_t npts, uint32_t T, const uint32_t* pset,
                            const uint32_t* smark, uint32_t* flag) {
  const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < npts) flag[p] = (prio_of(p) < T && smark[pset[p]]) ? 1u : 0u;
}

__global__ void k_seed_gather(const double4* pts, const uint32_t* sidx, uint32_t m,
                              double4* spts) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) spts[i] = pts[sidx[i]];
}

// Seed the sets of a batched run into the pool and the point records.
// DT_OK: *ncells cells made, seeded0[s] the first cell of every seeded set
// (DONE for the others, which start from one simplex), *thresh the first
// activation threshold above the seeds, *nseeded the sets seeded;
// DT_E_NOT_READY or DT_E_INTERNAL: not seeded (the caller clears the point
// records and starts every set from one simplex).
static int seed_sets(const LocalJob& job, const K4Args& a, DevBuf& seeded0, uint32_t* ncells,
                     uint32_t* thresh, uint32_t* nseeded, hipStream_t st) {
  const int D = job.D;
  const uint32_t npts = job.npts, ns = job.nsets;
  const uint32_t PMAX = 1u << 20;
  *nseeded = 0;
  std::vector<uint32_t> off(ns + 1);
  DT_HIP(hipMemcpyAsync(off.data(), job.set_off, (size_t)(ns + 1) * 4, hipMemcpyDeviceToHost,
                        st));
  DT_HIP(hipStreamSynchronize(st));
  uint32_t nmax = 0, nbig = 0;
  uint64_t pbig = 0;
  for (uint32_t i = 0; i < ns; i++) {
    const uint32_t n = off[i + 1] - off[i];
    nmax = std::max(nmax, n);
    if (n >= SEED_SET_MIN) {
      nbig++;
      pbig += n;
    }
  }
  if (nbig == 0) return DT_E_NOT_READY;
  // the seed of a set of average size among those seeded, at most 3/4 of
  // the wrap's limit in the largest
  const uint64_t per =
      std::min<uint64_t>(SEED_SET_POINTS, (D == 2 ? SEED_TOTAL_2D : SEED_TOTAL_3D) / nbig);
  uint64_t T = (uint64_t)PMAX * per * nbig / pbig;
  T = std::min<uint64_t>(T, (uint64_t)PMAX * (GW_MAX_SET_POINTS * 3 / 4) / nmax);
  if (T < 16) return DT_E_NOT_READY;
  DevBuf scnt, smark, flag, sidx, spts, soff;
  DT_TRY(scnt.alloc((size_t)ns * 4));
  hipLaunchKernelGGL(k_seed_count, dim3(ns), dim3(BLOCK), 0, st, job.set_off, (uint32_t)T,
                     scnt.as<uint32_t>());
  DT_HIP(hipGetLastError());
  std::vector<uint32_t> cnt(ns), mark(ns), so(ns + 1);
  DT_HIP(hipMemcpyAsync(cnt.data(), scnt.p, (size_t)ns * 4, hipMemcpyDeviceToHost, st));
  DT_HIP(hipStreamSynchronize(st));
  uint32_t m = 0, mmax = 0, nsd = 0;
  for (uint32_t i = 0; i < ns; i++) {
    mark[i] = (off[i + 1] - off[i] >= SEED_SET_MIN && cnt[i] >= SEED_SET_MIN_SEED &&
               cnt[i] <= GW_MAX_SET_POINTS) ? 1u : 0u;
    so[i] = m;
    if (mark[i]) {
      m += cnt[i];
      mmax = std::max(mmax, cnt[i]);
      nsd++;
    }
  }
  so[ns] = m;
  // seed indices share 21-bit fields in the facet keys
  if (nsd == 0 || m >= (1u << SEED_KEY_BITS)) return DT_E_NOT_READY;
  DT_TRY(smark.alloc((size_t)ns * 4));
  DT_TRY(soff.alloc((size_t)(ns + 1) * 4));
  DT_TRY(flag.alloc((size_t)npts * 4));
  DT_HIP(hipMemcpyAsync(smark.p, mark.data(), (size_t)ns * 4, hipMemcpyHostToDevice, st));
  DT_HIP(hipMemcpyAsync(soff.p, so.data(), (size_t)(ns + 1) * 4, hipMemcpyHostToDevice, st));
  hipLaunchKernelGGL(k_seed_flag, dim3(nblk(npts)), dim3(BLOCK), 0, st, npts, (uint32_t)T,
                     job.pset, smark.as<uint32_t>(), flag.as<uint32_t>());
  DT_HIP(hipGetLastError());
  uint32_t mc = 0;
  DT_TRY(compact_indices(flag.as<uint32_t>(), npts, sidx, &mc, st));
  if (mc != m) return DT_E_INTERNAL;
  DT_TRY(spts.alloc((size_t)m * sizeof(double4)));
  hipLaunchKernelGGL(k_seed_gather, dim3(nblk(m)), dim3(BLOCK), 0, st, job.pts,
                     sidx.as<uint32_t>(), m, spts.as<double4>());
  DT_HIP(hipGetLastError());
  CellPool wp;
  uint32_t levels = 0;
  const bool dbg = getenv("DT_DEBUG") != nullptr;
  // the first cell of every seeded set: its seed simplex (unseeded: DONE)
  DT_TRY(seeded0.alloc((size_t)ns * 4));
  DT_HIP(hipMemsetAsync(seeded0.p, 0xFF, (size_t)ns * 4, st));
  const int g = gift_wrap_sets(spts.as<double4>(), m, soff.as<uint32_t>(), ns, mmax, D, wp,
                               &levels, st, seeded0.as<uint32_t>());
  if (dbg)
    fprintf(stderr, "[seed] sets %u of %u, %u points (largest %u), T %llu: wrap %d, %u levels\n",
            nsd, ns, m, mmax, (unsigned long long)T, g, levels);
  if (g != DT_OK) return g;
  const int l = seed_link(job, a, sidx, wp, ncells, st);
  if (dbg && l != DT_OK) fprintf(stderr, "[seed] link %d\n", l);
  DT_TRY(l);
  const uint64_t t1 = T + T / 2;
  *thresh = (uint32_t)(t1 > PMAX ? PMAX : t1);
  *nseeded = nsd;
  return DT_OK;
}

static int seed_link(const LocalJob& job, const K4Args& a, const DevBuf& sidx, CellPool& wp,
                     uint32_t* ncells, hipStream_t st) {
  const int D = job.D;
  DevBuf flags;
  DT_TRY(flags.alloc(16));
  DT_HIP(hipMemsetAsync(flags.p, 0, 4, st));
  const uint32_t nf = wp.ncells;
  if (nf == 0 || (uint64_t)nf * 2 + 64 > a.cap) return DT_E_NOT_READY;
  // facets: (D+1) per cell, at most half of them twins
  uint32_t fsz = 64;
  while (fsz < 2u * (D + 1) * nf) fsz <<= 1;
  uint32_t rsz = 64;
  while (rsz < 2u * (D + 1) * nf) rsz <<= 1;
  DevBuf fk, f0, f1, rk, r0, r1, nc;
  DT_TRY(fk.alloc((size_t)fsz * 8));
  DT_TRY(f0.alloc((size_t)fsz * 4));
  DT_TRY(f1.alloc((size_t)fsz * 4));
  DT_TRY(rk.alloc((size_t)rsz * 8));
  DT_TRY(r0.alloc((size_t)rsz * 4));
  DT_TRY(r1.alloc((size_t)rsz * 4));
  DT_TRY(nc.alloc(16));
  DT_HIP(hipMemsetAsync(fk.p, 0xFF, (size_t)fsz * 8, st));
  DT_HIP(hipMemsetAsync(f1.p, 0xFF, (size_t)fsz * 4, st));
  DT_HIP(hipMemsetAsync(rk.p, 0xFF, (size_t)rsz * 8, st));
  DT_HIP(hipMemsetAsync(r1.p, 0xFF, (size_t)rsz * 4, st));
  DT_HIP(hipMemcpyAsync(nc.p, &nf, 4, hipMemcpyHostToDevice, st));
  const SeedTab ft{fk.as<unsigned long long>(), f0.as<uint32_t>(), f1.as<uint32_t>(), fsz - 1};
  const SeedTab rt{rk.as<unsigned long long>(), r0.as<uint32_t>(), r1.as<uint32_t>(), rsz - 1};
  if (D == 2) {
    hipLaunchKernelGGL(k_seed_cells<2>, dim3(nblk(nf)), dim3(BLOCK), 0, st, wp.cells.as<Cell>(),
                       nf, sidx.as<uint32_t>(), a.cells, a.bid, a.vcell, a.ploc);
    hipLaunchKernelGGL(k_seed_facets<2>, dim3(nblk(nf * 3)), dim3(BLOCK), 0, st,
                       wp.cells.as<Cell>(), nf, ft, flags.as<uint32_t>());
    hipLaunchKernelGGL(k_seed_link<2>, dim3(nblk(fsz)), dim3(BLOCK), 0, st, wp.cells.as<Cell>(),
                       sidx.as<uint32_t>(), a.cells, ft, rt, nc.as<uint32_t>(), a.cap, a.bid,
                       flags.as<uint32_t>());
  } else {
    hipLaunchKernelGGL(k_seed_cells<3>, dim3(nblk(nf)), dim3(BLOCK), 0, st, wp.cells.as<Cell>(),
                       nf, sidx.as<uint32_t>(), a.cells, a.bid, a.vcell, a.ploc);
    hipLaunchKernelGGL(k_seed_facets<3>, dim3(nblk(nf * 4)), dim3(BLOCK), 0, st,
                       wp.cells.as<Cell>(), nf, ft, flags.as<uint32_t>());
    hipLaunchKernelGGL(k_seed_link<3>, dim3(nblk(fsz)), dim3(BLOCK), 0, st, wp.cells.as<Cell>(),
                       sidx.as<uint32_t>(), a.cells, ft, rt, nc.as<uint32_t>(), a.cap, a.bid,
                       flags.as<uint32_t>());
  }
  hipLaunchKernelGGL(k_seed_ridges, dim3(nblk(rsz)), dim3(BLOCK), 0, st, a.cells, rt,
                     flags.as<uint32_t>());
  DT_HIP(hipGetLastError());
  uint32_t h[2] = {0, 0};
  DT_HIP(hipMemcpyAsync(&h[0], nc.p, 4, hipMemcpyDeviceToHost, st));
  DT_HIP(hipMemcpyAsync(&h[1], flags.p, 4, hipMemcpyDeviceToHost, st));
  DT_HIP(hipStreamSynchronize(st));
  if (h[1]) return DT_E_INTERNAL;
  *ncells = h[0];
  return DT_OK;
}

// ------------------------------------------------------------ host driver
static inline uint32_t nblk(uint32_t n) { return (n + BLOCK - 1) / BLOCK; }

int k4_run(const LocalJob& job, CellPool& pool, Counters* dctr, Counters* hctr, hipStream_t st,
           K4Stats& ks) {
  const int D = job.D;
  uint32_t npts = job.npts;
  // cell pool: every insertion appends one cell per boundary facet
  size_t cap = (size_t)npts * (D == 2 ? 12 : 40) + (size_t)job.nsets * 8 + 4096;
  if (cap > 0xF0000000ull / 1) cap = 0xF0000000ull;
  if (cap > (1ull << 30) - 1) cap = (1ull << 30) - 1;   // neighbour encoding uses 30 bits
  pool.cap = (uint32_t)cap;
  // every cell is written whole when it is created: no clearing needed
  DT_TRY(pool.cells.alloc(cap * sizeof(Cell)));
  DT_TRY(pool.set_cell0.alloc((size_t)job.nsets * sizeof(uint32_t)));

  uint32_t cavcap = (D == 2) ? 96 : 192;
  uint32_t maxcand = npts < (1u << 19) ? (npts ? npts : 1) : (1u << 19);
  DevBuf ploc, cand_pt, cand_n, cav, cavinfo, cand_ext, extcell, extinfo, actbuf, stripes;
  DT_TRY(stripes.alloc(sizeof(Stripes)));
  DT_HIP(hipMemsetAsync(stripes.p, 0, sizeof(Stripes), st));
  DT_TRY(actbuf.alloc((size_t)(npts ? npts : 1) * 4));
  DT_TRY(cand_ext.alloc((size_t)maxcand * 4));
  DT_TRY(extcell.alloc((size_t)MAXEXT * EXTCAP * 4));
  DT_TRY(extinfo.alloc((size_t)MAXEXT * EXTCAP * 4));
  DT_TRY(ploc.alloc((size_t)npts * 4));
  DevBuf vcell, bidbuf;
  DT_TRY(vcell.alloc((size_t)(npts ? npts : 1) * 4));
  DT_TRY(bidbuf.alloc((size_t)cap * 8));
  DT_TRY(cand_pt.alloc((size_t)maxcand * 4));
  DT_TRY(cand_n.alloc((size_t)maxcand * 4));
  DT_TRY(cav.alloc((size_t)maxcand * cavcap * 4));
  DT_TRY(cavinfo.alloc((size_t)maxcand * cavcap * 4));
  DT_HIP(hipMemsetAsync(ploc.p, 0, (size_t)npts * 4, st));
  DT_HIP(hipMemsetAsync(dctr, 0, sizeof(Counters), st));

  K4Args a;
  a.pts = job.pts;
  a.pset = job.pset;
  a.set_off = job.set_off;
  a.ploc = ploc.as<uint32_t>();
  a.cells = pool.cells.as<Cell>();
  a.set_cell0 = pool.set_cell0.as<uint32_t>();
  a.cand_pt = cand_pt.as<uint32_t>();
  a.cand_n = cand_n.as<uint32_t>();
  a.cav = cav.as<uint32_t>();
  a.cavinfo = cavinfo.as<uint32_t>();
  a.cand_ext = cand_ext.as<uint32_t>();
  a.extcell = extcell.as<uint32_t>();
  a.extinfo = extinfo.as<uint32_t>();
  a.ctr = dctr;
  a.sx = stripes.as<Stripes>();
  a.npts = npts;
  a.nsets = job.nsets;
  a.cap = pool.cap;
  a.maxcand = maxcand;
  a.cavcap = cavcap;
  a.round = 0;
  a.fp32 = job.fp32 ? 1 : 0;
  a.vcell = vcell.as<uint32_t>();
  a.bid = bidbuf.as<unsigned long long>();
  DevBuf gcell, ginfo;
  a.gcell = nullptr;
  a.ginfo = nullptr;
  a.gcap = 0;

  // a large single set, and every large set of a batched run, starts from
  // a gift-wrapped seed (see above)
  uint32_t seed_cells = 0, seed_thresh = 0;
  DevBuf seeded0;
  // (not inside a caller's workspace: the seed's scratch is not counted
  // in its size)
  if (job.nsets == 1 && job.seed && npts >= SEED_MIN_SET && (D == 2 || D == 3) &&
      workspace() == nullptr) {
    const int sr = seed_single_set(job, a, &seed_cells, &seed_thresh, st);
    if (sr == DT_OK) {
      // seed_cells outlives the copy (the stream is synchronised below)
      DT_HIP(hipMemcpyAsync(&dctr->cells, &seed_cells, 4, hipMemcpyHostToDevice, st));
      DT_HIP(hipMemsetAsync(pool.set_cell0.p, 0, 4, st));
      ks.seeded = 1;
    } else if (sr == DT_E_NOT_READY || sr == DT_E_INTERNAL) {
      // start from one simplex: clear what the seed wrote
      seed_cells = 0;
      DT_HIP(hipMemsetAsync(ploc.p, 0, (size_t)npts * 4, st));
      DT_HIP(hipMemsetAsync(dctr, 0, sizeof(Counters), st));
    } else {
      return sr;
    }
  } else if (job.nsets > 1 && job.seed && (D == 2 || D == 3) && workspace() == nullptr) {
    uint32_t nsd = 0;
    const int sr = seed_sets(job, a, seeded0, &seed_cells, &seed_thresh, &nsd, st);
    if (sr == DT_OK) {
      DT_HIP(hipMemcpyAsync(&dctr->cells, &seed_cells, 4, hipMemcpyHostToDevice, st));
      ks.seeded = nsd;
    } else if (sr == DT_E_NOT_READY || sr == DT_E_INTERNAL) {
      seed_cells = 0;
      seeded0 = DevBuf();
      DT_HIP(hipMemsetAsync(ploc.p, 0, (size_t)npts * 4, st));
      DT_HIP(hipMemsetAsync(dctr, 0, sizeof(Counters), st));
    } else {
      return sr;
    }
  }
  if (!seed_cells || seeded0.p) {
    if (D == 2)
      hipLaunchKernelGGL(k4_init_sets<2>, dim3(nblk(job.nsets)), dim3(BLOCK), 0, st, a,
                         seeded0.as<uint32_t>());
    else
      hipLaunchKernelGGL(k4_init_sets<3>, dim3(nblk(job.nsets)), dim3(BLOCK), 0, st, a,
                         seeded0.as<uint32_t>());
  }
  hipLaunchKernelGGL(k4_place_init, dim3(nblk(npts)), dim3(BLOCK), 0, st, a);
  DT_HIP(hipGetLastError());
  DT_HIP(hipMemcpyAsync(hctr, dctr, sizeof(Counters), hipMemcpyDeviceToHost, st));
  DT_HIP(hipStreamSynchronize(st));
  const bool dbg = getenv("DT_DEBUG") != nullptr;
  if (dbg)
    fprintf(stderr, "[k4] init npts %u sets %u active %u cells %u flags %x\n", npts, job.nsets,
            hctr->active, hctr->cells, hctr->flags);
  if (hctr->flags) return DT_E_INTERNAL;
  // activation levels: about start_active points per set at first, grown
  // by grow_num/8 whenever fewer are pending than 1/grow_div of those
  // already inserted
  // (decided on the device, see k4_ctl_end)
  const uint32_t PMAX = 1u << 20;
  uint64_t t0 = ((uint64_t)PMAX * job.start_active * job.nsets) / (npts ? npts : 1);
  uint32_t thresh0 = (uint32_t)(t0 < 16 ? 16 : (t0 > PMAX ? PMAX : t0));
  if (seed_cells && seed_thresh > thresh0) thresh0 = seed_thresh;
  a.act = actbuf.as<uint32_t>();
  a.grow_div = job.grow_div ? job.grow_div : 64;
  // Smaller steps between levels keep the pending points sparser: fewer
  // candidates lose.  Many sets (the batched local triangulations) gain
  // most from x1.25; one set from x1.5 (measured on the 4M bubbles and 1M
  // uniform workloads).
  a.grow_num = job.grow_num ? job.grow_num : (job.nsets > 1 ? 10u : 12u);
  a.rings = 3;   // three rings of bids: fewest rounds on clustered 3D input
  hipLaunchKernelGGL(k4_ctl_init, dim3(1), dim3(1), 0, st, a, thresh0);
  // Rounds run back to back in groups; the host reads the control state
  // once per group.  Rounds past the end do nothing (the skip word).
  const uint32_t gb = npts ? (nblk(npts) < 2048 ? nblk(npts) : 2048) : 1;
  const uint32_t ga = npts ? (nblk(npts) < 8192 ? nblk(npts) : 8192) : 1;
  uint64_t cbound = npts < maxcand ? (npts ? npts : 1) : maxcand;
  const uint32_t gi = (uint32_t)(cbound < job.cand_blocks ? cbound : job.cand_blocks);
  // the insert runs INS_WAVES candidates per block
  const uint32_t gib = (gi + INS_WAVES - 1) / INS_WAVES;
  // the cavity search runs CAV_GROUPS candidates per block
  const uint32_t gc = (gi + CAV_GROUPS - 1) / CAV_GROUPS;
  // DT_DEBUG=2: one round per group, traced
  const bool trace = dbg && getenv("DT_DEBUG")[0] == '2';
  uint32_t round = 1, group = trace ? 1 : 4;
  for (;;) {
    for (uint32_t r = 0; r < group; r++, round++) {
      if (round >= (1u << 30)) return DT_E_INTERNAL;
      if ((round & 0xFFFu) == 0) {
        // the 12-bit round stamp wraps: clear every cavity and shell claim
        // in use (bids carry no stamp)
        DT_HIP(hipMemcpyAsync(hctr, dctr, sizeof(Counters), hipMemcpyDeviceToHost, st));
        DT_HIP(hipStreamSynchronize(st));
        size_t used = hctr->cells < pool.cap ? hctr->cells : pool.cap;
        if (used)
          hipLaunchKernelGGL(k4_reset_claims, dim3(nblk((uint32_t)used)), dim3(BLOCK), 0, st,
                             pool.cells.as<Cell>(), (uint32_t)used);
      }
      a.round = round;
      hipLaunchKernelGGL(k4_build_active, dim3(gb), dim3(BLOCK), 0, st, a);
      DT_PROF_BEGIN(DT_KERN_K4_PICK, st);
      if (D == 2 && a.fp32) hipLaunchKernelGGL((k4_pick<2, true>), dim3(ga), dim3(BLOCK), 0, st, a);
      else if (D == 2) hipLaunchKernelGGL((k4_pick<2, false>), dim3(ga), dim3(BLOCK), 0, st, a);
      else if (a.fp32) hipLaunchKernelGGL((k4_pick<3, true>), dim3(ga), dim3(BLOCK), 0, st, a);
      else hipLaunchKernelGGL((k4_pick<3, false>), dim3(ga), dim3(BLOCK), 0, st, a);
      DT_PROF_END(st);
      DT_PROF_BEGIN(DT_KERN_K4_SELECT, st);
      if (D == 2) hipLaunchKernelGGL(k4_select<2>, dim3(ga), dim3(BLOCK), 0, st, a);
      else hipLaunchKernelGGL(k4_select<3>, dim3(ga), dim3(BLOCK), 0, st, a);
      DT_PROF_END(st);
      DT_PROF_BEGIN(DT_KERN_K4_CAVITY, st);
      if (D == 2 && a.fp32) hipLaunchKernelGGL((k4_cavity<2, true>), dim3(gc), dim3(64), 0, st, a);
      else if (D == 2) hipLaunchKernelGGL((k4_cavity<2, false>), dim3(gc), dim3(64), 0, st, a);
      else if (a.fp32) hipLaunchKernelGGL((k4_cavity<3, true>), dim3(gc), dim3(64), 0, st, a);
      else hipLaunchKernelGGL((k4_cavity<3, false>), dim3(gc), dim3(64), 0, st, a);
      DT_PROF_END(st);
      DT_PROF_BEGIN(DT_KERN_K4_INSERT, st);
      if (D == 2) hipLaunchKernelGGL(k4_insert<2>, dim3(gib), dim3(64 * INS_WAVES), 0, st, a);
      else hipLaunchKernelGGL(k4_insert<3>, dim3(gib), dim3(64 * INS_WAVES), 0, st, a);
      DT_PROF_END(st);
      hipLaunchKernelGGL(k4_ctl_end, dim3(1), dim3(1), 0, st, a);
      DT_HIP(hipGetLastError());
    }
    DT_HIP(hipMemcpyAsync(hctr, dctr, sizeof(Counters), hipMemcpyDeviceToHost, st));
    DT_HIP(hipStreamSynchronize(st));
    if (dbg)
      fprintf(stderr,
              "[k4] round %u (device %u) thresh %u nact %u remaining %llu cells %u maxcav %u "
              "flags %x\n",
              round - 1, hctr->rounds, hctr->thresh, hctr->nact, hctr->remaining, hctr->cells,
              hctr->maxcav, hctr->flags);
    if (hctr->flags) { ks.rounds = (int)hctr->rounds; return DT_E_INTERNAL; }
    if (trace)
      fprintf(stderr, "[k4r] %u %u %u %u %u\n", hctr->rounds, hctr->thresh, hctr->nact,
              hctr->last_cand, hctr->last_ins);
    if (hctr->giant_need) {
      // a cavity outgrew the regular lists: give its candidate a list as
      // large as the pool (no cavity can hold more cells), then go on
      if (!gcell.p) {
        DT_TRY(gcell.alloc(cap * sizeof(uint32_t)));
        DT_TRY(ginfo.alloc(cap * sizeof(uint32_t)));
        a.gcell = gcell.as<uint32_t>();
        a.ginfo = ginfo.as<uint32_t>();
        a.gcap = pool.cap;
      }
      if (dbg) fprintf(stderr, "[k4] pool-sized cavity list for point %u\n", hctr->giant_owner);
      hipLaunchKernelGGL(k4_resume, dim3(1), dim3(1), 0, st, a);
      DT_HIP(hipGetLastError());
      continue;
    }
    if (hctr->skip) break;
    if (group < 32 && !trace) group *= 2;
  }
  ks.rounds = (int)hctr->rounds;
  ks.candidates = hctr->cand_total;
  ks.giant_rounds = hctr->giant_rounds;
  pool.ncells = hctr->cells;
  {
    Stripes hs;
    DT_HIP(hipMemcpyAsync(&hs, stripes.p, sizeof(Stripes), hipMemcpyDeviceToHost, st));
    DT_HIP(hipStreamSynchronize(st));
    ks.maxcav = 0;
    ks.cavity_cells = 0;
    for (int i = 0; i < 4; i++)
      for (int j = 0; j < 4; j++) ks.pred[i][j] = 0;
    for (uint32_t b = 0; b < NSTRIPE; b++) {
      for (int i = 0; i < 4; i++)
        for (int j = 0; j < 4; j++) ks.pred[i][j] += hs.pred[b][i * 4 + j];
      ks.cavity_cells += hs.cavcells[b];
      ks.verified += hs.verified[b];
      if (hs.maxcav[b] > ks.maxcav) ks.maxcav = hs.maxcav[b];
    }
  }
  if (dbg)
    fprintf(stderr, "[k4] done npts %u sets %u rounds %u candidates %llu searches completed %llu\n",
            npts, job.nsets, hctr->rounds, hctr->cand_total, ks.verified);
  return DT_OK;
}

int k4_extract(const LocalJob& job, const CellPool& pool, int32_t* rows, uint32_t* count_dev,
               uint32_t* set_rows, hipStream_t st) {
  DT_HIP(hipMemsetAsync(count_dev, 0, sizeof(uint32_t), st));
  if (pool.ncells == 0) return DT_OK;
  const uint32_t nb = nblk(pool.ncells);
  DevBuf bcnt, boff;
  DT_TRY(bcnt.alloc((size_t)(nb + 1) * 4));
  DT_TRY(boff.alloc((size_t)(nb + 1) * 4));
  DT_HIP(hipMemsetAsync(bcnt.as<uint32_t>() + nb, 0, 4, st));
  if (job.D == 2)
    hipLaunchKernelGGL(k4_count_rows<2>, dim3(nb), dim3(BLOCK), 0, st, job.pset,
                       pool.cells.as<Cell>(), pool.ncells,
                       bcnt.as<uint32_t>(), set_rows);
  else
    hipLaunchKernelGGL(k4_count_rows<3>, dim3(nb), dim3(BLOCK), 0, st, job.pset,
                       pool.cells.as<Cell>(), pool.ncells,
                       bcnt.as<uint32_t>(), set_rows);
  DT_HIP(hipGetLastError());
  DT_TRY(exclusive_scan(bcnt.as<uint32_t>(), boff.as<uint32_t>(), nb + 1, st));
  DT_HIP(hipMemcpyAsync(count_dev, boff.as<uint32_t>() + nb, 4, hipMemcpyDeviceToDevice, st));
  if (rows) {
    if (job.D == 2)
      hipLaunchKernelGGL(k4_write_rows<2>, dim3(nb), dim3(BLOCK), 0, st, job.pts,
                         pool.cells.as<Cell>(), pool.ncells,
                         boff.as<uint32_t>(), rows);
    else
      hipLaunchKernelGGL(k4_write_rows<3>, dim3(nb), dim3(BLOCK), 0, st, job.pts,
                         pool.cells.as<Cell>(), pool.ncells,
                         boff.as<uint32_t>(), rows);
    DT_HIP(hipGetLastError());
  }
  // the block offsets are freed on return: finish the launches first
  DT_HIP(hipStreamSynchronize(st));
  return DT_OK;
}

}  // namespace dtk
