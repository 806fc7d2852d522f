// The Voronoi region test of the sample divide, shared by the k-way merge
// and the merges of the recursive bisection.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dt_stages.hpp"

namespace dtk {

// Voronoi test over the sample's Delaunay graph, for the sample divide (the
// intersection test of Algorithm 1, "Border triangulation", against the
// regions of Algorithm 2's partition).
// First a greedy descent from the own sample t: move to the neighbour of
// smallest key (fl(d^2) to the centre, id) while it beats the current one;
// a sample that no Delaunay neighbour beats is the nearest to the centre up
// to rounding.  Then the cells the ball reaches: from a reached own sample
// u, a neighbour w is reached when the ball meets w's side of the bisector
// of u and w and also w's side of the bisector of t and w (the centre is at
// most r from each, with a slack far above the rounding of the distances);
// w's cell lies on w's side of both, so a cell that the ball meets passes
// both tests.  Voronoi cells are convex and tile space, so the cells that
// the ball meets are linked through shared facets, that is through
// Delaunay edges of the sample, and each of them is reached.  A reached
// sample of another block flags the simplex; so do a long descent or more
// than VW_CAP reached cells.  vis: VW_CAP slots, stride STRIDE.
constexpr int VW_CAP = 16;
constexpr int VW_STEPS = 64;

template <int D, int STRIDE>
__device__ bool voronoi_walk_hit(const Region& R, uint32_t me, const double* ctr, double r,
                                 uint32_t t, uint32_t* vis) {
  const double cx = ctr[0], cy = ctr[1], cz = D == 3 ? ctr[2] : 0.0;
  // does the ball reach w's side of the bisector of u and w?  (signed
  // distance of the centre from it, on u's side: (dw - du) / (2 |w - u|))
  auto reach = [&](const double4& up, double du, const double4& q, double dw) {
    const double ex = q.x - up.x, ey = q.y - up.y, ez = q.z - up.z;
    const double gap = sqrt(ex * ex + ey * ey + ez * ez);
    return dw - du <= 2.0 * gap * r + 2e-12 * (du + dw + 2.0 * r * r);
  };
  double4 tp = R.S[t];
  double dt;
  {
    const double dx = cx - tp.x, dy = cy - tp.y, dz = cz - tp.z;
    dt = (dx * dx + dy * dy) + dz * dz;
  }
  // the descent's last pass also tests t's neighbours for the search
  // (lists of up to 64), so the search starts one cell in
  uint64_t hits = 0;
  bool fused = false;
  for (int step = 0;; step++) {
    if (step == VW_STEPS) return true;
    uint32_t best = t;
    double bd = dt;
    long long bid = __double_as_longlong(tp.w);
    double4 bp = tp;
    const uint32_t a = R.goff[t], b = R.goff[t + 1];
    const bool track = b - a <= 64;
    uint64_t hm = 0;
    for (uint32_t j = a; j < b; j++) {
      const uint32_t w = R.gadj[j];
      const double4 q = R.S[w];
      const double dx = cx - q.x, dy = cy - q.y, dz = cz - q.z;
      const double d = (dx * dx + dy * dy) + dz * dz;
      const long long id = __double_as_longlong(q.w);
      if (d < bd || (d == bd && id < bid)) { best = w; bd = d; bid = id; bp = q; }
      if (track && reach(tp, dt, q, d)) hm |= 1ull << (j - a);
    }
    if (best == t) {
      hits = hm;
      fused = track;
      break;
    }
    t = best;
    dt = bd;
    tp = bp;
  }
  if (R.part[t] != me) return true;
  int nv = 1, head = 0;
  vis[0] = t;
  if (fused) {
    head = 1;
    const uint32_t a = R.goff[t];
    while (hits) {
      const uint32_t w = R.gadj[a + __builtin_ctzll(hits)];
      hits &= hits - 1;
      if (R.part[w] != me || nv == VW_CAP) return true;
      vis[(size_t)nv++ * STRIDE] = w;
    }
  }
  while (head < nv) {
    const uint32_t u = vis[(size_t)head++ * STRIDE];
    const double4 up = R.S[u];
    const double ux = cx - up.x, uy = cy - up.y, uz = cz - up.z;
    const double du = (ux * ux + uy * uy) + uz * uz;
    const uint32_t a = R.goff[u], b = R.goff[u + 1];
    for (uint32_t j = a; j < b; j++) {
      const uint32_t w = R.gadj[j];
      bool seen = false;
      for (int i = 0; i < nv; i++) seen |= vis[(size_t)i * STRIDE] == w;
      if (seen) continue;
      const double4 q = R.S[w];
      const double ax = cx - q.x, ay = cy - q.y, az = cz - q.z;
      const double dw = (ax * ax + ay * ay) + az * az;
      if (reach(up, du, q, dw) && (u == t || reach(tp, dt, q, dw))) {
        if (R.part[w] != me || nv == VW_CAP) return true;
        vis[(size_t)nv++ * STRIDE] = w;
      }
    }
  }
  return false;
}

}  // namespace dtk
