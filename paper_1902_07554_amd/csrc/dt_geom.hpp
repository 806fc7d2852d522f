// Device geometry shared by the border tests: a uniform grid over a box,
// and the conservative circumscribed ball of a simplex.
#pragma once
#include <math.h>

#include "dt_common.hpp"

namespace dtk {

struct BGrid {
  double lo[3];
  double h;
  int g[3];
};

__device__ __forceinline__ int bcoord(double x, const BGrid& G, int k) {
  double t = (x - G.lo[k]) / G.h;
  int c = (int)floor(t);
  return c < 0 ? 0 : (c >= G.g[k] ? G.g[k] - 1 : c);
}

// Circumscribed ball of the finite simplex with vertices a, b, c (, d):
// centre and radius in FP64, the radius enlarged by 1e-6 (r + longest
// edge) + 1e-12 |a| so that it covers the exact ball.  Returns false for a
// nearly flat simplex (|det| <= 1e-7 times the product of the edge
// lengths), whose ball is not computed reliably.
template <int D>
__device__ __forceinline__ bool circumball(const double4& a, const double4& pb,
                                           const double4& pc, const double4& pd, double ctr[3],
                                           double* rout) {
  if (D == 3) {
    double b0 = pb.x - a.x, b1 = pb.y - a.y, b2 = pb.z - a.z;
    double c0 = pc.x - a.x, c1 = pc.y - a.y, c2 = pc.z - a.z;
    double d0 = pd.x - a.x, d1 = pd.y - a.y, d2 = pd.z - a.z;
    double cd0 = c1 * d2 - c2 * d1, cd1 = c2 * d0 - c0 * d2, cd2 = c0 * d1 - c1 * d0;
    double db0 = d1 * b2 - d2 * b1, db1 = d2 * b0 - d0 * b2, db2 = d0 * b1 - d1 * b0;
    double bc0 = b1 * c2 - b2 * c1, bc1 = b2 * c0 - b0 * c2, bc2 = b0 * c1 - b1 * c0;
    double det = b0 * cd0 + b1 * cd1 + b2 * cd2;
    double lb = b0 * b0 + b1 * b1 + b2 * b2, lc = c0 * c0 + c1 * c1 + c2 * c2,
           ld = d0 * d0 + d1 * d1 + d2 * d2;
    double scale = sqrt(lb * lc * ld);
    if (!(fabs(det) > 1e-7 * scale)) return false;
    double inv = 0.5 / det;
    double x = (lb * cd0 + lc * db0 + ld * bc0) * inv;
    double y = (lb * cd1 + lc * db1 + ld * bc1) * inv;
    double z = (lb * cd2 + lc * db2 + ld * bc2) * inv;
    double r = sqrt(x * x + y * y + z * z);
    double L = sqrt(fmax(lb, fmax(lc, ld)));
    *rout = r + 1e-6 * (r + L) + 1e-12 * (fabs(a.x) + fabs(a.y) + fabs(a.z));
    ctr[0] = a.x + x;
    ctr[1] = a.y + y;
    ctr[2] = a.z + z;
    return true;
  } else {
    double b0 = pb.x - a.x, b1 = pb.y - a.y, c0 = pc.x - a.x, c1 = pc.y - a.y;
    double det = b0 * c1 - b1 * c0;
    double lb = b0 * b0 + b1 * b1, lc = c0 * c0 + c1 * c1;
    if (!(fabs(det) > 1e-7 * sqrt(lb * lc))) return false;
    double inv = 0.5 / det;
    double x = (c1 * lb - b1 * lc) * inv;
    double y = (b0 * lc - c0 * lb) * inv;
    double r = sqrt(x * x + y * y);
    double L = sqrt(fmax(lb, lc));
    *rout = r + 1e-6 * (r + L) + 1e-12 * (fabs(a.x) + fabs(a.y));
    ctr[0] = a.x + x;
    ctr[1] = a.y + y;
    ctr[2] = 0.0;
    return true;
  }
}

// Grid of about `cells_target` cells over [lo, hi] (at most 4096 per axis).
inline BGrid make_bgrid(const double lo[3], const double hi[3], int D, double cells_target,
                        uint64_t* total_out) {
  BGrid G;
  double vol = 1.0;
  int nd = 0;
  for (int a = 0; a < D; a++) {
    double e = hi[a] - lo[a];
    if (e > 0) { vol *= e; nd++; }
  }
  double h = nd ? pow(vol / (cells_target > 1 ? cells_target : 1.0), 1.0 / nd) : 1.0;
  if (!(h > 0)) h = 1.0;
  uint64_t total = 1;
  for (int a = 0; a < 3; a++) {
    G.lo[a] = lo[a];
    long g = (a < D) ? (long)floor((hi[a] - lo[a]) / h) + 1 : 1;
    if (g < 1) g = 1;
    if (g > 4096) g = 4096;
    G.g[a] = (int)g;
    total *= (uint64_t)g;
  }
  G.h = h;
  *total_out = total;
  return G;
}

}  // namespace dtk
