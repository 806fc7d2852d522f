// Uniform grid over the bounding box (shared by the nearest-sample search
// and the region border test).
#pragma once
#include "dt_common.hpp"

namespace dtk {

struct Grid {
  double lo[3];
  double h;
  int g[3];
};

__device__ __forceinline__ int cell_coord(double x, double lo, double h, int g) {
  double t = (x - lo) / h;
  int c = (int)floor(t);
  return c < 0 ? 0 : (c >= g ? g - 1 : c);
}

// Exact nearest sample of point x under the key (fl(d^2), sample id):
// visit grid shells of growing Chebyshev radius and stop once no
// unvisited cell can hold a closer sample (with a margin far above the
// rounding of d^2).  Returns the sample index; *d2 receives fl(d^2).
__device__ inline uint32_t grid_nearest(const double4* S, const uint32_t* start,
                                        const uint32_t* items, const Grid& G, double px,
                                        double py, double pz, double* d2out) {
  int c[3] = {cell_coord(px, G.lo[0], G.h, G.g[0]), cell_coord(py, G.lo[1], G.h, G.g[1]),
              cell_coord(pz, G.lo[2], G.h, G.g[2])};
  double pc[3] = {px, py, pz};
  double best = INFINITY;
  long long bestid = 0x7FFFFFFFFFFFFFFFll;
  uint32_t bests = 0;
  int gmax = max(G.g[0], max(G.g[1], G.g[2]));
  for (int r = 0; r <= gmax; r++) {
    int lo[3], hi[3];
    for (int k = 0; k < 3; k++) {
      lo[k] = max(c[k] - r, 0);
      hi[k] = min(c[k] + r, G.g[k] - 1);
    }
    for (int z = lo[2]; z <= hi[2]; z++)
      for (int y = lo[1]; y <= hi[1]; y++) {
        bool edge_zy = (z == c[2] - r) || (z == c[2] + r) || (y == c[1] - r) || (y == c[1] + r);
        for (int x = lo[0]; x <= hi[0]; x++) {
          if (!edge_zy && x != c[0] - r && x != c[0] + r) {
            if (x < c[0] + r) x = c[0] + r - 1;   // skip the shell's interior
            continue;
          }
          uint32_t cell = ((uint32_t)z * G.g[1] + y) * G.g[0] + x;
          for (uint32_t j = start[cell]; j < start[cell + 1]; j++) {
            uint32_t s = items[j];
            double4 q = S[s];
            double dx = px - q.x, dy = py - q.y, dz = pz - q.z;
            double d2 = (dx * dx + dy * dy) + dz * dz;
            long long sid = __double_as_longlong(q.w);
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
      double dm = fmax(dmin, 0.0) * (1.0 - 1e-9);
      if (dm * dm > best * (1.0 + 1e-9)) break;
    }
  }
  *d2out = best;
  return bests;
}

}  // namespace dtk
