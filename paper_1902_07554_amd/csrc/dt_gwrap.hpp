// Gift-wrapping triangulation of small point sets (dt_gwrap.hip).
#pragma once
#include "dt_internal.hpp"

namespace dtk {

// Sets of at most this many points are gift-wrapped (each facet search
// reads every point).
constexpr uint32_t GW_MAX_POINTS = 8192;

// The finite Delaunay simplices of the n points P (D = 2 or 3, indices into
// P, positively oriented) as live cells of `pool` (vertices only; no
// neighbour links, no hull cells).  DT_OK: done, *levels = facet levels
// searched.  DT_E_NOT_READY: not done (too many points, no empty seed
// simplex among point 0's nearest, or a capacity ran out); the caller
// triangulates the set by parallel insertion instead.  Synchronises `st`.
int gift_wrap(const double4* P, uint32_t n, int D, CellPool& pool, uint32_t* levels,
              hipStream_t st);

// The same for nsets independent sets wrapped together: set s is the points
// P[soff[s] .. soff[s+1]) (soff on the device; a set is empty or holds
// D+2 to GW_MAX_POINTS points, max_set the largest), and every cell's
// vertices lie in one set.  DT_E_NOT_READY when any set cannot be wrapped
// (or more sets than the simplex keys can tell apart).  Synchronises `st`.
int gift_wrap_sets(const double4* P, uint32_t n, const uint32_t* soff, uint32_t nsets,
                   uint32_t max_set, int D, CellPool& pool, uint32_t* levels, hipStream_t st);

}  // namespace dtk
