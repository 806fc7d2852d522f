// Gift-wrapping triangulation of small point sets (dt_gwrap.hip).
#pragma once
#include "dt_internal.hpp"

namespace dtk {

// A single set of at most this many points is gift-wrapped (16-bit point
// indices in the simplex keys), and each of several sets wrapped together
// at most GW_MAX_SET_POINTS (13 bits, the rest of the key is the set).
constexpr uint32_t GW_MAX_POINTS = 65536;
constexpr uint32_t GW_MAX_SET_POINTS = 8192;

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
// (or more sets than the simplex keys can tell apart).  first (device,
// nsets entries, may be null) receives a cell of every non-empty set (its
// seed simplex); other entries are left alone.  Synchronises `st`.
int gift_wrap_sets(const double4* P, uint32_t n, const uint32_t* soff, uint32_t nsets,
                   uint32_t max_set, int D, CellPool& pool, uint32_t* levels, hipStream_t st,
                   uint32_t* first = nullptr);

}  // namespace dtk
