// Device primitives (scan, radix sort, compaction, bounding box).
#pragma once
#include "dt_internal.hpp"

namespace dtk {
// out[i] = sum of in[0..i-1]; synchronises the stream.
int exclusive_scan(const uint32_t* in, uint32_t* out, uint32_t n, hipStream_t st);
// Stable LSD sort of (keys, vals) on the low `bits` bits of the keys; vals
// may be null.  In place; synchronises the stream.
int radix_sort_pairs(unsigned long long* keys, uint32_t* vals, uint32_t n, int bits,
                     hipStream_t st);
// out = ascending indices i with flag[i] != 0; *count = their number.
int compact_indices(const uint32_t* flag, uint32_t n, DevBuf& out, uint32_t* count,
                    hipStream_t st);
// Coordinate-wise bounding box of the first D coordinates (z = 0 in 2D).
int bbox(const double4* p, uint32_t n, double lo[3], double hi[3], hipStream_t st);
// Spatial sort keys: keys[i] = prefix[i] << 30 | Morton code of point i in
// the box [lo, hi] (10 bits per axis in 3D, 15 in 2D); prefix may be null.
// vals[i] = i.  Sorting by these keys groups the points by prefix and
// orders each group along a space-filling curve.
constexpr int MORTON_BITS = 30;
int spatial_keys(const double4* p, uint32_t n, int D, const double lo[3], const double hi[3],
                 const uint32_t* prefix, unsigned long long* keys, uint32_t* vals,
                 hipStream_t st);
}  // namespace dtk
