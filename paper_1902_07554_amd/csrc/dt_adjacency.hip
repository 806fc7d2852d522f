// Neighbourhood of the output simplices (Algorithm 1, neighbourhood
// update): two simplices of the result are neighbours when they share a
// facet, i.e. D of their vertex ids.  Every facet of every row gets a key
// (set, sorted ids of the facet); a stable radix sort on the key brings the
// two copies of an interior facet together, and each copy records the row
// of the other.  Facets with one copy lie on the convex hull (-1).
#include <vector>

#include "dt_common.hpp"
#include "dt_internal.hpp"
#include "dt_pipeline.hpp"
#include "dt_prims.hpp"

namespace dtk {

namespace {

constexpr int AB = 256;

inline uint32_t ablocks(uint64_t n) { return (uint32_t)((n + AB - 1) / AB); }

// set of row i: the s with off[s] <= i < off[s+1]
__device__ __forceinline__ uint32_t set_of_row(const int64_t* off, uint32_t nsets, int64_t i) {
  uint32_t lo = 0, hi = nsets;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (off[mid] <= i) lo = mid;
    else hi = mid;
  }
  return lo;
}

// The D ids of facet f (row f / (D+1) without its vertex f % (D+1)); rows
// hold their ids in ascending order, so the facet's ids are ascending too.
template <int D>
__device__ __forceinline__ void facet_ids(const int32_t* rows, uint64_t f, uint32_t id[3]) {
  const uint64_t i = f / (D + 1);
  const int j = (int)(f % (D + 1));
  int t = 0;
  id[2] = 0;
#pragma unroll
  for (int r = 0; r <= D; r++)
    if (r != j) id[t++] = (uint32_t)rows[i * (D + 1) + r];
}

// first sort key: the last facet id (3D) or 0 (2D)
template <int D>
__global__ void k_facet_lo(const int32_t* rows, uint64_t nf, unsigned long long* keys,
                           uint32_t* vals) {
  const uint64_t f = (uint64_t)blockIdx.x * AB + threadIdx.x;
  if (f >= nf) return;
  uint32_t id[3];
  facet_ids<D>(rows, f, id);
  keys[f] = id[2];
  vals[f] = (uint32_t)f;
}

// second sort key: the first two facet ids (the set is sorted last)
template <int D>
__global__ void k_facet_mid(const int32_t* rows, uint64_t nf, const uint32_t* vals,
                            unsigned long long* keys) {
  const uint64_t p = (uint64_t)blockIdx.x * AB + threadIdx.x;
  if (p >= nf) return;
  uint32_t id[3];
  facet_ids<D>(rows, vals[p], id);
  keys[p] = ((unsigned long long)id[0] << 32) | id[1];
}

template <int D>
__global__ void k_facet_set(uint64_t nf, const uint32_t* vals, const int64_t* off, uint32_t nsets,
                            unsigned long long* keys) {
  const uint64_t p = (uint64_t)blockIdx.x * AB + threadIdx.x;
  if (p >= nf) return;
  keys[p] = set_of_row(off, nsets, (int64_t)(vals[p] / (D + 1)));
}

template <int D>
__device__ __forceinline__ bool same_facet(const int32_t* rows, const int64_t* off, uint32_t nsets,
                                           uint32_t f, uint32_t g) {
  uint32_t a[3], b[3];
  facet_ids<D>(rows, f, a);
  facet_ids<D>(rows, g, b);
  if (a[0] != b[0] || a[1] != b[1] || a[2] != b[2]) return false;
  return nsets == 1 ||
         set_of_row(off, nsets, f / (D + 1)) == set_of_row(off, nsets, g / (D + 1));
}

template <int D>
__global__ void k_facet_pair(const int32_t* rows, uint64_t nf, const uint32_t* vals,
                             const int64_t* off, uint32_t nsets, int32_t* nbr) {
  const uint64_t p = (uint64_t)blockIdx.x * AB + threadIdx.x;
  if (p >= nf) return;
  const uint32_t f = vals[p];
  int32_t other = -1;
  if (p + 1 < nf && same_facet<D>(rows, off, nsets, f, vals[p + 1]))
    other = (int32_t)(vals[p + 1] / (D + 1));
  else if (p > 0 && same_facet<D>(rows, off, nsets, f, vals[p - 1]))
    other = (int32_t)(vals[p - 1] / (D + 1));
  nbr[f] = other;
}

}  // namespace

int compute_neighbors(const dt_result& r, DevBuf& nbr, hipStream_t st) {
  const int D = r.D;
  const uint64_t nf = (uint64_t)r.m * (D + 1);
  DT_TRY(nbr.alloc_plain((size_t)(nf ? nf : 1) * 4));
  if (nf == 0) return DT_OK;
  if (nf > 0xFFFFFFFFull) return DT_E_INVALID_ARG;
  const uint32_t nsets = r.set_offsets.size() > 1 ? (uint32_t)(r.set_offsets.size() - 1) : 1u;
  DevBuf keys, vals, off;
  DT_TRY(keys.alloc(nf * 8));
  DT_TRY(vals.alloc(nf * 4));
  DT_TRY(off.alloc((size_t)(nsets + 1) * 8));
  std::vector<int64_t> hoff(nsets + 1, 0);
  if (r.set_offsets.size() > 1) hoff = r.set_offsets;
  else hoff[1] = r.m;
  DT_HIP(hipMemcpyAsync(off.p, hoff.data(), (size_t)(nsets + 1) * 8, hipMemcpyHostToDevice, st));
  const int32_t* rows = r.rows.as<int32_t>();
  const uint32_t nb = ablocks(nf);
  const int idbits = 32;   // labels are int32: sort on all their bits
  // least significant key first: last id, then the first two ids, then the set
  if (D == 3) {
    hipLaunchKernelGGL(k_facet_lo<3>, dim3(nb), dim3(AB), 0, st, rows, nf,
                       keys.as<unsigned long long>(), vals.as<uint32_t>());
    DT_TRY(radix_sort_pairs(keys.as<unsigned long long>(), vals.as<uint32_t>(), (uint32_t)nf,
                            idbits, st));
    hipLaunchKernelGGL(k_facet_mid<3>, dim3(nb), dim3(AB), 0, st, rows, nf, vals.as<uint32_t>(),
                       keys.as<unsigned long long>());
  } else {
    hipLaunchKernelGGL(k_facet_lo<2>, dim3(nb), dim3(AB), 0, st, rows, nf,
                       keys.as<unsigned long long>(), vals.as<uint32_t>());
    hipLaunchKernelGGL(k_facet_mid<2>, dim3(nb), dim3(AB), 0, st, rows, nf, vals.as<uint32_t>(),
                       keys.as<unsigned long long>());
  }
  DT_TRY(radix_sort_pairs(keys.as<unsigned long long>(), vals.as<uint32_t>(), (uint32_t)nf, 64,
                          st));
  if (nsets > 1) {
    int sbits = 1;
    while (sbits < 32 && (1ull << sbits) < nsets) sbits++;
    if (D == 3)
      hipLaunchKernelGGL(k_facet_set<3>, dim3(nb), dim3(AB), 0, st, nf, vals.as<uint32_t>(),
                         off.as<int64_t>(), nsets, keys.as<unsigned long long>());
    else
      hipLaunchKernelGGL(k_facet_set<2>, dim3(nb), dim3(AB), 0, st, nf, vals.as<uint32_t>(),
                         off.as<int64_t>(), nsets, keys.as<unsigned long long>());
    DT_TRY(radix_sort_pairs(keys.as<unsigned long long>(), vals.as<uint32_t>(), (uint32_t)nf,
                            sbits, st));
  }
  if (D == 3)
    hipLaunchKernelGGL(k_facet_pair<3>, dim3(nb), dim3(AB), 0, st, rows, nf, vals.as<uint32_t>(),
                       off.as<int64_t>(), nsets, nbr.as<int32_t>());
  else
    hipLaunchKernelGGL(k_facet_pair<2>, dim3(nb), dim3(AB), 0, st, rows, nf, vals.as<uint32_t>(),
                       off.as<int64_t>(), nsets, nbr.as<int32_t>());
  DT_HIP(hipGetLastError());
  DT_HIP(hipStreamSynchronize(st));
  return DT_OK;
}

}  // namespace dtk
