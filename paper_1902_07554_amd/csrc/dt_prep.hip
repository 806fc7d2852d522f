// Input preparation kernels: validation (finite coordinates, no duplicate
// points -- the paper's input is a set, Section "Delaunay Triangulations")
// and conversion of row-major coordinates to the double4 point records used
// by the triangulation kernels.
#include "dt_common.hpp"
#include "dt_internal.hpp"
#include "dt_prep.hpp"

namespace dtk {

constexpr int PB = 256;

// Row-major n x D doubles -> double4 (x, y, z or 0, key bits).  keys may be
// null (key = row index).  Flags non-finite coordinates.
__global__ void k_pack(const double* __restrict__ in, const long long* __restrict__ keys,
                       uint32_t n, int D, double4* __restrict__ out, uint32_t* flags) {
  uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double x = in[(size_t)i * D], y = in[(size_t)i * D + 1];
  double z = (D == 3) ? in[(size_t)i * D + 2] : 0.0;
  if (!isfinite(x) || !isfinite(y) || !isfinite(z)) atomicOr(flags, 1u);
  long long k = keys ? keys[i] : (long long)i;
  // +0.0 turns -0.0 into +0.0 so that equal coordinates have equal bits
  out[i] = make_double4(x + 0.0, y + 0.0, z + 0.0, __longlong_as_double(k));
}

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z ^= z >> 33;
  z *= 0xFF51AFD7ED558CCDull;
  z ^= z >> 33;
  z *= 0xC4CEB9FE1A85EC53ull;
  z ^= z >> 33;
  return z;
}

// Duplicate detection by open addressing on the coordinate bits (and the
// set, when points belong to independent sets): the table stores point
// index + 1; a collision compares coordinates and set.
__global__ void k_dupcheck(const double4* __restrict__ p, const uint32_t* __restrict__ pset,
                           uint32_t n, uint32_t* table, uint32_t tmask, uint32_t* flags) {
  uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double4 a = p[i];
  uint32_t sa = pset ? pset[i] : 0u;
  uint64_t bx = (uint64_t)__double_as_longlong(a.x), by = (uint64_t)__double_as_longlong(a.y),
           bz = (uint64_t)__double_as_longlong(a.z);
  uint32_t h = (uint32_t)mix64(bx ^ mix64(by ^ mix64(bz ^ mix64(sa))));
  for (uint32_t probe = 0; probe <= tmask; probe++) {
    uint32_t s = (h + probe) & tmask;
    uint32_t old = atomicCAS(&table[s], 0u, i + 1);
    if (old == 0) return;
    double4 b = p[old - 1];
    if (b.x == a.x && b.y == a.y && b.z == a.z && (!pset || pset[old - 1] == sa)) {
      atomicOr(flags, 2u);
      return;
    }
  }
  atomicOr(flags, 4u);
}

int prep_points(const double* dev_in, const long long* dev_keys, const uint32_t* pset, uint32_t n,
                int D, double4* out, DevBuf& scratch, uint32_t* dflag, uint32_t* hflag,
                hipStream_t st) {
  if (n == 0) return DT_OK;
  uint32_t tsize = 1;
  while (tsize < 2 * n) tsize <<= 1;
  DT_TRY(scratch.alloc((size_t)tsize * 4));
  DT_HIP(hipMemsetAsync(scratch.p, 0, (size_t)tsize * 4, st));
  DT_HIP(hipMemsetAsync(dflag, 0, 4, st));
  hipLaunchKernelGGL(k_pack, dim3((n + PB - 1) / PB), dim3(PB), 0, st, dev_in, dev_keys, n, D, out,
                     dflag);
  hipLaunchKernelGGL(k_dupcheck, dim3((n + PB - 1) / PB), dim3(PB), 0, st, out, pset, n,
                     scratch.as<uint32_t>(), tsize - 1, dflag);
  DT_HIP(hipGetLastError());
  DT_HIP(hipMemcpyAsync(hflag, dflag, 4, hipMemcpyDeviceToHost, st));
  DT_HIP(hipStreamSynchronize(st));
  if (*hflag & 1u) return DT_E_NONFINITE;
  if (*hflag & 2u) return DT_E_DUPLICATE;
  if (*hflag & 4u) return DT_E_INTERNAL;
  return DT_OK;
}

}  // namespace dtk
