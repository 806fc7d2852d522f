// Device primitives used by the divide, border and merge stages:
// exclusive scan, stable LSD radix sort of (key, value) pairs, ordered
// compaction and bounding-box reduction.
//
// The radix sort is also the bucket scatter of Algorithm 2 (points grouped
// by partition, stable in input order): one pass per 8-bit digit, each pass
// = per-tile digit histogram, global scan of (digit, tile) counts, and a
// scatter in which every element's rank among equal digits of its tile is
// found with wavefront ballots (64-lane match on the 8 digit bits) and a
// running per-digit counter in LDS, so the order is stable.
#include "dt_common.hpp"
#include "dt_internal.hpp"
#include "dt_prims.hpp"

#include <string.h>

#include <vector>

namespace dtk {

constexpr int SB = 1024;   // scan block (elements)
constexpr int RT = 256;    // radix threads per block
constexpr int RI = 8;      // elements per thread per radix tile
constexpr int TILE = RT * RI;

// ------------------------------------------------------------ scan
__global__ void k_scan_block(const uint32_t* in, uint32_t* out, uint32_t n, uint32_t* sums) {
  __shared__ uint32_t s[SB];
  uint32_t base = blockIdx.x * SB;
  for (int i = threadIdx.x; i < SB; i += blockDim.x) s[i] = (base + i < n) ? in[base + i] : 0u;
  __syncthreads();
  // Hillis-Steele inclusive scan over the block
  for (int off = 1; off < SB; off <<= 1) {
    uint32_t v[SB / 256];
    int t = 0;
    for (int i = threadIdx.x; i < SB; i += blockDim.x) v[t++] = (i >= off) ? s[i - off] : 0u;
    __syncthreads();
    t = 0;
    for (int i = threadIdx.x; i < SB; i += blockDim.x) s[i] += v[t++];
    __syncthreads();
  }
  for (int i = threadIdx.x; i < SB; i += blockDim.x)
    if (base + i < n) out[base + i] = (i == 0) ? 0u : s[i - 1];
  if (threadIdx.x == 0 && sums) sums[blockIdx.x] = s[SB - 1];
}

__global__ void k_scan_add(uint32_t* out, uint32_t n, const uint32_t* sums) {
  uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] += sums[i / SB];
}

static int scan_rec(const uint32_t* in, uint32_t* out, uint32_t n, hipStream_t st,
                    std::vector<DevBuf>& tmp) {
  uint32_t nb = (n + SB - 1) / SB;
  if (nb <= 1) {
    hipLaunchKernelGGL(k_scan_block, dim3(1), dim3(256), 0, st, in, out, n, (uint32_t*)nullptr);
    DT_HIP(hipGetLastError());
    return DT_OK;
  }
  tmp.emplace_back();
  DevBuf& sums = tmp.back();
  DT_TRY(sums.alloc((size_t)nb * 4));
  tmp.emplace_back();
  DevBuf& ssc = tmp.back();
  DT_TRY(ssc.alloc((size_t)nb * 4));
  uint32_t* ps = sums.as<uint32_t>();
  uint32_t* pss = ssc.as<uint32_t>();
  hipLaunchKernelGGL(k_scan_block, dim3(nb), dim3(256), 0, st, in, out, n, ps);
  DT_HIP(hipGetLastError());
  DT_TRY(scan_rec(ps, pss, nb, st, tmp));
  hipLaunchKernelGGL(k_scan_add, dim3((n + 255) / 256), dim3(256), 0, st, out, n, pss);
  DT_HIP(hipGetLastError());
  return DT_OK;
}

int exclusive_scan(const uint32_t* in, uint32_t* out, uint32_t n, hipStream_t st) {
  if (n == 0) return DT_OK;
  if (n <= (uint32_t)SB) {
    // one block, no temporaries: nothing to wait for
    hipLaunchKernelGGL(k_scan_block, dim3(1), dim3(256), 0, st, in, out, n, (uint32_t*)nullptr);
    DT_HIP(hipGetLastError());
    return DT_OK;
  }
  std::vector<DevBuf> tmp;
  tmp.reserve(16);
  DT_TRY(scan_rec(in, out, n, st, tmp));
  // temporaries are freed at return; make sure the kernels using them ran
  DT_HIP(hipStreamSynchronize(st));
  return DT_OK;
}

// ------------------------------------------------------------ radix sort
__device__ __forceinline__ uint32_t digit_of(unsigned long long k, int shift) {
  return (uint32_t)(k >> shift) & 0xFFu;
}

__global__ void k_radix_hist(const unsigned long long* keys, uint32_t n, int shift, uint32_t* hist,
                             uint32_t ntiles) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  uint32_t base = blockIdx.x * TILE;
  for (int r = 0; r < RI; r++) {
    uint32_t i = base + r * RT + threadIdx.x;
    if (i < n) atomicAdd(&h[digit_of(keys[i], shift)], 1u);
  }
  __syncthreads();
  hist[threadIdx.x * ntiles + blockIdx.x] = h[threadIdx.x];
}

__global__ void k_radix_scatter(const unsigned long long* keys, const uint32_t* vals, uint32_t n,
                                int shift, const uint32_t* offs, uint32_t ntiles,
                                unsigned long long* okeys, uint32_t* ovals) {
  __shared__ uint32_t running[256];
  __shared__ uint32_t wcnt[RT / 64][256];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  running[threadIdx.x] = offs[threadIdx.x * ntiles + blockIdx.x];
  uint32_t base = blockIdx.x * TILE;
  const unsigned long long lt = (1ull << lane) - 1ull;
  for (int r = 0; r < RI; r++) {
    for (int w = 0; w < RT / 64; w++) wcnt[w][threadIdx.x] = 0;
    __syncthreads();
    uint32_t i = base + r * RT + threadIdx.x;
    bool act = i < n;
    unsigned long long k = act ? keys[i] : 0ull;
    uint32_t dg = digit_of(k, shift);
    unsigned long long m = __ballot(act);
#pragma unroll
    for (int b = 0; b < 8; b++) {
      unsigned long long bb = __ballot((dg >> b) & 1u);
      m &= ((dg >> b) & 1u) ? bb : ~bb;
    }
    uint32_t rk = (uint32_t)__popcll(m & lt);
    if (act && rk == 0) wcnt[wave][dg] = (uint32_t)__popcll(m);
    __syncthreads();
    if (act) {
      uint32_t pos = running[dg] + rk;
      for (int w = 0; w < wave; w++) pos += wcnt[w][dg];
      okeys[pos] = k;
      if (vals) ovals[pos] = vals[i];
    }
    __syncthreads();
    uint32_t add = 0;
    for (int w = 0; w < RT / 64; w++) add += wcnt[w][threadIdx.x];
    running[threadIdx.x] += add;
    __syncthreads();
  }
}

int radix_sort_pairs(unsigned long long* keys, uint32_t* vals, uint32_t n, int bits,
                     hipStream_t st) {
  if (n <= 1) return DT_OK;
  uint32_t ntiles = (n + TILE - 1) / TILE;
  DevBuf k2, v2, hist, offs;
  DT_TRY(k2.alloc((size_t)n * 8));
  if (vals) DT_TRY(v2.alloc((size_t)n * 4));
  DT_TRY(hist.alloc((size_t)ntiles * 256 * 4));
  DT_TRY(offs.alloc((size_t)ntiles * 256 * 4));
  unsigned long long* ka = keys;
  unsigned long long* kb = k2.as<unsigned long long>();
  uint32_t* va = vals;
  uint32_t* vb = vals ? v2.as<uint32_t>() : nullptr;
  int passes = (bits + 7) / 8;
  for (int p = 0; p < passes; p++) {
    hipLaunchKernelGGL(k_radix_hist, dim3(ntiles), dim3(RT), 0, st, ka, n, 8 * p,
                       hist.as<uint32_t>(), ntiles);
    DT_HIP(hipGetLastError());
    DT_TRY(exclusive_scan(hist.as<uint32_t>(), offs.as<uint32_t>(), ntiles * 256, st));
    hipLaunchKernelGGL(k_radix_scatter, dim3(ntiles), dim3(RT), 0, st, ka, va, n, 8 * p,
                       offs.as<uint32_t>(), ntiles, kb, vb);
    DT_HIP(hipGetLastError());
    std::swap(ka, kb);
    std::swap(va, vb);
  }
  if (ka != keys) {
    DT_HIP(hipMemcpyAsync(keys, ka, (size_t)n * 8, hipMemcpyDeviceToDevice, st));
    if (vals) DT_HIP(hipMemcpyAsync(vals, va, (size_t)n * 4, hipMemcpyDeviceToDevice, st));
  }
  DT_HIP(hipStreamSynchronize(st));
  return DT_OK;
}

// ------------------------------------------------------------ compaction
__global__ void k_compact_write(const uint32_t* flag, const uint32_t* pos, uint32_t n,
                                uint32_t* out) {
  uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && flag[i]) out[pos[i]] = i;
}

int compact_indices(const uint32_t* flag, uint32_t n, DevBuf& out, uint32_t* count,
                    hipStream_t st) {
  *count = 0;
  if (n == 0) return out.alloc(16);
  DevBuf pos;
  DT_TRY(pos.alloc((size_t)n * 4));
  DT_TRY(exclusive_scan(flag, pos.as<uint32_t>(), n, st));
  uint32_t last_pos = 0, last_flag = 0;
  DT_HIP(hipMemcpyAsync(&last_pos, pos.as<uint32_t>() + n - 1, 4, hipMemcpyDeviceToHost, st));
  DT_HIP(hipMemcpyAsync(&last_flag, flag + n - 1, 4, hipMemcpyDeviceToHost, st));
  DT_HIP(hipStreamSynchronize(st));
  uint32_t c = last_pos + (last_flag ? 1 : 0);
  DT_TRY(out.alloc((size_t)(c ? c : 1) * 4));
  hipLaunchKernelGGL(k_compact_write, dim3((n + 255) / 256), dim3(256), 0, st, flag,
                     pos.as<uint32_t>(), n, out.as<uint32_t>());
  DT_HIP(hipGetLastError());
  DT_HIP(hipStreamSynchronize(st));
  *count = c;
  return DT_OK;
}

// ------------------------------------------------------------ bbox
// Doubles mapped to unsigned integers whose order matches the doubles'.
__device__ __forceinline__ unsigned long long ord_bits(double x) {
  unsigned long long u = (unsigned long long)__double_as_longlong(x);
  return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}

__global__ void k_bbox(const double4* p, uint32_t n, unsigned long long* mn,
                       unsigned long long* mx) {
  unsigned long long lo[3] = {~0ull, ~0ull, ~0ull}, hi[3] = {0, 0, 0};
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    double4 q = p[i];
    unsigned long long a = ord_bits(q.x), b = ord_bits(q.y), c = ord_bits(q.z);
    lo[0] = min(lo[0], a); hi[0] = max(hi[0], a);
    lo[1] = min(lo[1], b); hi[1] = max(hi[1], b);
    lo[2] = min(lo[2], c); hi[2] = max(hi[2], c);
  }
  for (int k = 0; k < 3; k++) {
    for (int off = 32; off > 0; off >>= 1) {
      lo[k] = min(lo[k], (unsigned long long)__shfl_xor((long long)lo[k], off));
      hi[k] = max(hi[k], (unsigned long long)__shfl_xor((long long)hi[k], off));
    }
  }
  if ((threadIdx.x & 63) == 0) {
    for (int k = 0; k < 3; k++) {
      atomicMin(&mn[k], lo[k]);
      atomicMax(&mx[k], hi[k]);
    }
  }
}

static double from_ord(unsigned long long u) {
  unsigned long long b = (u >> 63) ? (u & 0x7FFFFFFFFFFFFFFFull) : ~u;
  double d;
  memcpy(&d, &b, 8);
  return d;
}

int bbox(const double4* p, uint32_t n, double lo[3], double hi[3], hipStream_t st) {
  DevBuf b;
  DT_TRY(b.alloc(48));
  unsigned long long init[6] = {~0ull, ~0ull, ~0ull, 0, 0, 0};
  DT_HIP(hipMemcpyAsync(b.p, init, 48, hipMemcpyHostToDevice, st));
  uint32_t nb = (n + 255) / 256;
  if (nb > 2048) nb = 2048;
  if (nb == 0) nb = 1;
  unsigned long long* d = b.as<unsigned long long>();
  hipLaunchKernelGGL(k_bbox, dim3(nb), dim3(256), 0, st, p, n, d, d + 3);
  DT_HIP(hipGetLastError());
  unsigned long long h[6];
  DT_HIP(hipMemcpyAsync(h, b.p, 48, hipMemcpyDeviceToHost, st));
  DT_HIP(hipStreamSynchronize(st));
  for (int k = 0; k < 3; k++) {
    lo[k] = from_ord(h[k]);
    hi[k] = from_ord(h[3 + k]);
  }
  return DT_OK;
}

// Bits of v (at most 10 or 15 used) spread to every third / second bit.
__device__ __forceinline__ unsigned long long spread_bits(uint32_t v, int D) {
  unsigned long long r = 0;
  if (D == 3) {
    for (int b = 0; b < 10; b++) r |= (unsigned long long)((v >> b) & 1u) << (3 * b);
  } else {
    for (int b = 0; b < 15; b++) r |= (unsigned long long)((v >> b) & 1u) << (2 * b);
  }
  return r;
}

__global__ void k_spatial_keys(const double4* __restrict__ p, uint32_t n, int D, double3 lo,
                               double3 inv, const uint32_t* __restrict__ prefix,
                               unsigned long long* __restrict__ keys, uint32_t* __restrict__ vals) {
  uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double4 q = p[i];
  const double cells = (D == 3) ? 1023.0 : 32767.0;
  uint32_t x = (uint32_t)(fmin(fmax((q.x - lo.x) * inv.x, 0.0), 1.0) * cells);
  uint32_t y = (uint32_t)(fmin(fmax((q.y - lo.y) * inv.y, 0.0), 1.0) * cells);
  uint32_t z = (uint32_t)(fmin(fmax((q.z - lo.z) * inv.z, 0.0), 1.0) * cells);
  unsigned long long m = spread_bits(x, D) | (spread_bits(y, D) << 1);
  if (D == 3) m |= spread_bits(z, D) << 2;
  keys[i] = (prefix ? ((unsigned long long)prefix[i] << MORTON_BITS) : 0ull) | m;
  vals[i] = i;
}

int spatial_keys(const double4* p, uint32_t n, int D, const double lo[3], const double hi[3],
                 const uint32_t* prefix, unsigned long long* keys, uint32_t* vals,
                 hipStream_t st) {
  if (n == 0) return DT_OK;
  double inv[3];
  for (int k = 0; k < 3; k++) {
    double w = hi[k] - lo[k];
    inv[k] = w > 0 ? 1.0 / w : 0.0;
  }
  hipLaunchKernelGGL(k_spatial_keys, dim3((n + 255) / 256), dim3(256), 0, st, p, n, D,
                     make_double3(lo[0], lo[1], lo[2]), make_double3(inv[0], inv[1], inv[2]),
                     prefix, keys, vals);
  DT_HIP(hipGetLastError());
  return DT_OK;
}

}  // namespace dtk
