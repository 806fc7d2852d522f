// Divide step on the GPU.
//
// Sample-based divide (paper, Algorithm 2):
//   1. choose eta(n) points uniformly at random without replacement -- the
//      eta points with the smallest keys splitmix64(seed ^ id*golden), ties
//      by id (a histogram of the top 16 key bits finds the threshold bucket;
//      its few members are ordered exactly);
//   2. triangulate the sample (the batched local-DT kernels, one set);
//   3. graph G = (sample, Delaunay edges, w) with the weights of the paper's
//      Table "weights", d = |v-w| / d*, d* = bounding-box diagonal;
//   4. balanced k-way partition of G, |V_i| <= (1+eps) ceil(|V|/k): a
//      recursive coordinate bisection of the sample (Morton-order chunks
//      when k is not a power of two), then label-propagation sweeps that
//      move vertices to the block they are most strongly connected to when
//      the gain is positive and the target block has room (proposals into a
//      block are ranked by gain, then vertex id, so the result does not
//      depend on thread timing);
//   5. every point gets the block of its nearest sample point, key
//      (fl(d^2), sample id) with d^2 = ((dx dx + dy dy) + dz dz) rounded
//      after each operation; the search visits grid shells around the point
//      and stops once no unvisited cell can hold a closer sample, with a
//      margin far above the rounding error of d^2, so the result is the
//      exact argmin of the key.
// kd divide (Section "Recursive Bisection", the cyclic scheme): log2 k
// levels; at level l every block is split at the median of coordinate
// l mod D, the lower half being the floor(m/2) smallest (coordinate, id).
#include <math.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "dt_common.hpp"
#include "dt_internal.hpp"
#include "dt_prims.hpp"
#include "dt_grid.hpp"
#include "dt_stages.hpp"

namespace dtk {

constexpr int DB = 256;
static inline uint32_t dblocks(uint64_t n) { return (uint32_t)((n + DB - 1) / DB); }

__device__ __forceinline__ unsigned long long splitmix64(unsigned long long z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__device__ __forceinline__ unsigned long long sample_key(unsigned long long seed, uint32_t id) {
  return splitmix64(seed ^ ((unsigned long long)id * 0x9E3779B97F4A7C15ull));
}

// ------------------------------------------------------------ 1. sample
__global__ void k_sample_hist(uint32_t n, unsigned long long seed, uint32_t* hist) {
  uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  atomicAdd(&hist[sample_key(seed, i) >> 48], 1u);
}

__global__ void k_sample_mark(uint32_t n, unsigned long long seed, uint32_t thr, uint32_t* flag,
                              unsigned long long* cand, uint32_t* ncand, uint32_t cap) {
  uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  unsigned long long k = sample_key(seed, i);
  uint32_t top = (uint32_t)(k >> 48);
  flag[i] = top < thr ? 1u : 0u;
  if (top == thr) {
    uint32_t s = atomicAdd(ncand, 1u);
    if (s < cap) {
      cand[2 * s] = k;
      cand[2 * s + 1] = i;
    }
  }
}

__global__ void k_set_flags(const uint32_t* idx, uint32_t m, uint32_t* flag) {
  uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) flag[idx[i]] = 1u;
}

int select_sample(uint32_t n, uint32_t eta, uint64_t seed, DevBuf& sid, hipStream_t st) {
  DevBuf hist, flag, cand, ncand;
  DT_TRY(hist.alloc(65536 * 4));
  DT_TRY(flag.alloc((size_t)n * 4));
  DT_HIP(hipMemsetAsync(hist.p, 0, 65536 * 4, st));
  hipLaunchKernelGGL(k_sample_hist, dim3(dblocks(n)), dim3(DB), 0, st, n,
                     (unsigned long long)seed, hist.as<uint32_t>());
  DT_HIP(hipGetLastError());
  std::vector<uint32_t> h(65536);
  DT_HIP(hipMemcpyAsync(h.data(), hist.p, 65536 * 4, hipMemcpyDeviceToHost, st));
  DT_HIP(hipStreamSynchronize(st));
  uint32_t thr = 0, below = 0;
  while (thr < 65536 && below + h[thr] < eta) below += h[thr++];
  if (thr >= 65536) thr = 65535;
  uint32_t cap = h[thr] + 16;
  DT_TRY(cand.alloc((size_t)cap * 16));
  DT_TRY(ncand.alloc(4));
  DT_HIP(hipMemsetAsync(ncand.p, 0, 4, st));
  hipLaunchKernelGGL(k_sample_mark, dim3(dblocks(n)), dim3(DB), 0, st, n,
                     (unsigned long long)seed, thr, flag.as<uint32_t>(),
                     cand.as<unsigned long long>(), ncand.as<uint32_t>(), cap);
  DT_HIP(hipGetLastError());
  uint32_t nc = 0;
  DT_HIP(hipMemcpyAsync(&nc, ncand.p, 4, hipMemcpyDeviceToHost, st));
  DT_HIP(hipStreamSynchronize(st));
  if (nc > cap) return DT_E_INTERNAL;
  std::vector<unsigned long long> c(2 * (size_t)nc);
  if (nc) DT_HIP(hipMemcpyAsync(c.data(), cand.p, (size_t)nc * 16, hipMemcpyDeviceToHost, st));
  DT_HIP(hipStreamSynchronize(st));
  std::vector<std::pair<unsigned long long, uint32_t>> v(nc);
  for (uint32_t i = 0; i < nc; i++) v[i] = {c[2 * i], (uint32_t)c[2 * i + 1]};
  std::sort(v.begin(), v.end());
  uint32_t need = eta - below;
  if (need > nc) return DT_E_INTERNAL;
  std::vector<uint32_t> pick(need);
  for (uint32_t i = 0; i < need; i++) pick[i] = v[i].second;
  if (need) {
    DevBuf dp;
    DT_TRY(dp.alloc((size_t)need * 4));
    DT_HIP(hipMemcpyAsync(dp.p, pick.data(), (size_t)need * 4, hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_set_flags, dim3(dblocks(need)), dim3(DB), 0, st, dp.as<uint32_t>(), need,
                       flag.as<uint32_t>());
    DT_HIP(hipGetLastError());
    DT_HIP(hipStreamSynchronize(st));
  }
  uint32_t cnt = 0;
  DT_TRY(compact_indices(flag.as<uint32_t>(), n, sid, &cnt, st));
  if (cnt != eta) return DT_E_INTERNAL;
  return DT_OK;
}

__global__ void k_gather_pts(const double4* P, const uint32_t* idx, uint32_t m, double4* out) {
  uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) out[i] = P[idx[i]];
}

int gather_points(const double4* P, const uint32_t* idx, uint32_t m, double4* out,
                  hipStream_t st) {
  if (m == 0) return DT_OK;
  hipLaunchKernelGGL(k_gather_pts, dim3(dblocks(m)), dim3(DB), 0, st, P, idx, m, out);
  DT_HIP(hipGetLastError());
  return DT_OK;
}

int spatial_sort(DevBuf& pts, uint32_t n, int D, const double lo[3], const double hi[3],
                 const uint32_t* prefix, int prefix_bits, hipStream_t st) {
  if (n < 2) return DT_OK;
  DevBuf keys, order, sorted;
  DT_TRY(keys.alloc((size_t)n * 8));
  DT_TRY(order.alloc((size_t)n * 4));
  DT_TRY(sorted.alloc((size_t)n * sizeof(double4)));
  DT_TRY(spatial_keys(pts.as<double4>(), n, D, lo, hi, prefix, keys.as<unsigned long long>(),
                      order.as<uint32_t>(), st));
  DT_TRY(radix_sort_pairs(keys.as<unsigned long long>(), order.as<uint32_t>(), n,
                          (prefix ? prefix_bits : 0) + MORTON_BITS, st));
  DT_TRY(gather_points(pts.as<double4>(), order.as<uint32_t>(), n, sorted.as<double4>(), st));
  pts = std::move(sorted);
  return DT_OK;
}

// ------------------------------------------------------------ 3. graph
// Unique Delaunay edges of the sample triangulation through an
// open-addressing set keyed by (u << 32 | v), u < v (sample-local ids).
__global__ void k_edges(const Cell* cells, uint32_t ncells, int D,
                        unsigned long long* table, uint32_t tmask, uint32_t* elist,
                        uint32_t* ecount, uint32_t ecap) {
  uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncells || cells[c].fwd != ALIVE) return;
  uint4 v4 = cells[c].v;
  uint32_t v[4] = {v4.x, v4.y, v4.z, v4.w};
  for (int i = 0; i <= D; i++)
    for (int j = i + 1; j <= D; j++) {
      uint32_t a = v[i], b = v[j];
      if (a == INF_V || b == INF_V) continue;
      if (a > b) { uint32_t t = a; a = b; b = t; }
      unsigned long long key = ((unsigned long long)a << 32) | b;
      uint32_t h = (uint32_t)((key * 0x9E3779B97F4A7C15ull) >> 32);
      for (uint32_t pr = 0; pr <= tmask; pr++) {
        uint32_t s = (h + pr) & tmask;
        unsigned long long old = atomicCAS(&table[s], ~0ull, key);
        if (old == ~0ull) {
          uint32_t e = atomicAdd(ecount, 1u);
          if (e < ecap) {
            elist[2 * e] = a;
            elist[2 * e + 1] = b;
          }
          break;
        }
        if (old == key) break;
      }
    }
}

__global__ void k_degree(const uint32_t* elist, uint32_t m, uint32_t* deg) {
  uint32_t e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m) return;
  atomicAdd(&deg[elist[2 * e]], 1u);
  atomicAdd(&deg[elist[2 * e + 1]], 1u);
}

__global__ void k_fill_adj(const uint32_t* elist, uint32_t m, const uint32_t* off, uint32_t* cur,
                           uint32_t* adj) {
  uint32_t e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m) return;
  uint32_t a = elist[2 * e], b = elist[2 * e + 1];
  adj[off[a] + atomicAdd(&cur[a], 1u)] = b;
  adj[off[b] + atomicAdd(&cur[b], 1u)] = a;
}

// Sort each adjacency list (deterministic summation order) and compute the
// edge weights.  d* = bounding-box diagonal of the whole input.
__global__ void k_adj_weights(const double4* S, uint32_t eta, const uint32_t* off, uint32_t* adj,
                              double* w, int kind, double dstar) {
  uint32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= eta) return;
  uint32_t a = off[v], b = off[v + 1];
  for (uint32_t i = a + 1; i < b; i++)
    for (uint32_t j = i; j > a && adj[j] < adj[j - 1]; j--) {
      uint32_t t = adj[j]; adj[j] = adj[j - 1]; adj[j - 1] = t;
    }
  double4 p = S[v];
  for (uint32_t i = a; i < b; i++) {
    double4 q = S[adj[i]];
    double dx = p.x - q.x, dy = p.y - q.y, dz = p.z - q.z;
    double d = sqrt(dx * dx + dy * dy + dz * dz) / dstar;
    if (d < 1e-300) d = 1e-300;
    double x;
    switch (kind) {
      case DT_WEIGHT_CONST: x = 1.0; break;
      case DT_WEIGHT_INVERSE: x = 1.0 / d; break;
      case DT_WEIGHT_LINEAR: x = 1.0 - d; break;
      default: x = -log(d); break;
    }
    w[i] = x;
  }
}

// ------------------------------------------------------------ 4. partition
__device__ __forceinline__ unsigned long long spread3(unsigned long long x) {
  x &= 0x1FFFFFull;
  x = (x | (x << 32)) & 0x1F00000000FFFFull;
  x = (x | (x << 16)) & 0x1F0000FF0000FFull;
  x = (x | (x << 8)) & 0x100F00F00F00F00Full;
  x = (x | (x << 4)) & 0x10C30C30C30C30C3ull;
  x = (x | (x << 2)) & 0x1249249249249249ull;
  return x;
}
__device__ __forceinline__ unsigned long long spread2(unsigned long long x) {
  x &= 0xFFFFFFFFull;
  x = (x | (x << 16)) & 0x0000FFFF0000FFFFull;
  x = (x | (x << 8)) & 0x00FF00FF00FF00FFull;
  x = (x | (x << 4)) & 0x0F0F0F0F0F0F0F0Full;
  x = (x | (x << 2)) & 0x3333333333333333ull;
  x = (x | (x << 1)) & 0x5555555555555555ull;
  return x;
}

__global__ void k_morton(const double4* S, uint32_t m, int D, double3 lo, double3 inv,
                         unsigned long long* keys, uint32_t* vals) {
  uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  double4 p = S[i];
  double scale = (D == 3) ? 2097151.0 : 4294967295.0;
  unsigned long long x = (unsigned long long)(fmin(fmax((p.x - lo.x) * inv.x, 0.0), 1.0) * scale);
  unsigned long long y = (unsigned long long)(fmin(fmax((p.y - lo.y) * inv.y, 0.0), 1.0) * scale);
  unsigned long long z = (unsigned long long)(fmin(fmax((p.z - lo.z) * inv.z, 0.0), 1.0) * scale);
  keys[i] = (D == 3) ? (spread3(x) | (spread3(y) << 1) | (spread3(z) << 2))
                     : (spread2(x) | (spread2(y) << 1));
  vals[i] = i;
}

__global__ void k_init_blocks(const uint32_t* order, uint32_t m, uint32_t k, uint32_t* part) {
  uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= m) return;
  part[order[r]] = (uint32_t)(((unsigned long long)r * k) / m);
}

__device__ __forceinline__ uint32_t mix32(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7FEB352Du;
  x ^= x >> 15;
  x *= 0x846CA68Bu;
  x ^= x >> 16;
  return x;
}

// Proposal: move v to the neighbouring block with the largest connection
// weight if that beats the current block.  Half the vertices (by a hash
// alternating with the sweep) may move per sweep to damp oscillation.
// One wavefront per vertex: lane i holds neighbour i's block and weight in
// LDS, and sums the weights of the lanes with its block in neighbour order
// (the same order for every lane of that block); a reduction picks the
// largest sum, ties to the smaller block.  Degrees above 64 are summed by
// lane 0 in the same order.
constexpr uint32_t LP_WAVES = 4;   // vertices per 256-thread block

__global__ __launch_bounds__(64 * LP_WAVES) void k_lp_propose(
    uint32_t eta, const uint32_t* off, const uint32_t* adj, const double* w,
    const uint32_t* part, uint32_t sweep, uint32_t* pblock, double* pgain, uint32_t* pcount) {
  __shared__ uint32_t s_b[LP_WAVES][64];
  __shared__ double s_w[LP_WAVES][64];
  const uint32_t lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const uint32_t v = blockIdx.x * LP_WAVES + wv;
  if (v >= eta) return;   // whole wavefronts leave together
  if (lane == 0) pblock[v] = DONE;
  if (((mix32(v) + sweep) & 1u) != 0) return;
  const uint32_t a = off[v], b = off[v + 1], d = b - a;
  const uint32_t cur = part[v];
  double c = 0.0;          // this lane's block sum
  uint32_t pb = DONE;      // this lane's block
  double own = 0.0;
  if (d <= 64) {
    if (lane < d) {
      pb = part[adj[a + lane]];
      s_b[wv][lane] = pb;
      s_w[wv][lane] = w[a + lane];
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    for (uint32_t j = 0; j < d; j++)
      if (s_b[wv][j] == cur) own += s_w[wv][j];
    if (lane < d && pb != cur)
      for (uint32_t j = 0; j < d; j++)
        if (s_b[wv][j] == pb) c += s_w[wv][j];
  } else if (lane == 0) {
    // long lists: lane 0 alone, same sums, first occurrences in order
    for (uint32_t i = a; i < b; i++)
      if (part[adj[i]] == cur) own += w[i];
    double bestw = 0.0;
    uint32_t best = DONE;
    for (uint32_t i = a; i < b; i++) {
      const uint32_t q = part[adj[i]];
      if (q == cur) continue;
      bool seen = false;
      for (uint32_t j = a; j < i; j++)
        if (part[adj[j]] == q) { seen = true; break; }
      if (seen) continue;
      double t = 0.0;
      for (uint32_t j = i; j < b; j++)
        if (part[adj[j]] == q) t += w[j];
      if (t > bestw || (t == bestw && best != DONE && q < best)) { bestw = t; best = q; }
    }
    c = bestw;
    pb = best;
  }
  // largest sum, ties to the smaller block; a sum must be positive
  if (!(c > 0.0)) pb = DONE;
  for (int o = 32; o > 0; o >>= 1) {
    const double oc = __shfl_xor(c, o, 64);
    const uint32_t ob = __shfl_xor(pb, o, 64);
    if (ob != DONE && (pb == DONE || oc > c || (oc == c && ob < pb))) { c = oc; pb = ob; }
  }
  if (lane == 0 && pb != DONE && c - own > 1e-12 * (c + own + 1.0)) {
    pblock[v] = pb;
    pgain[v] = c - own;
    atomicAdd(&pcount[pb], 1u);
  }
}

__global__ void k_lp_list(uint32_t eta, const uint32_t* pblock, const uint32_t* poff,
                          uint32_t* pcur, uint32_t* plist) {
  uint32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= eta) return;
  uint32_t b = pblock[v];
  if (b == DONE) return;
  plist[poff[b] + atomicAdd(&pcur[b], 1u)] = v;
}

// Pair exchanges between full blocks.  A proposal A -> B whose block B has
// no room cannot move alone; it is paired with the proposal B -> A of the
// same rank (gains descending, ties to the smaller vertex), and the pair
// swaps when the exchange lowers the cut: g_v + g_u - 2 w(u, v) > 0, the
// exchange gain of Kernighan and Lin.  Block sizes do not change, so the
// balance bound holds with no room at all (8 samples per block at the
// default sample size and k = 256).  Decided from the sweep's starting
// blocks; k_lp_accept applies the swaps.
__global__ void k_lp_swap(uint32_t eta, const uint32_t* off, const uint32_t* adj, const double* w,
                          const uint32_t* part, const uint32_t* pblock, const double* pgain,
                          const uint32_t* poff, const uint32_t* pcount, const uint32_t* plist,
                          const int* size, int lmax, const int* lmax_of, uint32_t* pswap) {
  uint32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= eta) return;
  uint32_t swap = 0;
  const uint32_t b = pblock[v];
  if (b != DONE) {
    const uint32_t a = part[v];
    const int room_b = (lmax_of ? lmax_of[b] : lmax) - size[b];
    const int room_a = (lmax_of ? lmax_of[a] : lmax) - size[a];
    if (room_a <= 0 && room_b <= 0) {
      const double g = pgain[v];
      uint32_t rank = 0;
      for (uint32_t i = poff[b]; i < poff[b] + pcount[b]; i++) {
        const uint32_t x = plist[i];
        if (part[x] != a) continue;
        const double gx = pgain[x];
        if (gx > g || (gx == g && x < v)) rank++;
      }
      // the partner: rank-th proposal B -> A
      uint32_t u = DONE;
      double gu = 0.0;
      for (uint32_t i = poff[a]; i < poff[a] + pcount[a] && u == DONE; i++) {
        const uint32_t x = plist[i];
        if (part[x] != b) continue;
        const double gx = pgain[x];
        uint32_t rx = 0;
        for (uint32_t j = poff[a]; j < poff[a] + pcount[a]; j++) {
          const uint32_t y = plist[j];
          if (part[y] != b) continue;
          const double gy = pgain[y];
          if (gy > gx || (gy == gx && y < x)) rx++;
        }
        if (rx == rank) { u = x; gu = gx; }
      }
      if (u != DONE) {
        double wuv = 0.0;
        for (uint32_t i = off[v]; i < off[v + 1]; i++)
          if (adj[i] == u) wuv += w[i];
        const double sum = g + gu, cost = 2.0 * wuv;
        if (sum - cost > 1e-12 * (sum + cost + 1.0)) swap = 1;
      }
    }
  }
  pswap[v] = swap;
}

// Accept the best proposals into each block up to its free capacity
// (capacity measured at the start of the sweep, so the bound always holds),
// and the pair exchanges decided by k_lp_swap.
__global__ void k_lp_accept(uint32_t eta, const uint32_t* pblock, const double* pgain,
                            const uint32_t* poff, const uint32_t* pcount, const uint32_t* plist,
                            const int* size, int lmax, const int* lmax_of, const uint32_t* pswap,
                            uint32_t* part, int* delta) {
  uint32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= eta) return;
  uint32_t b = pblock[v];
  if (b == DONE) return;
  if (pswap && pswap[v]) {
    part[v] = b;
    return;
  }
  int room = (lmax_of ? lmax_of[b] : lmax) - size[b];
  if (room <= 0) return;
  double g = pgain[v];
  uint32_t rank = 0;
  for (uint32_t i = poff[b]; i < poff[b] + pcount[b]; i++) {
    uint32_t u = plist[i];
    double gu = pgain[u];
    if (gu > g || (gu == g && u < v)) rank++;
  }
  if ((int)rank < room) {
    atomicAdd(&delta[part[v]], -1);
    atomicAdd(&delta[b], 1);
    part[v] = b;
  }
}

__global__ void k_apply_delta(uint32_t k, int* size, int* delta) {
  uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= k) return;
  size[b] += delta[b];
  delta[b] = 0;
}

__global__ void k_cut(uint32_t eta, const uint32_t* off, const uint32_t* adj, const double* w,
                      const uint32_t* part, double* cut) {
  uint32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= eta) return;
  double c = 0.0;
  for (uint32_t i = off[v]; i < off[v + 1]; i++)
    if (adj[i] > v && part[adj[i]] != part[v]) c += w[i];
  if (c != 0.0) atomicAdd(cut, c);
}

__global__ void k_count_u32(const uint32_t* x, uint32_t m, uint32_t* cnt) {
  uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) atomicAdd(&cnt[x[i]], 1u);
}

// the same count with a per-block table in LDS (few keys, many items):
// one global atomic per key and block instead of one per item
constexpr uint32_t COUNT_LDS_KEYS = 4096;
__global__ __launch_bounds__(256) void k_count_u32_lds(const uint32_t* x, uint32_t m, uint32_t k,
                                                       uint32_t* cnt) {
  __shared__ uint32_t s_c[COUNT_LDS_KEYS];
  for (uint32_t j = threadIdx.x; j < k; j += blockDim.x) s_c[j] = 0;
  __syncthreads();
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += gridDim.x * blockDim.x)
    atomicAdd(&s_c[x[i]], 1u);
  __syncthreads();
  for (uint32_t j = threadIdx.x; j < k; j += blockDim.x)
    if (s_c[j]) atomicAdd(&cnt[j], s_c[j]);
}

int sample_graph(const double4* S, uint32_t eta, int D, const CellPool& pool, int weight,
                 double dstar, DevBuf& goff, DevBuf& gadj, DevBuf& gw, hipStream_t st) {
  // edges
  uint32_t ncells = pool.ncells;
  uint32_t tsize = 1024;
  while (tsize < (uint64_t)ncells * (D == 3 ? 4 : 3)) tsize <<= 1;
  DevBuf table, elist, ecount;
  DT_TRY(table.alloc((size_t)tsize * 8));
  uint32_t ecap = tsize;
  DT_TRY(elist.alloc((size_t)ecap * 8));
  DT_TRY(ecount.alloc(4));
  DT_HIP(hipMemsetAsync(table.p, 0xFF, (size_t)tsize * 8, st));
  DT_HIP(hipMemsetAsync(ecount.p, 0, 4, st));
  if (ncells)
    hipLaunchKernelGGL(k_edges, dim3(dblocks(ncells)), dim3(DB), 0, st, pool.cells.as<Cell>(),
                       ncells, D, table.as<unsigned long long>(), tsize - 1, elist.as<uint32_t>(),
                       ecount.as<uint32_t>(), ecap);
  DT_HIP(hipGetLastError());
  uint32_t m = 0;
  DT_HIP(hipMemcpyAsync(&m, ecount.p, 4, hipMemcpyDeviceToHost, st));
  DT_HIP(hipStreamSynchronize(st));
  if (m > ecap) return DT_E_INTERNAL;
  DevBuf deg, off, cur, adj, w;
  DT_TRY(deg.alloc((size_t)(eta + 1) * 4));
  DT_TRY(off.alloc((size_t)(eta + 1) * 4));
  DT_TRY(cur.alloc((size_t)(eta + 1) * 4));
  DT_TRY(adj.alloc((size_t)2 * m * 4 + 4));
  DT_TRY(w.alloc((size_t)2 * m * 8 + 8));
  DT_HIP(hipMemsetAsync(deg.p, 0, (size_t)(eta + 1) * 4, st));
  DT_HIP(hipMemsetAsync(cur.p, 0, (size_t)(eta + 1) * 4, st));
  if (m)
    hipLaunchKernelGGL(k_degree, dim3(dblocks(m)), dim3(DB), 0, st, elist.as<uint32_t>(), m,
                       deg.as<uint32_t>());
  DT_TRY(exclusive_scan(deg.as<uint32_t>(), off.as<uint32_t>(), eta + 1, st));
  if (m)
    hipLaunchKernelGGL(k_fill_adj, dim3(dblocks(m)), dim3(DB), 0, st, elist.as<uint32_t>(), m,
                       off.as<uint32_t>(), cur.as<uint32_t>(), adj.as<uint32_t>());
  if (!(dstar > 0)) dstar = 1.0;
  hipLaunchKernelGGL(k_adj_weights, dim3(dblocks(eta)), dim3(DB), 0, st, S, eta,
                     off.as<uint32_t>(), adj.as<uint32_t>(), w.as<double>(), weight, dstar);
  DT_HIP(hipGetLastError());
  goff = std::move(off);
  gadj = std::move(adj);
  gw = std::move(w);
  return DT_OK;
}

int refine_partition(uint32_t eta, const uint32_t* goff, const uint32_t* gadj, const double* gw,
                     uint32_t* part, uint32_t k, int lmax, const int* lmax_of, int iters,
                     bool swaps, hipStream_t st) {
  DevBuf size, delta, pblock, pgain, pcount, poff, pcur, plist, pswap;
  DT_TRY(size.alloc((size_t)k * 4));
  DT_TRY(delta.alloc((size_t)k * 4));
  DT_TRY(pblock.alloc((size_t)eta * 4));
  DT_TRY(pgain.alloc((size_t)eta * 8));
  DT_TRY(pcount.alloc((size_t)(k + 1) * 4));
  DT_TRY(poff.alloc((size_t)(k + 1) * 4));
  DT_TRY(pcur.alloc((size_t)(k + 1) * 4));
  DT_TRY(plist.alloc((size_t)eta * 4));
  if (swaps) DT_TRY(pswap.alloc((size_t)eta * 4));
  DT_HIP(hipMemsetAsync(size.p, 0, (size_t)k * 4, st));
  DT_HIP(hipMemsetAsync(delta.p, 0, (size_t)k * 4, st));
  hipLaunchKernelGGL(k_count_u32, dim3(dblocks(eta)), dim3(DB), 0, st, part, eta,
                     (uint32_t*)size.p);
  for (int it = 0; it < iters; it++) {
    DT_HIP(hipMemsetAsync(pcount.p, 0, (size_t)(k + 1) * 4, st));
    DT_HIP(hipMemsetAsync(pcur.p, 0, (size_t)(k + 1) * 4, st));
    hipLaunchKernelGGL(k_lp_propose, dim3((eta + LP_WAVES - 1) / LP_WAVES), dim3(64 * LP_WAVES), 0,
                       st, eta, goff, gadj, gw, part, (uint32_t)it, pblock.as<uint32_t>(),
                       pgain.as<double>(), pcount.as<uint32_t>());
    DT_TRY(exclusive_scan(pcount.as<uint32_t>(), poff.as<uint32_t>(), k + 1, st));
    hipLaunchKernelGGL(k_lp_list, dim3(dblocks(eta)), dim3(DB), 0, st, eta,
                       pblock.as<uint32_t>(), poff.as<uint32_t>(), pcur.as<uint32_t>(),
                       plist.as<uint32_t>());
    if (swaps)
      hipLaunchKernelGGL(k_lp_swap, dim3(dblocks(eta)), dim3(DB), 0, st, eta, goff, gadj, gw,
                         part, pblock.as<uint32_t>(), pgain.as<double>(), poff.as<uint32_t>(),
                         pcount.as<uint32_t>(), plist.as<uint32_t>(), (const int*)size.p, lmax,
                         lmax_of, pswap.as<uint32_t>());
    hipLaunchKernelGGL(k_lp_accept, dim3(dblocks(eta)), dim3(DB), 0, st, eta,
                       pblock.as<uint32_t>(), pgain.as<double>(), poff.as<uint32_t>(),
                       pcount.as<uint32_t>(), plist.as<uint32_t>(), (const int*)size.p, lmax,
                       lmax_of, swaps ? pswap.as<uint32_t>() : nullptr, part, (int*)delta.p);
    hipLaunchKernelGGL(k_apply_delta, dim3(dblocks(k)), dim3(DB), 0, st, k, (int*)size.p,
                       (int*)delta.p);
    DT_HIP(hipGetLastError());
  }
  // the buffers are freed on return
  DT_HIP(hipStreamSynchronize(st));
  return DT_OK;
}

int partition_sample(const double4* S, uint32_t eta, int D, const CellPool& pool, uint32_t k,
                     const dt_options& o, const double lo[3], const double hi[3],
                     DevBuf& part, double* cut, DevBuf& goff, DevBuf& gadj, DevBuf& gw,
                     hipStream_t st) {
  double dx = hi[0] - lo[0], dy = hi[1] - lo[1], dz = hi[2] - lo[2];
  double dstar = sqrt(dx * dx + dy * dy + dz * dz);
  DT_TRY(sample_graph(S, eta, D, pool, o.weight, dstar, goff, gadj, gw, st));
  // initial blocks: recursive coordinate bisection of the sample (compact,
  // balanced to +-1 vertex when k is a power of two); otherwise k equal
  // chunks of the sample in Morton order
  if ((k & (k - 1)) == 0) {
    DevBuf boxes_unused;
    DT_TRY(kd_divide(S, eta, D, k, part, boxes_unused, st));
  } else {
    DevBuf mk, mv;
    DT_TRY(mk.alloc((size_t)eta * 8));
    DT_TRY(mv.alloc((size_t)eta * 4));
    double3 dlo = make_double3(lo[0], lo[1], lo[2]);
    double3 inv = make_double3(dx > 0 ? 1.0 / dx : 0.0, dy > 0 ? 1.0 / dy : 0.0,
                               dz > 0 ? 1.0 / dz : 0.0);
    hipLaunchKernelGGL(k_morton, dim3(dblocks(eta)), dim3(DB), 0, st, S, eta, D, dlo, inv,
                       mk.as<unsigned long long>(), mv.as<uint32_t>());
    DT_HIP(hipGetLastError());
    DT_TRY(radix_sort_pairs(mk.as<unsigned long long>(), mv.as<uint32_t>(), eta, 64, st));
    DT_TRY(part.alloc((size_t)eta * 4));
    hipLaunchKernelGGL(k_init_blocks, dim3(dblocks(eta)), dim3(DB), 0, st, mv.as<uint32_t>(), eta,
                       k, part.as<uint32_t>());
  }
  // label propagation under the balance bound
  uint32_t avg = (eta + k - 1) / k;
  int lmax = (int)floor((1.0 + o.eps) * (double)avg + 1e-9);
  DT_TRY(refine_partition(eta, goff.as<uint32_t>(), gadj.as<uint32_t>(), gw.as<double>(),
                          part.as<uint32_t>(), k, lmax, nullptr, o.refine_iters,
                          o.refine_swaps == 0, st));
  DevBuf dcut;
  DT_TRY(dcut.alloc(8));
  DT_HIP(hipMemsetAsync(dcut.p, 0, 8, st));
  hipLaunchKernelGGL(k_cut, dim3(dblocks(eta)), dim3(DB), 0, st, eta, goff.as<uint32_t>(),
                     gadj.as<uint32_t>(), gw.as<double>(), part.as<uint32_t>(), dcut.as<double>());
  DT_HIP(hipGetLastError());
  DT_HIP(hipMemcpyAsync(cut, dcut.p, 8, hipMemcpyDeviceToHost, st));
  DT_HIP(hipStreamSynchronize(st));
  return DT_OK;
}

// ------------------------------------------------------------ 5. assign
// start-grid cells per sample for the descent of the assignment
constexpr double AW_CELLS = 32.0;
static Grid make_grid(const double lo[3], const double hi[3], int D, double cells_target) {
  Grid G;
  double vol = 1.0;
  int nd = 0;
  for (int k = 0; k < D; k++) {
    double e = hi[k] - lo[k];
    if (e > 0) { vol *= e; nd++; }
  }
  double h = (nd > 0) ? pow(vol / (cells_target > 1 ? cells_target : 1), 1.0 / nd) : 1.0;
  if (!(h > 0)) h = 1.0;
  for (int k = 0; k < 3; k++) {
    G.lo[k] = lo[k];
    double e = (k < D) ? hi[k] - lo[k] : 0.0;
    long g = (long)floor(e / h) + 1;
    if (g < 1) g = 1;
    if (g > 4096) g = 4096;
    G.g[k] = (k < D) ? (int)g : 1;
  }
  G.h = h;
  return G;
}

__global__ void k_grid_count(const double4* S, uint32_t m, Grid G, uint32_t* cnt, uint32_t* cellof) {
  uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  double4 p = S[i];
  int cx = cell_coord(p.x, G.lo[0], G.h, G.g[0]);
  int cy = cell_coord(p.y, G.lo[1], G.h, G.g[1]);
  int cz = cell_coord(p.z, G.lo[2], G.h, G.g[2]);
  uint32_t c = ((uint32_t)cz * G.g[1] + cy) * G.g[0] + cx;
  cellof[i] = c;
  atomicAdd(&cnt[c], 1u);
}

__global__ void k_grid_fill(uint32_t m, const uint32_t* cellof, const uint32_t* start, uint32_t* cur,
                            uint32_t* items) {
  uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  uint32_t c = cellof[i];
  items[start[c] + atomicAdd(&cur[c], 1u)] = i;
}

// Start sample of every cell of a finer grid: the sample nearest to the
// cell's centre.
__global__ void k_start_cells(const double4* S, const uint32_t* start, const uint32_t* items,
                              Grid G, Grid F, uint32_t nf, uint32_t* first) {
  const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nf) return;
  const uint32_t x = c % F.g[0], y = (c / F.g[0]) % F.g[1], z = c / (F.g[0] * F.g[1]);
  double d2;
  first[c] = grid_nearest(S, start, items, G, F.lo[0] + (x + 0.5) * F.h,
                          F.lo[1] + (y + 0.5) * F.h, F.lo[2] + (z + 0.5) * F.h, &d2);
}

// Nearest sample (Algorithm 2: every point joins the block of its nearest
// sample point) by descent over the sample's Delaunay graph, exact under
// the key (fl(d^2), id).  The squared distance to x, taken over the sample
// points, is the lifted height less an affine function, and the Delaunay
// triangulation is the lower hull of the lifted points; so every set
// {s : |x - s|^2 <= L} is connected through Delaunay edges, and a sample no
// neighbour beats is the nearest.  With rounding, the descent stops at a
// sample t that no neighbour beats under the key; every sample whose key
// could be below t's lies in {|x - s|^2 <= fl(d_t^2)(1 + 1e-9)}, which is
// connected and holds t, so the search through that set finds the least
// key.  When no neighbour of t is in it, t is the answer.  A long descent
// or a large near-tie set falls back to the grid search.
constexpr int AW_CAP = 16;
constexpr int AW_STEPS = 256;

__global__ __launch_bounds__(DB) void k_assign_walk(const double4* P, uint32_t n, const double4* S,
                                                    const uint32_t* goff, const uint32_t* gadj,
                                                    Grid F, const uint32_t* first,
                                                    const uint32_t* start, const uint32_t* items,
                                                    Grid G, const uint32_t* part, uint32_t* pid,
                                                    uint32_t* nearest) {
  __shared__ uint32_t s_vis[AW_CAP * DB];
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint32_t* vis = s_vis + threadIdx.x;
  const double4 p = P[i];
  const uint32_t fc = ((uint32_t)cell_coord(p.z, F.lo[2], F.h, F.g[2]) * F.g[1] +
                       cell_coord(p.y, F.lo[1], F.h, F.g[1])) * F.g[0] +
                      cell_coord(p.x, F.lo[0], F.h, F.g[0]);
  uint32_t t = first[fc];
  double4 tp = S[t];
  double bd;
  {
    const double dx = p.x - tp.x, dy = p.y - tp.y, dz = p.z - tp.z;
    bd = (dx * dx + dy * dy) + dz * dz;
  }
  long long bid = __double_as_longlong(tp.w);
  bool fallback = true, ties = false;
  for (int step = 0; step < AW_STEPS; step++) {
    uint32_t best = t;
    double nd = bd, dmin = INFINITY;
    long long nid = bid;
    const uint32_t a = goff[t], b = goff[t + 1];
    for (uint32_t j = a; j < b; j++) {
      const uint32_t w = gadj[j];
      const double4 q = S[w];
      const double dx = p.x - q.x, dy = p.y - q.y, dz = p.z - q.z;
      const double d = (dx * dx + dy * dy) + dz * dz;
      const long long id = __double_as_longlong(q.w);
      dmin = fmin(dmin, d);
      if (d < nd || (d == nd && id < nid)) { best = w; nd = d; nid = id; }
    }
    if (best == t) {
      fallback = false;
      ties = dmin <= bd * (1.0 + 1e-9);
      break;
    }
    t = best;
    bd = nd;
    bid = nid;
  }
  if (!fallback && ties) {
    // the near-tie set around t
    const double lim = bd * (1.0 + 1e-9);
    uint32_t bs = t;
    double kd = bd;
    long long kid = bid;
    int nv = 1, head = 0;
    vis[0] = t;
    while (head < nv && !fallback) {
      const uint32_t u = vis[(size_t)head++ * DB];
      const uint32_t a = goff[u], b = goff[u + 1];
      for (uint32_t j = a; j < b; j++) {
        const uint32_t w = gadj[j];
        bool seen = false;
        for (int k = 0; k < nv; k++) seen |= vis[(size_t)k * DB] == w;
        if (seen) continue;
        const double4 q = S[w];
        const double dx = p.x - q.x, dy = p.y - q.y, dz = p.z - q.z;
        const double d = (dx * dx + dy * dy) + dz * dz;
        if (!(d <= lim)) continue;
        if (nv == AW_CAP) { fallback = true; break; }
        vis[(size_t)nv++ * DB] = w;
        const long long id = __double_as_longlong(q.w);
        if (d < kd || (d == kd && id < kid)) { bs = w; kd = d; kid = id; }
      }
    }
    t = bs;
  }
  if (fallback) {
    double d2;
    t = grid_nearest(S, start, items, G, p.x, p.y, p.z, &d2);
  }
  nearest[i] = t;
  pid[i] = part[t];
}

int assign_points(const double4* P, uint32_t n, const double4* S, uint32_t eta, int D,
                  const uint32_t* part, const double lo[3], const double hi[3],
                  const uint32_t* goff, const uint32_t* gadj, DevBuf& pid,
                  DevBuf& nearest, SampleGrid& sg, hipStream_t st) {
  if (!goff || !gadj) return DT_E_INTERNAL;
  Grid G = make_grid(lo, hi, D, eta / 2.0);
  sg.G = G;
  uint32_t ncell = (uint32_t)G.g[0] * G.g[1] * G.g[2];
  DevBuf cnt, cur, cellof;
  DevBuf& start = sg.start;
  DevBuf& items = sg.items;
  DT_TRY(cnt.alloc((size_t)(ncell + 1) * 4));
  DT_TRY(start.alloc((size_t)(ncell + 1) * 4));
  DT_TRY(cur.alloc((size_t)(ncell + 1) * 4));
  DT_TRY(items.alloc((size_t)eta * 4));
  DT_TRY(cellof.alloc((size_t)eta * 4));
  DT_HIP(hipMemsetAsync(cnt.p, 0, (size_t)(ncell + 1) * 4, st));
  DT_HIP(hipMemsetAsync(cur.p, 0, (size_t)(ncell + 1) * 4, st));
  hipLaunchKernelGGL(k_grid_count, dim3(dblocks(eta)), dim3(DB), 0, st, S, eta, G,
                     cnt.as<uint32_t>(), cellof.as<uint32_t>());
  DT_TRY(exclusive_scan(cnt.as<uint32_t>(), start.as<uint32_t>(), ncell + 1, st));
  hipLaunchKernelGGL(k_grid_fill, dim3(dblocks(eta)), dim3(DB), 0, st, eta,
                     cellof.as<uint32_t>(), start.as<uint32_t>(), cur.as<uint32_t>(),
                     items.as<uint32_t>());
  DT_TRY(pid.alloc((size_t)n * 4));
  DT_TRY(nearest.alloc((size_t)n * 4));
  // start samples on a grid of about AW_CELLS cells per sample
  const Grid F = make_grid(lo, hi, D, eta * AW_CELLS);
  const uint32_t nf = (uint32_t)F.g[0] * F.g[1] * F.g[2];
  DevBuf first;
  DT_TRY(first.alloc((size_t)nf * 4));
  hipLaunchKernelGGL(k_start_cells, dim3(dblocks(nf)), dim3(DB), 0, st, S, start.as<uint32_t>(),
                     items.as<uint32_t>(), G, F, nf, first.as<uint32_t>());
  DT_PROF_BEGIN(DT_KERN_ASSIGN, st);
  hipLaunchKernelGGL(k_assign_walk, dim3(dblocks(n)), dim3(DB), 0, st, P, n, S, goff, gadj, F,
                     first.as<uint32_t>(), start.as<uint32_t>(), items.as<uint32_t>(), G, part,
                     pid.as<uint32_t>(), nearest.as<uint32_t>());
  DT_PROF_END(st);
  DT_HIP(hipGetLastError());
  DT_HIP(hipStreamSynchronize(st));
  return DT_OK;
}

// ------------------------------------------------------------ kd divide
__device__ __forceinline__ unsigned long long ord_bits(double x) {
  unsigned long long u = (unsigned long long)__double_as_longlong(x);
  return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}
__device__ __forceinline__ double from_ord_d(unsigned long long o) {
  const unsigned long long u = (o >> 63) ? (o & 0x7FFFFFFFFFFFFFFFull) : ~o;
  return __longlong_as_double((long long)u);
}

__global__ void k_kd_keys(const double4* P, uint32_t n, int dim, unsigned long long* keys,
                          uint32_t* vals) {
  uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double4 p = P[i];
  double x = dim == 0 ? p.x : (dim == 1 ? p.y : p.z);
  keys[i] = ord_bits(x);
  vals[i] = i;
}

__global__ void k_kd_segkeys(const uint32_t* vals, uint32_t n, const uint32_t* seg,
                             unsigned long long* keys) {
  uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < n) keys[j] = seg[vals[j]];
}

__global__ void k_kd_split(const unsigned long long* segk, const uint32_t* vals, uint32_t n,
                           const uint32_t* segoff, uint32_t* seg, const double4* P, int dim,
                           double* split) {
  uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  uint32_t s = (uint32_t)segk[j];
  uint32_t a = segoff[s], b = segoff[s + 1];
  uint32_t half = (b - a) / 2;
  seg[vals[j]] = 2 * s + ((j - a) >= half ? 1u : 0u);
  if (j - a == half) {
    // first element of the upper half: lower child x <= v, upper child x >= v
    double4 p = P[vals[j]];
    split[s] = dim == 0 ? p.x : (dim == 1 ? p.y : p.z);
  }
}

// ---- kd level by selection (instead of sorting): per segment, the
// element of rank floor(m/2) in (coordinate, id) order is found by a
// histogram of the coordinate over the candidates' extent, narrowed to the
// bin that holds the wanted rank until that bin is small, then an exact
// sort of that bin, then a comparison of every point with the element
// found.  The split is the one a full sort gives.  The bin of a coordinate
// is a monotone function of it, so equal coordinates share a bin, the
// order of the bins is the order of the coordinates, and the points of one
// bin are exactly those between its smallest and largest coordinate.
constexpr uint32_t KD_HIST = 16384;  // bins of all segments of one level
constexpr uint32_t KD_MINBINS = 64;
constexpr uint32_t KD_CAP = 4096;    // largest median bin sorted in LDS
constexpr uint32_t KD_MAXSEG = 1024; // segments with an LDS extent table
constexpr uint32_t KD_GRID = 1024;   // blocks of the streaming passes
constexpr int KD_NARROW = 4;         // narrowing passes before the sort

__device__ __forceinline__ double kd_coord(const double4& p, int dim) {
  return dim == 0 ? p.x : (dim == 1 ? p.y : p.z);
}

// bin of x among `bins` equal parts of the segment's candidate range
__device__ __forceinline__ uint32_t kd_bin(double x, const unsigned long long* cand, uint32_t s,
                                           uint32_t bins) {
  const double lo = from_ord_d(cand[2 * s]), hi = from_ord_d(cand[2 * s + 1]);
  const double w = hi - lo;
  if (!(w > 0)) return 0;
  const double t = (x - lo) / w * (double)bins;
  const int b = (int)t;
  return b < 0 ? 0u : (b >= (int)bins ? bins - 1 : (uint32_t)b);
}

// extent of the candidates of every active segment (those in its range,
// and, when narrowing, in its chosen bin): per-block table in LDS, then
// one global atomic per segment and block
__global__ __launch_bounds__(256) void k_kd_extent(const double4* P, uint32_t n, int dim,
                                                   const uint32_t* seg, uint32_t nseg,
                                                   const unsigned long long* cand,
                                                   const uint32_t* act, const uint32_t* info,
                                                   uint32_t bins, int narrow,
                                                   unsigned long long* out) {
  __shared__ unsigned long long s_lo[KD_MAXSEG], s_hi[KD_MAXSEG];
  for (uint32_t s = threadIdx.x; s < nseg; s += blockDim.x) {
    s_lo[s] = ~0ull;
    s_hi[s] = 0ull;
  }
  __syncthreads();
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const uint32_t s = seg[i];
    if (!act[s]) continue;
    const double x = kd_coord(P[i], dim);
    const unsigned long long o = ord_bits(x);
    if (o < cand[2 * s] || o > cand[2 * s + 1]) continue;
    if (narrow && kd_bin(x, cand, s, bins) != info[4 * s]) continue;
    atomicMin(&s_lo[s], o);
    atomicMax(&s_hi[s], o);
  }
  __syncthreads();
  for (uint32_t s = threadIdx.x; s < nseg; s += blockDim.x)
    if (s_lo[s] != ~0ull) {
      atomicMin(&out[2 * s], s_lo[s]);
      atomicMax(&out[2 * s + 1], s_hi[s]);
    }
}

// the new candidate range of every active segment
__global__ void k_kd_adopt(uint32_t nseg, const uint32_t* act, const unsigned long long* ext,
                           unsigned long long* cand) {
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nseg || !act[s]) return;
  cand[2 * s] = ext[2 * s];
  cand[2 * s + 1] = ext[2 * s + 1];
}

// histogram of the candidates of all active segments (nseg * bins <=
// KD_HIST): per-block in LDS, then added to the global one
__global__ __launch_bounds__(256) void k_kd_hist(const double4* P, uint32_t n, int dim,
                                                 const uint32_t* seg, uint32_t bins,
                                                 uint32_t total, const unsigned long long* cand,
                                                 const uint32_t* act, uint32_t* hist) {
  __shared__ uint32_t s_h[KD_HIST];
  for (uint32_t j = threadIdx.x; j < total; j += blockDim.x) s_h[j] = 0;
  __syncthreads();
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const uint32_t s = seg[i];
    if (!act[s]) continue;
    const double x = kd_coord(P[i], dim);
    const unsigned long long o = ord_bits(x);
    if (o < cand[2 * s] || o > cand[2 * s + 1]) continue;
    atomicAdd(&s_h[s * bins + kd_bin(x, cand, s, bins)], 1u);
  }
  __syncthreads();
  for (uint32_t j = threadIdx.x; j < total; j += blockDim.x)
    if (s_h[j]) atomicAdd(&hist[j], s_h[j]);
}

// one block per active segment: the bin holding the wanted rank among the
// candidates (on the first pass floor(m/2) of the m points), the rank
// inside that bin and the bin's count; the first pass also records m
__global__ __launch_bounds__(256) void k_kd_findbin(const uint32_t* hist, uint32_t bins,
                                                    const uint32_t* act, int first,
                                                    uint32_t* info) {
  __shared__ uint32_t s_sum[256];
  const uint32_t s = blockIdx.x;
  if (!act[s]) return;
  const uint32_t* h = hist + (size_t)s * bins;
  const uint32_t chunk = (bins + 255) / 256;
  const uint32_t b0 = threadIdx.x * chunk, b1 = min(b0 + chunk, bins);
  uint32_t local = 0;
  for (uint32_t b = b0; b < b1; b++) local += h[b];
  s_sum[threadIdx.x] = local;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t m = 0;
    for (uint32_t t = 0; t < 256; t++) m += s_sum[t];
    const uint32_t want = first ? m / 2 : info[4 * s + 1];
    uint32_t cum = 0, bin = 0, cnt = 0, rank = 0;
    if (want < m) {
      uint32_t t = 0;
      while (cum + s_sum[t] <= want) cum += s_sum[t++];
      for (uint32_t b = t * chunk;; b++) {
        if (cum + h[b] > want) {
          bin = b;
          cnt = h[b];
          rank = want - cum;
          break;
        }
        cum += h[b];
      }
    }
    info[4 * s] = bin;
    info[4 * s + 1] = rank;
    info[4 * s + 2] = cnt;
    if (first) info[4 * s + 3] = m;
  }
}

__global__ void k_kd_collect(const double4* P, uint32_t n, int dim, const uint32_t* seg,
                             uint32_t bins, const unsigned long long* cand, const uint32_t* info,
                             const uint32_t* base, uint32_t* fill, uint32_t* items) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t s = seg[i];
  const double x = kd_coord(P[i], dim);
  const unsigned long long o = ord_bits(x);
  if (o < cand[2 * s] || o > cand[2 * s + 1]) return;
  if (kd_bin(x, cand, s, bins) != info[4 * s]) return;
  const uint32_t slot = atomicAdd(&fill[s], 1u);
  if (slot < info[4 * s + 2]) items[base[s] + slot] = i;
}

// one block per segment: sort the chosen bin's elements by (coordinate,
// id) in LDS (bitonic) and keep the one of the wanted rank
__global__ __launch_bounds__(256) void k_kd_select(const double4* P, int dim, const uint32_t* info,
                                                   const uint32_t* base, const uint32_t* items,
                                                   unsigned long long* med, double* split) {
  __shared__ unsigned long long s_key[KD_CAP];
  __shared__ uint32_t s_id[KD_CAP];
  const uint32_t s = blockIdx.x;
  const uint32_t cnt = info[4 * s + 2], rank = info[4 * s + 1], m = info[4 * s + 3];
  if (m == 0) {
    if (threadIdx.x == 0) {
      med[2 * s] = ~0ull;
      med[2 * s + 1] = ~0ull;
      split[s] = NAN;
    }
    return;
  }
  uint32_t np2 = 1;
  while (np2 < cnt) np2 <<= 1;
  for (uint32_t j = threadIdx.x; j < np2; j += blockDim.x) {
    if (j < cnt) {
      const uint32_t id = items[base[s] + j];
      s_key[j] = ord_bits(kd_coord(P[id], dim));
      s_id[j] = id;
    } else {
      s_key[j] = ~0ull;
      s_id[j] = 0xFFFFFFFFu;
    }
  }
  __syncthreads();
  for (uint32_t size = 2; size <= np2; size <<= 1)
    for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
      for (uint32_t j = threadIdx.x; j < np2; j += blockDim.x) {
        const uint32_t o = j ^ stride;
        if (o > j) {
          const bool up = (j & size) == 0;
          const bool gt = s_key[j] > s_key[o] || (s_key[j] == s_key[o] && s_id[j] > s_id[o]);
          if (gt == up) {
            const unsigned long long tk = s_key[j];
            s_key[j] = s_key[o];
            s_key[o] = tk;
            const uint32_t ti = s_id[j];
            s_id[j] = s_id[o];
            s_id[o] = ti;
          }
        }
      }
      __syncthreads();
    }
  if (threadIdx.x == 0) {
    med[2 * s] = s_key[rank];
    med[2 * s + 1] = s_id[rank];
    split[s] = kd_coord(P[s_id[rank]], dim);
  }
}

// lower child: the floor(m/2) smallest (coordinate, id); upper: the rest
__global__ void k_kd_classify(const double4* P, uint32_t n, int dim, uint32_t* seg,
                              const unsigned long long* med) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t s = seg[i];
  const unsigned long long key = ord_bits(kd_coord(P[i], dim));
  const unsigned long long mk = med[2 * s], mi = med[2 * s + 1];
  const bool upper = key > mk || (key == mk && (unsigned long long)i >= mi);
  seg[i] = 2 * s + (upper ? 1u : 0u);
}

// One level of the kd split by selection.  *done stays false when the
// level does not fit the selection (too many segments, or a median bin
// that stays larger than the LDS sort takes, as with many equal
// coordinates); the caller then sorts.
static int kd_level_select(const double4* P, uint32_t n, int dim, int l, uint32_t nseg,
                           DevBuf& pid, DevBuf& dsplit, bool* done, hipStream_t st) {
  *done = false;
  uint32_t bins = KD_HIST >> l;
  if (bins < KD_MINBINS) bins = KD_MINBINS;
  if (nseg > KD_MAXSEG || (uint64_t)nseg * bins > KD_HIST || n == 0) return DT_OK;
  const uint32_t total = nseg * bins;
  uint32_t grid = dblocks(n);
  if (grid > KD_GRID) grid = KD_GRID;
  DevBuf cand, ext, act, hist, info, base, fill, items, med;
  DT_TRY(cand.alloc((size_t)nseg * 16));
  DT_TRY(ext.alloc((size_t)nseg * 16));
  DT_TRY(act.alloc((size_t)nseg * 4));
  DT_TRY(hist.alloc((size_t)total * 4));
  DT_TRY(info.alloc((size_t)nseg * 16));
  std::vector<unsigned long long> all(2 * nseg), empty(2 * nseg);
  for (uint32_t s = 0; s < nseg; s++) {
    all[2 * s] = 0ull;
    all[2 * s + 1] = ~0ull;
    empty[2 * s] = ~0ull;
    empty[2 * s + 1] = 0ull;
  }
  std::vector<uint32_t> hact(nseg, 1u);
  DT_HIP(hipMemcpyAsync(cand.p, all.data(), (size_t)nseg * 16, hipMemcpyHostToDevice, st));
  DT_HIP(hipMemcpyAsync(ext.p, empty.data(), (size_t)nseg * 16, hipMemcpyHostToDevice, st));
  DT_HIP(hipMemcpyAsync(act.p, hact.data(), (size_t)nseg * 4, hipMemcpyHostToDevice, st));
  const uint32_t sb = (nseg + 255) / 256;
  // candidate range of every segment: all of its points
  hipLaunchKernelGGL(k_kd_extent, dim3(grid), dim3(256), 0, st, P, n, dim, pid.as<uint32_t>(),
                     nseg, cand.as<unsigned long long>(), act.as<uint32_t>(), info.as<uint32_t>(),
                     bins, 0, ext.as<unsigned long long>());
  hipLaunchKernelGGL(k_kd_adopt, dim3(sb), dim3(256), 0, st, nseg, act.as<uint32_t>(),
                     ext.as<unsigned long long>(), cand.as<unsigned long long>());
  std::vector<uint32_t> hinfo(4 * nseg);
  bool small = false;
  for (int pass = 0; pass <= KD_NARROW; pass++) {
    if (pass > 0) {
      // narrow the still active segments to their chosen bin
      DT_HIP(hipMemcpyAsync(ext.p, empty.data(), (size_t)nseg * 16, hipMemcpyHostToDevice, st));
      hipLaunchKernelGGL(k_kd_extent, dim3(grid), dim3(256), 0, st, P, n, dim,
                         pid.as<uint32_t>(), nseg, cand.as<unsigned long long>(),
                         act.as<uint32_t>(), info.as<uint32_t>(), bins, 1,
                         ext.as<unsigned long long>());
      hipLaunchKernelGGL(k_kd_adopt, dim3(sb), dim3(256), 0, st, nseg, act.as<uint32_t>(),
                         ext.as<unsigned long long>(), cand.as<unsigned long long>());
    }
    DT_HIP(hipMemsetAsync(hist.p, 0, (size_t)total * 4, st));
    hipLaunchKernelGGL(k_kd_hist, dim3(grid), dim3(256), 0, st, P, n, dim, pid.as<uint32_t>(),
                       bins, total, cand.as<unsigned long long>(), act.as<uint32_t>(),
                       hist.as<uint32_t>());
    hipLaunchKernelGGL(k_kd_findbin, dim3(nseg), dim3(256), 0, st, hist.as<uint32_t>(), bins,
                       act.as<uint32_t>(), pass == 0 ? 1 : 0, info.as<uint32_t>());
    DT_HIP(hipGetLastError());
    DT_HIP(hipMemcpyAsync(hinfo.data(), info.p, (size_t)nseg * 16, hipMemcpyDeviceToHost, st));
    DT_HIP(hipStreamSynchronize(st));
    small = true;
    for (uint32_t s = 0; s < nseg; s++) {
      if (!hact[s]) continue;
      if (hinfo[4 * s + 2] <= KD_CAP) hact[s] = 0;
      else small = false;
    }
    if (small) break;
    DT_HIP(hipMemcpyAsync(act.p, hact.data(), (size_t)nseg * 4, hipMemcpyHostToDevice, st));
  }
  if (!small) return DT_OK;   // coordinates too close or equal: sort
  std::vector<uint32_t> hbase(nseg);
  uint64_t tot = 0;
  for (uint32_t s = 0; s < nseg; s++) {
    hbase[s] = (uint32_t)tot;
    tot += hinfo[4 * s + 2];
  }
  DT_TRY(base.alloc((size_t)nseg * 4));
  DT_TRY(fill.alloc((size_t)nseg * 4));
  DT_TRY(items.alloc((size_t)(tot ? tot : 1) * 4));
  DT_TRY(med.alloc((size_t)nseg * 16));
  DT_HIP(hipMemcpyAsync(base.p, hbase.data(), (size_t)nseg * 4, hipMemcpyHostToDevice, st));
  DT_HIP(hipMemsetAsync(fill.p, 0, (size_t)nseg * 4, st));
  hipLaunchKernelGGL(k_kd_collect, dim3(dblocks(n)), dim3(DB), 0, st, P, n, dim,
                     pid.as<uint32_t>(), bins, cand.as<unsigned long long>(), info.as<uint32_t>(),
                     base.as<uint32_t>(), fill.as<uint32_t>(), items.as<uint32_t>());
  hipLaunchKernelGGL(k_kd_select, dim3(nseg), dim3(256), 0, st, P, dim, info.as<uint32_t>(),
                     base.as<uint32_t>(), items.as<uint32_t>(), med.as<unsigned long long>(),
                     dsplit.as<double>());
  hipLaunchKernelGGL(k_kd_classify, dim3(dblocks(n)), dim3(DB), 0, st, P, n, dim,
                     pid.as<uint32_t>(), med.as<unsigned long long>());
  DT_HIP(hipGetLastError());
  *done = true;
  return DT_OK;
}

int kd_divide(const double4* P, uint32_t n, int D, uint32_t k, DevBuf& pid, DevBuf& boxes,
              hipStream_t st) {
  int levels = 0;
  while ((1u << levels) < k) levels++;
  // region of every block: [lo, hi] per dimension, refined by each split
  std::vector<double> box((size_t)k * 6);
  for (uint32_t b = 0; b < k; b++)
    for (int a = 0; a < 3; a++) {
      box[b * 6 + a] = -INFINITY;
      box[b * 6 + 3 + a] = INFINITY;
    }
  DevBuf dsplit;
  DT_TRY(dsplit.alloc((size_t)k * 8));
  DT_TRY(pid.alloc((size_t)n * 4));
  DT_HIP(hipMemsetAsync(pid.p, 0, (size_t)n * 4, st));
  DevBuf keys, vals, cnt, off;
  DT_TRY(keys.alloc((size_t)n * 8));
  DT_TRY(vals.alloc((size_t)n * 4));
  DT_TRY(cnt.alloc((size_t)(k + 1) * 4));
  DT_TRY(off.alloc((size_t)(k + 1) * 4));
  for (int l = 0; l < levels; l++) {
    uint32_t nseg = 1u << l;
    bool selected = false;
    DT_TRY(kd_level_select(P, n, l % D, l, nseg, pid, dsplit, &selected, st));
    if (!selected) {
    hipLaunchKernelGGL(k_kd_keys, dim3(dblocks(n)), dim3(DB), 0, st, P, n, l % D,
                       keys.as<unsigned long long>(), vals.as<uint32_t>());
    DT_TRY(radix_sort_pairs(keys.as<unsigned long long>(), vals.as<uint32_t>(), n, 64, st));
    hipLaunchKernelGGL(k_kd_segkeys, dim3(dblocks(n)), dim3(DB), 0, st, vals.as<uint32_t>(), n,
                       pid.as<uint32_t>(), keys.as<unsigned long long>());
    int sbits = l == 0 ? 1 : l;
    DT_TRY(radix_sort_pairs(keys.as<unsigned long long>(), vals.as<uint32_t>(), n, sbits, st));
    DT_HIP(hipMemsetAsync(cnt.p, 0, (size_t)(k + 1) * 4, st));
    hipLaunchKernelGGL(k_count_u32, dim3(dblocks(n)), dim3(DB), 0, st, pid.as<uint32_t>(), n,
                       cnt.as<uint32_t>());
    DT_TRY(exclusive_scan(cnt.as<uint32_t>(), off.as<uint32_t>(), nseg + 1, st));
    std::vector<double> nanv(nseg, NAN);
    DT_HIP(hipMemcpyAsync(dsplit.p, nanv.data(), (size_t)nseg * 8, hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_kd_split, dim3(dblocks(n)), dim3(DB), 0, st,
                       keys.as<unsigned long long>(), vals.as<uint32_t>(), n, off.as<uint32_t>(),
                       pid.as<uint32_t>(), P, l % D, dsplit.as<double>());
    DT_HIP(hipGetLastError());
    }
    std::vector<double> hs(nseg);
    DT_HIP(hipMemcpyAsync(hs.data(), dsplit.p, (size_t)nseg * 8, hipMemcpyDeviceToHost, st));
    DT_HIP(hipStreamSynchronize(st));
    // leaves below segment s at this level: [s << (levels-l), (s+1) << (levels-l))
    int sh = levels - l;
    for (uint32_t sgm = 0; sgm < nseg; sgm++) {
      double v = hs[sgm];
      if (v != v) continue;   // empty block
      uint32_t mid = (2 * sgm + 1) << (sh - 1);
      for (uint32_t b = sgm << sh; b < mid; b++) box[b * 6 + 3 + l % D] = v;
      for (uint32_t b = mid; b < ((sgm + 1) << sh); b++) box[b * 6 + l % D] = v;
    }
  }
  DT_TRY(boxes.alloc((size_t)k * 48));
  DT_HIP(hipMemcpyAsync(boxes.p, box.data(), (size_t)k * 48, hipMemcpyHostToDevice, st));
  DT_HIP(hipStreamSynchronize(st));
  return DT_OK;
}

int count_by(const uint32_t* x, uint32_t m, uint32_t k, uint32_t* cnt, hipStream_t st) {
  DT_HIP(hipMemsetAsync(cnt, 0, (size_t)k * 4, st));
  if (m == 0) return DT_OK;
  if (k <= COUNT_LDS_KEYS && m >= 65536) {
    const uint32_t nb = dblocks(m) < 512 ? dblocks(m) : 512;
    hipLaunchKernelGGL(k_count_u32_lds, dim3(nb), dim3(256), 0, st, x, m, k, cnt);
  } else {
    hipLaunchKernelGGL(k_count_u32, dim3(dblocks(m)), dim3(DB), 0, st, x, m, cnt);
  }
  DT_HIP(hipGetLastError());
  return DT_OK;
}

}  // namespace dtk
