// Block-wide prefix counts for ordered, atomic-free compaction: a block
// counts its items, the block counts are scanned on the device, and every
// block writes its items at its offset in block order.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dtk {

// Exclusive prefix of v over the NT threads of the block; *total gets the
// block's sum.  Every thread of the block must call it (it synchronises).
template <int NT>
__device__ __forceinline__ uint32_t block_exclusive(uint32_t v, uint32_t* total) {
  static_assert(NT % 64 == 0, "whole wavefronts");
  __shared__ uint32_t s_w[NT / 64];
  const uint32_t lane = threadIdx.x & 63u, w = threadIdx.x >> 6;
  uint32_t incl = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t y = __shfl_up(incl, off, 64);
    if ((int)lane >= off) incl += y;
  }
  if (lane == 63u) s_w[w] = incl;
  __syncthreads();
  uint32_t before = 0, tot = 0;
#pragma unroll
  for (uint32_t i = 0; i < NT / 64; i++) {
    const uint32_t x = s_w[i];
    if (i < w) before += x;
    tot += x;
  }
  __syncthreads();
  *total = tot;
  return before + incl - v;
}

}  // namespace dtk
