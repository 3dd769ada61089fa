// Block-wide and single-pass device-wide exclusive scans of (a, b) pairs of
// 31-bit counts: wave64 shuffles inside a block, decoupled look-back across
// blocks (one status word per tile, read by the first wave, 64 predecessors
// at a time). Tiles take their ids from a ticket counter, so a tile only ever
// waits for tiles that already started and the spin always ends.
#pragma once

#include "common.h"

namespace polylla {

constexpr uint64_t kStatAggregate = 1ull << 62;
constexpr uint64_t kStatPrefix = 2ull << 62;
constexpr uint32_t kSpinLimit = 1u << 24;

__device__ __forceinline__ uint64_t pack_pair(uint32_t a, uint32_t b) {
  return ((uint64_t)(a & 0x7FFFFFFFu) << 31) | (uint64_t)(b & 0x7FFFFFFFu);
}

__device__ __forceinline__ void status_store(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint64_t status_load(uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Tile id from a ticket counter (all threads get the same value).
__device__ __forceinline__ uint32_t take_tile(uint32_t* ticket) {
  __shared__ uint32_t s_tile;
  if (threadIdx.x == 0) s_tile = atomicAdd(ticket, 1u);
  __syncthreads();
  uint32_t t = s_tile;
  __syncthreads();
  return t;
}

// Exclusive scan of (a, b) over the threads of a block; *total gets the block
// sums. BLOCK must be a multiple of 64.
template <int BLOCK>
__device__ __forceinline__ uint2 block_exclusive_scan(uint32_t a, uint32_t b, uint2* total) {
  __shared__ uint32_t wa[BLOCK / 64], wb[BLOCK / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  uint32_t ia = a, ib = b;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    uint32_t ta = __shfl_up(ia, o, 64), tb = __shfl_up(ib, o, 64);
    if (lane >= o) { ia += ta; ib += tb; }
  }
  if (lane == 63) { wa[wid] = ia; wb[wid] = ib; }
  __syncthreads();
  uint32_t oa = 0, ob = 0, sa = 0, sb = 0;
#pragma unroll
  for (int w = 0; w < BLOCK / 64; ++w) {
    if (w < wid) { oa += wa[w]; ob += wb[w]; }
    sa += wa[w];
    sb += wb[w];
  }
  *total = make_uint2(sa, sb);
  __syncthreads();
  return make_uint2(oa + ia - a, ob + ib - b);
}

// Publishes this tile's sums for later tiles (its prefix if it is tile 0).
// Call once per tile, as early as the sums are known; tile_lookback then
// gives the exclusive prefix.
__device__ __forceinline__ void tile_publish(uint64_t* status, uint32_t tile, uint2 agg) {
  if (threadIdx.x == 0)
    status_store(&status[tile], (tile == 0 ? kStatPrefix : kStatAggregate) | pack_pair(agg.x, agg.y));
}

// Exclusive prefix of tile `tile` across the grid, given this tile's sums.
// Called by every thread of the block; all get the same result. With
// `published`, tile_publish has already been called for this tile.
__device__ __forceinline__ uint2 tile_lookback(uint64_t* status, uint32_t tile, uint2 agg, Counters* cnt,
                                               bool published = false) {
  __shared__ uint2 s_ex;
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    uint32_t ea = 0, eb = 0;
    if (tile == 0) {
      if (lane == 0 && !published) status_store(&status[0], kStatPrefix | pack_pair(agg.x, agg.y));
    } else {
      if (lane == 0 && !published) status_store(&status[tile], kStatAggregate | pack_pair(agg.x, agg.y));
      int64_t base = (int64_t)tile - 1;
      uint32_t spins = 0;
      for (;;) {
        int64_t idx = base - lane;
        uint64_t w = idx >= 0 ? status_load(&status[idx]) : kStatPrefix;
        uint32_t flag = (uint32_t)(w >> 62);
        uint64_t pre = __ballot(flag == 2);
        uint64_t none = __ballot(flag == 0);
        int first = pre ? (__ffsll((unsigned long long)pre) - 1) : 63;
        uint64_t need = (2ull << first) - 1ull;
        if (none & need) {
          if (++spins > kSpinLimit) {
            if (lane == 0) set_error(cnt, POLYLLA_EINTERNAL);
            break;
          }
          __builtin_amdgcn_s_sleep(1);
          continue;
        }
        uint32_t va = lane <= first ? (uint32_t)((w >> 31) & 0x7FFFFFFFu) : 0u;
        uint32_t vb = lane <= first ? (uint32_t)(w & 0x7FFFFFFFu) : 0u;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
          va += __shfl_xor(va, o, 64);
          vb += __shfl_xor(vb, o, 64);
        }
        ea += va;
        eb += vb;
        if (pre) break;
        base -= 64;
      }
      if (lane == 0) status_store(&status[tile], kStatPrefix | pack_pair(ea + agg.x, eb + agg.y));
    }
    if (lane == 0) s_ex = make_uint2(ea, eb);
  }
  __syncthreads();
  uint2 r = s_ex;
  __syncthreads();
  return r;
}

}  // namespace polylla
