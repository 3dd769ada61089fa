// Label phase (Algorithm 2 of the paper: LabelMax, LabelSeed, LabelFrontier)
// as two gfx950 kernels, plus seed compaction.
//
// k_longest : two triangles per thread. Gathers the three vertices, compares the
//             squared edge lengths in binary64 (each product and sum rounded,
//             no fused multiply-add) and writes the local index of the longest
//             edge (the paper's Max array) as one byte per triangle.
// k_label   : one tile of 2048 triangles per block, eight per thread; in
//             whole tiles lane l of a wave takes every 64th triangle from l,
//             so twin, origin and walk-word accesses of a wave are contiguous
//             12-byte triples. Writes the half-edge labels and
//             the SEED flag, the walk word of every half-edge (the twin of
//             an internal one, -1 - origin of a frontier one: all a polygon
//             walk reads) and the tile's seed count (also added to the sum of
//             its group of 64 tiles).
// k_seeds   : the seed triangles in increasing index: each tile finds the
//             seeds before it from the group sums and the counts of its own
//             group, then places its seeds after them (no tile waits for
//             another).
#include "common.h"
#include "scan.h"

namespace polylla {

struct alignas(4) Int3 {
  int32_t x, y, z;
};

__device__ __forceinline__ double sq_length(double2 a, double2 b) {
  double dx = __dsub_rn(b.x, a.x);
  double dy = __dsub_rn(b.y, a.y);
  return __dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy));
}

// Edge key used to order equal lengths: the smaller half-edge of the edge.
__device__ __forceinline__ int32_t edge_key(const int32_t* __restrict__ twin, int32_t h, int32_t nhe,
                                            Counters* cnt) {
  int32_t tw = twin[h];
  if (tw < -1 || tw >= nhe) {
    set_error(cnt, POLYLLA_ETOPO);
    return h;
  }
  return (tw < 0 || h < tw) ? h : tw;
}

__global__ void k_reset(Counters* cnt, uint64_t* status, int64_t n_status, const int64_t* n_from, int keep) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t k = i; k < n_status; k += stride) status[k] = 0;
  if (blockIdx.x == 0) {
    // keep != 0: the error word and the batch sums survive (later groups of a batched call)
    int32_t* w = reinterpret_cast<int32_t*>(cnt);
    const size_t acc_lo = offsetof(Counters, acc) / 4, acc_hi = acc_lo + sizeof(cnt->acc) / 4;
    for (size_t k = threadIdx.x; k < sizeof(Counters) / 4; k += blockDim.x)
      if (!keep || (k != 0 && (k < acc_lo || k >= acc_hi))) w[k] = 0;
    __syncthreads();
    if (threadIdx.x == 0 && n_from) cnt->n_seeds = (uint32_t)(*n_from);
  }
}

// Adds the path counters of the group just run to the batch sums.
__global__ void k_accumulate(Counters* cnt) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const uint32_t v[7] = {cnt->n_seeds, cnt->n_deferred, cnt->n_tips, cnt->n_splits,
                         cnt->n_big, cnt->n_fallback, cnt->n_lane};
  for (int k = 0; k < 7; ++k) cnt->acc[k] += v[k];
}

template <int kK>
__global__ __launch_bounds__(256) void k_longest(int64_t nt, int64_t nv, const double* __restrict__ xy,
                                                 const int32_t* __restrict__ origin,
                                                 const int32_t* __restrict__ twin, uint8_t* __restrict__ lg,
                                                 uint8_t* __restrict__ vtx, Counters* cnt) {
  const int64_t gid = (int64_t)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  if (vtx)
    for (int64_t v = gid; v < nv; v += stride) vtx[v] = 0;
  const int32_t nhe = (int32_t)(3 * nt);
  const double2* __restrict__ p = reinterpret_cast<const double2*>(xy);
  // kK triangles per thread, 64 apart within the wave's span of 64 kK: all
  // origin triples, then all vertex loads, are issued before first use (at
  // 10M: 105, 95 and 135 us for 1, 2 and 4; the autotuner can choose)
  const int64_t wbase = (gid & ~(int64_t)63) * kK + (gid & 63);
  const int64_t wstride = stride * kK;
  for (int64_t t0 = wbase; t0 < nt; t0 += wstride) {
    Int3 o3[kK];
    bool ok[kK];
#pragma unroll
    for (int k = 0; k < kK; ++k) {
      const int64_t t = t0 + 64 * k;
      ok[k] = t < nt;
      o3[k] = ok[k] ? *reinterpret_cast<const Int3*>(origin + 3 * t) : Int3{0, 0, 0};
    }
    double2 pa[kK], pb[kK], pc[kK];
#pragma unroll
    for (int k = 0; k < kK; ++k) {
      const int32_t a = o3[k].x, b = o3[k].y, c = o3[k].z;
      const bool in = (uint64_t)(uint32_t)a < (uint64_t)nv && (uint64_t)(uint32_t)b < (uint64_t)nv &&
                      (uint64_t)(uint32_t)c < (uint64_t)nv;
      if (ok[k] && !in) set_error(cnt, POLYLLA_ETOPO);
      ok[k] = ok[k] && in;
      pa[k] = ok[k] ? p[a] : make_double2(0.0, 0.0);
      pb[k] = ok[k] ? p[b] : make_double2(0.0, 0.0);
      pc[k] = ok[k] ? p[c] : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int k = 0; k < kK; ++k) {
      const int64_t t = t0 + 64 * k;
      if (t >= nt) continue;
      if (!ok[k]) {
        lg[t] = 0;
        continue;
      }
      const int32_t h0 = (int32_t)(3 * t);
      double l0 = sq_length(pa[k], pb[k]), l1 = sq_length(pb[k], pc[k]), l2 = sq_length(pc[k], pa[k]);
      int best = 0;
      double lb = l0;
      if (l1 > lb) {
        best = 1;
        lb = l1;
      } else if (l1 == lb && edge_key(twin, h0 + 1, nhe, cnt) < edge_key(twin, h0, nhe, cnt)) {
        best = 1;
      }
      if (l2 > lb) {
        best = 2;
      } else if (l2 == lb && edge_key(twin, h0 + 2, nhe, cnt) < edge_key(twin, h0 + best, nhe, cnt)) {
        best = 2;
      }
      lg[t] = (uint8_t)best;
    }
  }
}

// Max of triangle u: from the block's LDS window of Max bytes when u falls in
// it (most neighbours do: triangles are numbered along a space-filling order),
// else from global memory.
struct LgView {
  const uint8_t* __restrict__ lg;
  const uint8_t* win;  // LDS copy of lg[lo, lo + n), or null
  int64_t lo;
  int n;
  __device__ __forceinline__ uint8_t operator[](int64_t u) const {
    const int64_t r = u - lo;
    return (win && (uint64_t)r < (uint64_t)n) ? win[r] : lg[u];
  }
};

// Labels of the three half-edges of triangle t and whether t is a seed. Bit
// i of fx: half-edge i is a side of an input segment, labelled like a
// boundary edge (frontier; a boundary terminal edge where it is the longest).
template <class LG>
__device__ __forceinline__ uint32_t label_triangle(int64_t t, int m, const int32_t tw[3], const LG& lg, int32_t nhe,
                                                   Counters* cnt, bool* seed, uint32_t fx = 0) {
  uint32_t packed = 0;
  bool s = false;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const bool mine = (m == i);
    uint32_t lab = mine ? kLongest : 0u;
    int32_t u = tw[i];
    if (((fx >> i) & 1u) && u >= 0) {
      lab |= kFrontier | kConstrained;
      if (mine) {
        lab |= kTerminal;
        s = true;
      }
    } else if (u < 0) {
      lab |= kFrontier | kBorder;
      if (mine) {
        lab |= kTerminal;
        s = true;
      }
      if (u != -1) set_error(cnt, POLYLLA_ETOPO);
    } else {
      if (u >= nhe) {
        set_error(cnt, POLYLLA_ETOPO);
        u = 0;
      }
      const int64_t tu = u / 3;
      const bool theirs = lg[tu] == (uint8_t)(u - 3 * tu);
      if (mine && theirs) {
        lab |= kTerminal;
        if (t < tu) s = true;
      }
      if (!mine && !theirs) lab |= kFrontier;
    }
    packed |= lab << (8 * i);
  }
  *seed = s;
  return packed;
}

constexpr int kLabelItems = 8;  // triangles per thread of k_label (multiple of 4)

// 3 ITEMS consecutive words as 16-byte loads / stores (16-byte aligned).
template <int ITEMS>
__device__ __forceinline__ void load_words(const int32_t* __restrict__ src, int32_t (&w)[3 * ITEMS]) {
  const int4* s4 = reinterpret_cast<const int4*>(src);
#pragma unroll
  for (int k = 0; k < 3 * ITEMS / 4; ++k) {
    const int4 q = s4[k];
    w[4 * k] = q.x;
    w[4 * k + 1] = q.y;
    w[4 * k + 2] = q.z;
    w[4 * k + 3] = q.w;
  }
}
template <int ITEMS>
__device__ __forceinline__ void store_words(int32_t* __restrict__ dst, const int32_t (&w)[3 * ITEMS]) {
  int4* d4 = reinterpret_cast<int4*>(dst);
#pragma unroll
  for (int k = 0; k < 3 * ITEMS / 4; ++k) d4[k] = make_int4(w[4 * k], w[4 * k + 1], w[4 * k + 2], w[4 * k + 3]);
}

// Walk words of one triangle, in place of its twins: the twin of an internal
// half-edge, -1 - origin of a frontier one.
__device__ __forceinline__ void walk_words(uint32_t lab, int32_t* tw, const int32_t* og) {
#pragma unroll
  for (int e = 0; e < 3; ++e)
    if ((lab >> (8 * e)) & kFrontier) tw[e] = -1 - og[e];
}
constexpr int kLgMargin = 2048;  // Max bytes before and after a tile kept in LDS
constexpr int kLgWin = 256 * kLabelItems + 2 * kLgMargin;

// COMPUTE = true : labels from twin + Max, then seed compaction.
// COMPUTE = false: seed compaction only, from existing triangle labels.
// Segment bits of triangle t (bit i: half-edge 3t+i is a side of an input segment).
__device__ __forceinline__ uint32_t seg_bits(const uint8_t* __restrict__ fixed, int64_t t) {
  if (!fixed) return 0u;
  return (fixed[3 * t] ? 1u : 0u) | (fixed[3 * t + 1] ? 2u : 0u) | (fixed[3 * t + 2] ? 4u : 0u);
}

template <bool COMPUTE>
__global__ __launch_bounds__(256) void k_label(int64_t nt, const int32_t* __restrict__ twin,
                                               const uint8_t* __restrict__ lg, uint8_t* __restrict__ he,
                                               uint8_t* __restrict__ tri, const int32_t* __restrict__ origin,
                                               int32_t* __restrict__ wk, uint32_t* __restrict__ tcount,
                                               uint32_t* __restrict__ tsuper, Counters* cnt, bool vec,
                                               const uint8_t* __restrict__ fixed) {
  constexpr int ITEMS = kLabelItems;
  const uint32_t tile = xcd_block(blockIdx.x, gridDim.x);
  const int64_t t0 = ((int64_t)tile * 256 + threadIdx.x) * ITEMS;
  const int32_t nhe = (int32_t)(3 * nt);
  bool sd[ITEMS];
  // Whole tiles stage their label bytes in LDS and write them with coalesced
  // 16-byte stores.
  __shared__ uint4 s_w4[256 * ITEMS / 4];  // he words, then tri words of the tile
  const int64_t tile_t0 = (int64_t)tile * 256 * ITEMS;
  const bool full = COMPUTE && vec && tile_t0 + 256 * ITEMS <= nt && (reinterpret_cast<uintptr_t>(wk) & 15) == 0;
  __shared__ uint4 s_lg4[kLgWin / 16];
  if (full) {
    // Max bytes of the tile and its margins (16-byte aligned: tiles and
    // margins are multiples of 16 triangles)
    const int64_t wlo = tile_t0 - kLgMargin;
    for (int k = threadIdx.x; k < kLgWin / 16; k += 256) {
      const int64_t g = wlo + 16 * (int64_t)k;
      uint4 w = make_uint4(0u, 0u, 0u, 0u);
      if (g >= 0 && g + 16 <= nt) {
        w = *reinterpret_cast<const uint4*>(lg + g);
      } else {
        uint8_t* wb = reinterpret_cast<uint8_t*>(&w);
        for (int b = 0; b < 16; ++b)
          if (g + b >= 0 && g + b < nt) wb[b] = lg[g + b];
      }
      s_lg4[k] = w;
    }
    __syncthreads();
    const LgView lgv{lg, reinterpret_cast<const uint8_t*>(s_lg4), wlo, kLgWin};
    // interleaved: lane l of wave w takes triangles tile_t0 + 512 w + l + 64 k,
    // so every twin / origin / walk-word access of a wave covers 768
    // contiguous bytes
    uint8_t* s_heb = reinterpret_cast<uint8_t*>(s_w4);
    uint8_t* s_trib = s_heb + 256 * ITEMS * 3;
    const int lane = threadIdx.x & 63;
    const int wbase = (threadIdx.x >> 6) * 64 * ITEMS;  // tile-local first triangle of the wave
    Int3 tw3[ITEMS], og3[ITEMS];
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
      const int64_t t = tile_t0 + wbase + lane + 64 * k;
      tw3[k] = *reinterpret_cast<const Int3*>(twin + 3 * t);
      og3[k] = *reinterpret_cast<const Int3*>(origin + 3 * t);
    }
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
      const int lt = wbase + lane + 64 * k;
      const int64_t t = tile_t0 + lt;
      int32_t tw[3] = {tw3[k].x, tw3[k].y, tw3[k].z};
      const int32_t og[3] = {og3[k].x, og3[k].y, og3[k].z};
      const uint32_t lab = label_triangle(t, reinterpret_cast<const uint8_t*>(s_lg4)[kLgMargin + lt], tw, lgv, nhe,
                                          cnt, &sd[k], seg_bits(fixed, t));
      walk_words(lab, tw, og);
      Int3 w3;
      w3.x = tw[0];
      w3.y = tw[1];
      w3.z = tw[2];
      *reinterpret_cast<Int3*>(wk + 3 * t) = w3;
      s_heb[3 * lt] = (uint8_t)lab;
      s_heb[3 * lt + 1] = (uint8_t)(lab >> 8);
      s_heb[3 * lt + 2] = (uint8_t)(lab >> 16);
      s_trib[lt] = sd[k] ? kSeed : 0;
    }
    __syncthreads();
    if (((reinterpret_cast<uintptr_t>(he) | reinterpret_cast<uintptr_t>(tri)) & 15) == 0) {
      uint4* ghe = reinterpret_cast<uint4*>(he + 3 * tile_t0);
      uint4* gtri = reinterpret_cast<uint4*>(tri + tile_t0);
      for (int k = threadIdx.x; k < 256 * ITEMS * 3 / 16; k += 256) ghe[k] = s_w4[k];
      for (int k = threadIdx.x; k < 256 * ITEMS / 16; k += 256) gtri[k] = s_w4[256 * ITEMS * 3 / 16 + k];
    } else {
      // label arrays at any byte offset (a group of a batch starts at an
      // arbitrary half-edge): byte stores, contiguous over each wave
      for (int k = threadIdx.x; k < 256 * ITEMS * 3; k += 256) he[3 * tile_t0 + k] = s_heb[k];
      for (int k = threadIdx.x; k < 256 * ITEMS; k += 256) tri[tile_t0 + k] = s_trib[k];
    }
  } else if (COMPUTE) {
    if (vec && t0 + ITEMS <= nt &&
        ((reinterpret_cast<uintptr_t>(he) | reinterpret_cast<uintptr_t>(tri)) & 3) == 0) {
      // ITEMS triangles: twins and origins as int4, ITEMS Max bytes and labels as words
      int32_t tw[3 * ITEMS], og[3 * ITEMS];
      load_words<ITEMS>(twin + 3 * t0, tw);
      load_words<ITEMS>(origin + 3 * t0, og);
      uint32_t mm[ITEMS / 4];
#pragma unroll
      for (int k = 0; k < ITEMS / 4; ++k) mm[k] = reinterpret_cast<const uint32_t*>(lg + t0)[k];
      uint32_t* he4 = reinterpret_cast<uint32_t*>(he + 3 * t0);
      uint32_t* tr4 = reinterpret_cast<uint32_t*>(tri + t0);
#pragma unroll
      for (int g = 0; g < ITEMS / 4; ++g) {
        uint32_t lab[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          lab[j] = label_triangle(t0 + 4 * g + j, (mm[g] >> (8 * j)) & 0xFF, tw + 3 * (4 * g + j),
                                  LgView{lg, nullptr, 0, 0}, nhe, cnt, &sd[4 * g + j], seg_bits(fixed, t0 + 4 * g + j));
          walk_words(lab[j], tw + 3 * (4 * g + j), og + 3 * (4 * g + j));
        }
        // 12 label bytes of 4 triangles -> three 32-bit words
        he4[3 * g] = lab[0] | (lab[1] << 24);
        he4[3 * g + 1] = (lab[1] >> 8) | (lab[2] << 16);
        he4[3 * g + 2] = (lab[2] >> 16) | (lab[3] << 8);
        tr4[g] = (sd[4 * g] ? kSeed : 0u) | ((sd[4 * g + 1] ? kSeed : 0u) << 8) |
                 ((sd[4 * g + 2] ? kSeed : 0u) << 16) | ((sd[4 * g + 3] ? kSeed : 0u) << 24);
      }
      store_words<ITEMS>(wk + 3 * t0, tw);
    } else {
#pragma unroll
      for (int j = 0; j < ITEMS; ++j) {
        sd[j] = false;
        const int64_t t = t0 + j;
        if (t >= nt) continue;
        int32_t tw[3] = {twin[3 * t], twin[3 * t + 1], twin[3 * t + 2]};
        const int32_t og[3] = {origin[3 * t], origin[3 * t + 1], origin[3 * t + 2]};
        uint32_t lab = label_triangle(t, lg[t], tw, LgView{lg, nullptr, 0, 0}, nhe, cnt, &sd[j], seg_bits(fixed, t));
        walk_words(lab, tw, og);
        wk[3 * t] = tw[0];
        wk[3 * t + 1] = tw[1];
        wk[3 * t + 2] = tw[2];
        he[3 * t] = (uint8_t)lab;
        he[3 * t + 1] = (uint8_t)(lab >> 8);
        he[3 * t + 2] = (uint8_t)(lab >> 16);
        tri[t] = sd[j] ? kSeed : 0;
      }
    }
  } else {
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
      const int64_t t = t0 + j;
      sd[j] = t < nt && (tri[t] & kSeed);
    }
  }
  uint32_t mine = 0;
#pragma unroll
  for (int j = 0; j < ITEMS; ++j) mine += sd[j] ? 1u : 0u;
  uint2 total;
  (void)block_exclusive_scan<256>(mine, 0u, &total);
  if (threadIdx.x == 0) {
    tcount[tile] = total.x;
    if (total.x) atomicAdd(&tsuper[tile >> 6], total.x);
  }
}

// Seed list of the tiles of k_label (tsuper zeroed before k_label ran).
__global__ __launch_bounds__(256) void k_seeds(int64_t nt, const uint8_t* __restrict__ tri,
                                               const uint32_t* __restrict__ tcount,
                                               const uint32_t* __restrict__ tsuper, int32_t* __restrict__ seeds,
                                               Counters* cnt) {
  constexpr int ITEMS = kLabelItems;
  static_assert(ITEMS == 8, "flags are read as two words");
  __shared__ uint32_t s_base;
  const uint32_t tile = blockIdx.x;
  if (threadIdx.x < 64) {
    const uint32_t lane = threadIdx.x;
    uint32_t acc = 0;
    for (uint32_t k = lane; k < (tile >> 6); k += 64) acc += tsuper[k];
    const uint32_t c = (tile & ~63u) + lane;
    if (c < tile) acc += tcount[c];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if (lane == 0) s_base = acc;
  }
  __syncthreads();
  const uint32_t base = s_base;
  const int64_t t0 = ((int64_t)tile * 256 + threadIdx.x) * ITEMS;
  uint32_t bits = 0;  // bit j: triangle t0 + j is a seed
  if (t0 + ITEMS <= nt && (reinterpret_cast<uintptr_t>(tri) & 7) == 0) {
    const uint2 f = *reinterpret_cast<const uint2*>(tri + t0);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      bits |= ((f.x >> (8 * j)) & kSeed) ? (1u << j) : 0u;
      bits |= ((f.y >> (8 * j)) & kSeed) ? (1u << (4 + j)) : 0u;
    }
  } else {
#pragma unroll
    for (int j = 0; j < ITEMS; ++j)
      if (t0 + j < nt && (tri[t0 + j] & kSeed)) bits |= 1u << j;
  }
  uint2 total;
  const uint2 pre = block_exclusive_scan<256>((uint32_t)__popc(bits), 0u, &total);
  uint32_t pos = base + pre.x;
#pragma unroll
  for (int j = 0; j < ITEMS; ++j)
    if ((bits >> j) & 1u) seeds[pos++] = (int32_t)(t0 + j);
  if (tile == gridDim.x - 1 && threadIdx.x == 0) cnt->n_seeds = base + total.x;
}

// Full check of the input layout: grouped next, index ranges, twin involution
// and matching endpoints.
__global__ __launch_bounds__(256) void k_validate(int64_t nhe, int64_t nv, const int32_t* __restrict__ twin,
                                                  const int32_t* __restrict__ next,
                                                  const int32_t* __restrict__ origin,
                                                  const uint8_t* __restrict__ fixed, Counters* cnt) {
  for (int64_t h = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; h < nhe; h += (int64_t)gridDim.x * blockDim.x) {
    const int32_t hh = (int32_t)h;
    if (next[h] != he_next(hh)) {
      set_error(cnt, POLYLLA_ELAYOUT);
      continue;
    }
    const int32_t o = origin[h], tw = twin[h];
    if ((uint64_t)(uint32_t)o >= (uint64_t)nv || tw < -1 || tw >= nhe || tw == hh) {
      set_error(cnt, POLYLLA_ETOPO);
      continue;
    }
    if (tw >= 0) {
      const int32_t on = origin[he_next(hh)];
      if (twin[tw] != hh || origin[tw] != on) set_error(cnt, POLYLLA_ETOPO);
      if (fixed && (fixed[h] != 0) != (fixed[tw] != 0)) set_error(cnt, POLYLLA_ETOPO);
    }
  }
}

#define INSTANTIATE_K_LONGEST(K)                                                                            \
  template __global__ void k_longest<K>(int64_t, int64_t, const double*, const int32_t*, const int32_t*, uint8_t*, \
                                        uint8_t*, Counters*);
INSTANTIATE_K_LONGEST(1)
INSTANTIATE_K_LONGEST(2)
INSTANTIATE_K_LONGEST(4)
#undef INSTANTIATE_K_LONGEST
template __global__ void k_label<true>(int64_t, const int32_t*, const uint8_t*, uint8_t*, uint8_t*, const int32_t*,
                                       int32_t*, uint32_t*, uint32_t*, Counters*, bool, const uint8_t*);
template __global__ void k_label<false>(int64_t, const int32_t*, const uint8_t*, uint8_t*, uint8_t*, const int32_t*,
                                        int32_t*, uint32_t*, uint32_t*, Counters*, bool, const uint8_t*);

// Walk words from existing half-edge labels, for calls that start from them.
__global__ __launch_bounds__(256) void k_pack_walk(int64_t nhe, const uint8_t* __restrict__ he,
                                                   const int32_t* __restrict__ twin,
                                                   const int32_t* __restrict__ origin, int32_t* __restrict__ wk) {
  for (int64_t h = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; h < nhe; h += (int64_t)gridDim.x * blockDim.x)
    wk[h] = (he[h] & kFrontier) ? -1 - origin[h] : twin[h];
}

}  // namespace polylla

namespace polylla {

// ---------------------------------------------------------------------------
// Longest-edge propagation paths (Rivara's Lepp): from triangle t, step to the
// neighbour across the current triangle's longest edge (the Max bytes of
// k_longest) until that edge is also the neighbour's longest edge (a terminal
// edge) or a boundary or segment side. Per triangle: the key of the terminal
// edge (its smaller half-edge; the half-edge itself on a boundary) and the
// number of triangles on the path.
//
// k_lepp_chase follows each path for up to kLeppSteps triangles; a path not
// finished by then keeps its state {last triangle reached, triangles so far,
// -1} in `state` and is listed in `list`. k_lepp_jump then shortens the
// listed paths by pointer jumping (each round reads one state array and
// writes the other): a path ending at a finished triangle, or at a listed one
// whose state is resolved, is resolved; otherwise it jumps to the end of the
// other path, so every round doubles the length covered.
constexpr int kLeppSteps = 32;

__device__ __forceinline__ bool lepp_bounding(const int32_t* __restrict__ twin, const uint8_t* __restrict__ fixed,
                                              int32_t h) {
  return twin[h] < 0 || (fixed && fixed[h]);
}

__global__ __launch_bounds__(256) void k_lepp_chase(int64_t nt, const uint8_t* __restrict__ lg,
                                                    const int32_t* __restrict__ twin,
                                                    const uint8_t* __restrict__ fixed, int32_t* __restrict__ terminal,
                                                    int32_t* __restrict__ length, int4* __restrict__ state,
                                                    int32_t* __restrict__ list, uint32_t* __restrict__ n_list,
                                                    Counters* cnt) {
  const int64_t t = (int64_t)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (t >= nt) return;
  const int32_t nhe = (int32_t)(3 * nt);
  int32_t cur = (int32_t)t, n = 1, term = -1;
  for (int k = 0; k < kLeppSteps; ++k) {
    const uint8_t m = lg[cur];
    const int32_t h = 3 * cur + (m < 3 ? m : 0);
    if (lepp_bounding(twin, fixed, h)) {
      term = h;
      break;
    }
    const int32_t u = twin[h];
    if (u >= nhe) {
      set_error(cnt, POLYLLA_ETOPO);
      term = h;
      break;
    }
    const int32_t nb = u / 3;
    ++n;
    if (lg[nb] == (uint8_t)(u - 3 * nb)) {
      term = h < u ? h : u;
      break;
    }
    cur = nb;
  }
  if (term >= 0) {
    terminal[t] = term;
    length[t] = n;
  } else {
    terminal[t] = -1;
    state[t] = make_int4(cur, n, -1, 0);
    list[atomicAdd(n_list, 1u)] = (int32_t)t;
  }
}

__global__ __launch_bounds__(256) void k_lepp_jump(const int32_t* __restrict__ terminal,
                                                   const int32_t* __restrict__ length,
                                                   const int4* __restrict__ s_in, int4* __restrict__ s_out,
                                                   const int32_t* __restrict__ list, const uint32_t* n_list) {
  const uint32_t n = *n_list;
  for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += gridDim.x * blockDim.x) {
    const int32_t t = list[j];
    int4 s = s_in[t];
    if (s.z < 0) {
      const int32_t cur = s.x;
      if (terminal[cur] >= 0) {  // the path reached a triangle finished by the chase
        s = make_int4(cur, s.y - 1 + length[cur], terminal[cur], 0);
      } else {
        const int4 o = s_in[cur];
        s = o.z >= 0 ? make_int4(cur, s.y - 1 + o.y, o.z, 0) : make_int4(o.x, s.y - 1 + o.y, -1, 0);
      }
    }
    s_out[t] = s;
  }
}

__global__ __launch_bounds__(256) void k_lepp_finish(int32_t* __restrict__ terminal, int32_t* __restrict__ length,
                                                     const int4* __restrict__ s_fin, const int32_t* __restrict__ list,
                                                     const uint32_t* n_list, Counters* cnt) {
  const uint32_t n = *n_list;
  for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += gridDim.x * blockDim.x) {
    const int32_t t = list[j];
    const int4 s = s_fin[t];
    if (s.z < 0) {
      set_error(cnt, POLYLLA_EDEGEN);  // more pointer-jumping rounds than the host launched
      continue;
    }
    terminal[t] = s.z;
    length[t] = s.y;
  }
}

}  // namespace polylla
