// Internal definitions shared by the HIP kernels and the host side of
// libpolylla (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/polylla.h"

#pragma clang fp contract(off)

namespace polylla {

constexpr uint8_t kLongest = POLYLLA_LONGEST;
constexpr uint8_t kFrontier = POLYLLA_FRONTIER;
constexpr uint8_t kTerminal = POLYLLA_TERMINAL;
constexpr uint8_t kBorder = POLYLLA_BORDER;
constexpr uint8_t kBarrier = POLYLLA_BARRIER;
constexpr uint8_t kRepaired = POLYLLA_REPAIRED;
constexpr uint8_t kConstrained = POLYLLA_CONSTRAINED;
constexpr uint8_t kSeed = POLYLLA_SEED;
constexpr uint8_t kTip = POLYLLA_TIP;

// Device-side counters and error word, one block per context (zeroed by the
// first kernel of every call). Counters that many workgroups update during a
// kernel sit 256 bytes apart, so that their atomics do not queue on one line.
struct Counters {
  int32_t error;          // first error code (0 = none)
  uint32_t tile_ticket[4];  // dynamic tile ids of the look-back scans
  uint32_t n_seeds;       // R
  uint32_t n_tips;
  uint32_t n_splits;
  uint32_t n_fallback;    // polygons too large for the 1024-thread workgroup's LDS
  uint32_t n_lane;        // polygons too large for the global-memory workgroup path (one lane each)
  uint32_t mem_ticket;    // work counter of the global-memory workgroup path
  uint32_t mem_done;      // workgroups of that path that have finished
  uint32_t n_over;        // polygons too large for the one-wave workgroup's LDS
  uint32_t n_gen;         // short polygons the tip path leaves to the region path
  uint32_t n_lrest;       // long cycles the long-cycle tip path leaves to the region path
  uint32_t n_lepp;        // longest-edge paths left to pointer jumping
  alignas(256) uint32_t n_deferred;  // polygons handled by the general path
  alignas(256) uint32_t n_big;       // polygons longer than the walk cap (one-wave workgroup path)
  alignas(256) uint32_t stage_top;   // bump allocator of the staging buffer (ints)
  alignas(256) uint32_t arena_top;   // bump allocator of the general-path arena (ints)
  alignas(256) uint32_t big_ticket;  // work counter of the one-wave workgroup path
  alignas(256) uint32_t over_ticket; // work counter of the 1024-thread workgroup path
  alignas(256) uint32_t xcd_ticket[8 * 64];  // walk work queues, one per XCD (xcd_ticket[64 x])
  // Sums of the path counters over the groups of a batched call (n_seeds,
  // n_deferred, n_tips, n_splits, n_big, n_fallback, n_lane); a reset that
  // keeps them also keeps the error word.
  uint64_t acc[7];
};

// Per-polygon results of the walk / general path, in seed order: one 16-byte
// record {vertices of all pieces, pieces | rotation << 24, canonical start
// half-edge (one piece), staging offset} written with a single store, plus the
// arena offset of the piece records, read only for polygons of more than one
// piece. The rotation is the slot of the staged cycle that the output starts
// at (the walk stages cycles unrotated; the general paths stage them rotated).
// Output of one group of a batched call, written by the emitter itself: the
// caller's int64 offsets, mesh-local vertex ids and start half-edges, and the
// first output polygon of each mesh, after the totals of the earlier groups.
struct BatchEmit {
  const int32_t* seeds;   // seed triangle of each polygon record (group indices)
  int64_t nm;             // meshes of the group
  const int64_t* he_off;  // their half-edge offsets (at the group's first mesh)
  const int64_t* vtx_off; // their vertex offsets (at the group's first mesh)
  const int64_t* base;    // {polygons, vertices, failure} of the earlier groups
  int64_t* offsets;       // the caller's CSR
  int32_t* verts;
  int32_t* start;         // or null
  int64_t* poly_off;      // first output polygon of each mesh (at the group's first mesh)
  int64_t cap_polys, cap_verts;
  int64_t* counts_g;      // the group's {polygons, vertices}
};

constexpr int kRotShift = 24;
constexpr int32_t kPiecesMask = (1 << kRotShift) - 1;

struct PolyState {
  int4* rec;
  int32_t* prec;
  __device__ __forceinline__ void set(int64_t i, int32_t len, int32_t pieces, int32_t start, int32_t stage) const {
    rec[i] = make_int4(len, pieces, start, stage);
  }
  // the same with a streaming (non-temporal) store
  __device__ __forceinline__ void set_stream(int64_t i, int32_t len, int32_t pieces, int32_t start,
                                             int32_t stage) const {
    typedef int32_t v4 __attribute__((ext_vector_type(4)));
    const v4 r = {len, pieces, start, stage};
    __builtin_nontemporal_store(r, reinterpret_cast<v4*>(rec + i));
  }
  __device__ __forceinline__ void clear(int64_t i) const { rec[i] = make_int4(0, 0, -1, 0); }
  __device__ __forceinline__ void set_len(int64_t i, int32_t len) const { reinterpret_cast<int32_t*>(rec + i)[0] = len; }
  __device__ __forceinline__ int32_t len(int64_t i) const { return reinterpret_cast<const int32_t*>(rec + i)[0]; }
};

// Workgroups are dispatched to the 8 XCDs round-robin (workgroup b to XCD
// b % 8). Streaming kernels renumber them so that each XCD takes one
// contiguous eighth of the work in order, and neighbouring data (vertices of
// neighbouring triangles, Max bytes of neighbouring tiles) stays in one L2.
__device__ __forceinline__ uint32_t xcd_block(uint32_t b, uint32_t nb) {
  const uint32_t q = nb / 8, r = nb % 8, x = b % 8, i = b / 8;
  return x * q + min(x, r) + i;
}

// Staging and arena chunks that one workgroup of the region kernels reserves
// at a time (the host adds the unused tails to the capacities).
constexpr int32_t kBigStageChunk64 = 1024, kBigArenaChunk64 = 256;
constexpr int32_t kBigStageChunk1024 = 8192, kBigArenaChunk1024 = 2048;
constexpr int kBigGrid64 = 4096, kBigGrid1024 = 128;

// Global-memory workgroup path for regions beyond the LDS of the 1024-thread
// workgroup: kMemGrid workgroups, each with a store for one region of up to
// km triangles (km = min(triangles of the mesh, kMemRegionMax)) and 2 km
// frontier half-edges. Int32 words of one workgroup's store: 4 km for the
// triangle slots and their links, 2 hash areas of mem_hcap(km) words, 6 + 15
// arrays of 2 km (frontier slots; pieces) and 7 arrays of km (tips).
constexpr int kMemGrid = 8;
constexpr int64_t kMemRegionMax = 1 << 16;
__host__ __device__ inline int64_t mem_hcap(int64_t km) {
  int64_t h = 64;
  while (h < 4 * km) h <<= 1;
  return h;
}
__host__ __device__ inline int64_t mem_words(int64_t km) { return 4 * km + 2 * mem_hcap(km) + 42 * km + 7 * km; }

__device__ __forceinline__ int32_t he_next(int32_t h) {
  int32_t r = h % 3;
  return r == 2 ? h - 2 : h + 1;
}

// Sets label bits in byte i of a byte array with an atomic OR on the aligned
// 32-bit word that holds it, whose result is not needed, so the thread does
// not wait for it. The word stays in the page of the byte and its other
// bytes are ORed with zero.
__device__ __forceinline__ void or_bits(uint8_t* a, int64_t i, uint32_t bits) {
  const uintptr_t p = reinterpret_cast<uintptr_t>(a + i);
  atomicOr(reinterpret_cast<uint32_t*>(p & ~(uintptr_t)3), bits << (8 * (uint32_t)(p & 3)));
}

__device__ __forceinline__ void set_error(Counters* c, int32_t code) {
  atomicCAS(&c->error, 0, code);
}

}  // namespace polylla
