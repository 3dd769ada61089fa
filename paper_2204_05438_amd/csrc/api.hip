// Host side of libpolylla: contexts, scratch, argument checks and the kernel
// sequence of every entry point declared in include/polylla.h.
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <mutex>
#include <type_traits>
#include <vector>

#include "common.h"

namespace polylla {

__global__ void k_reset(Counters*, uint64_t*, int64_t, const int64_t*, int);
__global__ void k_accumulate(Counters*);
__global__ void k_lepp_chase(int64_t, const uint8_t*, const int32_t*, const uint8_t*, int32_t*, int32_t*, int4*,
                             int32_t*, uint32_t*, Counters*);
__global__ void k_lepp_jump(const int32_t*, const int32_t*, const int4*, int4*, const int32_t*, const uint32_t*);
__global__ void k_lepp_finish(int32_t*, int32_t*, const int4*, const int32_t*, const uint32_t*, Counters*);
template <int kK>
__global__ void k_longest(int64_t, int64_t, const double*, const int32_t*, const int32_t*, uint8_t*, uint8_t*,
                          Counters*);
template <bool COMPUTE>
__global__ void k_label(int64_t, const int32_t*, const uint8_t*, uint8_t*, uint8_t*, const int32_t*, int32_t*,
                        uint32_t*, uint32_t*, Counters*, bool, const uint8_t*);
__global__ void k_seeds(int64_t, const uint8_t*, const uint32_t*, const uint32_t*, int32_t*, Counters*);
__global__ void k_pack_walk(int64_t, const uint8_t*, const int32_t*, const int32_t*, int32_t*);
__global__ void k_repair_prep(const int32_t*, const int32_t*, const int32_t*, int32_t*, int64_t, PolyState, int32_t*,
                              int64_t, int, Counters*);
template <bool FROM_SEEDS>
__global__ void k_walk(const int32_t*, int32_t, const int32_t*, int32_t*, int64_t, PolyState, int32_t*, int64_t, int,
                       Counters*);
template <bool REPAIR>
__global__ void k_general_small(const int32_t*, bool, int32_t, int64_t, const int32_t*, const int32_t*,
                                const int32_t*, uint8_t*, uint8_t*, int32_t*, int64_t, int32_t*, int64_t, PolyState,
                                const int32_t*, const uint32_t*, uint32_t, Counters*);
template <bool REPAIR>
__global__ void k_tip(int32_t, int64_t, const int32_t*, const int32_t*, const int32_t*, uint8_t*, uint8_t*, int32_t*, int64_t,
                      int32_t*, int64_t, PolyState, const int32_t*, int32_t*, int64_t, Counters*);
template <bool REPAIR>
__global__ void k_tip_long(int32_t, int64_t, const int32_t*, const int32_t*, const int32_t*, uint8_t*, uint8_t*,
                           int32_t*, int64_t, int32_t*, int64_t, PolyState, const int32_t*, int64_t, const uint32_t*,
                           uint32_t, uint32_t, int32_t*, int64_t, uint32_t*, Counters*);
template <bool REPAIR, int NT, int KC, int LC, int HB>
__global__ void k_general_big(const int32_t*, bool, int32_t, int64_t, const int32_t*, const int32_t*, const int32_t*,
                              uint8_t*, uint8_t*, int32_t*, int64_t, int32_t*, int64_t, PolyState, const int32_t*,
                              bool, int64_t, const uint32_t*, uint32_t*, int32_t*, int64_t, uint32_t*,
                              const int32_t*, int64_t, const uint32_t*, uint32_t, uint32_t, int32_t, Counters*);
template <bool REPAIR>
__global__ void k_general_huge(const int32_t*, bool, int32_t, int64_t, const int32_t*, const int32_t*,
                               const int32_t*, uint8_t*, uint8_t*, int32_t*, int64_t, int32_t*, int64_t, PolyState,
                               const int32_t*, int64_t, int32_t*, int64_t, int32_t*, int64_t, int32_t, int32_t,
                               Counters*);
template <bool BATCH>
__global__ void k_scan_emit(PolyState, uint64_t*, const int32_t*, const int32_t*, int32_t*, int32_t*, int32_t*,
                            int64_t*, int64_t, int64_t, Counters*, BatchEmit, int32_t);
__global__ void k_validate(int64_t, int64_t, const int32_t*, const int32_t*, const int32_t*, const uint8_t*,
                           Counters*);
__global__ void k_batch_empty(int64_t, const int64_t*, const int64_t*, const int64_t*, int64_t*, const Counters*);
__global__ void k_group_rebase(const int32_t*, const int32_t*, int32_t*, int32_t*, int64_t, const int64_t*,
                               const int64_t*);
__global__ void k_batch_begin(int64_t*);
__global__ void k_group_advance(const int64_t*, int64_t*, bool, int64_t, int64_t*, int64_t*, int64_t*, int64_t,
                                int64_t, const Counters*);
__global__ void k_batch_close(const int64_t*, int64_t, int64_t*);
size_t gen_ws_bytes(int64_t g);
int gen_grid_run(int64_t g, double jitter, uint64_t seed, double* xy, int32_t* twin, int32_t* origin,
                 int64_t cap_tri, void* ws, Counters* cnt, hipStream_t s, int64_t* n_tri, int* rounds);
int host_repair(int64_t, const int32_t*, const int32_t*, uint8_t*, int64_t, const int32_t*, const int32_t*,
                const int32_t*, int32_t*, int32_t*, int32_t*, int64_t, int64_t, int64_t*, int64_t*);

}  // namespace polylla

using namespace polylla;

// Scratch of polylla_mesh_noalloc: one static array per device, never
// allocated by a call. Host code reaches it only through the device address
// hipGetSymbolAddress returns for each device (taken once per device when a
// context is created on it); the array's name itself is not a device address
// in host code.
constexpr size_t kNoallocBytes = (size_t)64 << 20;
constexpr int64_t kNoallocMaxTri = 262144;  // triangles of the largest mesh it takes
constexpr int64_t kNoallocMaxVtx = 262144;  // vertices
constexpr int kNoallocWalkGrid = 64, kNoallocGrid64 = 256, kNoallocGrid1024 = 16;  // launch grids it is sized for
constexpr int64_t kNoallocMemKm = 4096;     // store of the global-memory region path (triangles)
constexpr int kMaxDevices = 64;
static __device__ __align__(256) uint8_t scratch[kNoallocBytes];
static std::mutex g_noalloc_mu;
static void* g_noalloc_ptr[kMaxDevices] = {};

// default number of declined short polygons up to which each gets a wave
constexpr uint32_t kGenWaveMax = 2 * polylla::kBigGrid64;
// most half-edges of one group of a batched call: keeps every int32 offset of
// the scratch arrays (arena 6T, staging 5T plus chunk tails) below 2^31
constexpr int64_t kGroupHeMax = ((int64_t)1 << 30) - ((int64_t)1 << 24);

// Device scratch of one call sequence: every array is a 256-byte aligned
// slice of one block of device memory (the context's own allocation, or the
// library's static array for polylla_mesh_noalloc). The caps are the sizes the
// slices were carved for; the grids are the launch sizes whose chunk tails the
// staging and arena capacities include.
struct Scratch {
  int64_t cap_t = 0;  // triangles
  int64_t cap_v = 0;  // vertices
  uint8_t* lg = nullptr;
  int32_t* wk = nullptr;  // walk word per half-edge: twin (internal) or -1 - origin (frontier)
  int32_t* seeds = nullptr;
  int32_t* deferred = nullptr;
  int32_t* over = nullptr;  // regions beyond the one-wave workgroup's LDS
  int32_t* huge = nullptr;  // regions beyond the 1024-thread workgroup's LDS
  int32_t* lane = nullptr;  // regions beyond the global-memory workgroup path
  int64_t over_cap = 0, huge_cap = 0, lane_cap = 0;
  int32_t* mem_store = nullptr;  // region stores of the global-memory workgroup path
  int64_t mem_km = 0;            // triangles of capacity of one store
  int32_t* rest = nullptr;  // short polygons the tip path leaves to the region path
  int64_t rest_cap = 0;
  int32_t* lrest = nullptr;  // long cycles the long-cycle tip path leaves to the region path
  int64_t lrest_cap = 0;
  int32_t* poly_arrays = nullptr;  // per-polygon records: 4 ints + 1 int per polygon (PolyState)
  int32_t* stage = nullptr;
  int64_t stage_cap = 0;
  int32_t* arena = nullptr;
  int64_t arena_cap = 0;
  uint64_t* status = nullptr;
  int64_t n_status = 0;
  int64_t n_status_label = 0;  // the label tiles' part; the emitter's follows
  uint8_t* he_s = nullptr;
  uint8_t* tri_s = nullptr;
  uint8_t* vtx_s = nullptr;
  int walk_grid = 0, grid64 = 0, grid1024 = 0;
  void* block = nullptr;  // the owned allocation (null for a view)
};

struct polylla_ctx {
  int device = 0;
  Counters* cnt = nullptr;
  Scratch own;         // scratch owned by the context (one device allocation)
  Scratch* sc = &own;  // the scratch the calls use (own, or a view of the library's static array)
  Counters last{};
  bool last_batched = false;  // polylla_stats reports the sums over the groups of the last batched call
  // batched calls: a group's twin and origin with indices over the group, its
  // polygons in int32 CSR, the first polygon of each of its meshes, running
  // totals {polygons, vertices, capacity failure}
  int32_t* g_twin = nullptr;
  int32_t* g_origin = nullptr;
  int32_t* g_off = nullptr;
  int32_t* g_verts = nullptr;
  int32_t* g_start = nullptr;
  int64_t* g_counts = nullptr;
  int64_t* g_poly = nullptr;
  int64_t* g_base = nullptr;
  int64_t g_cap_he = 0, g_cap_m = 0;
  int64_t group_he = kGroupHeMax;
  int walk_cap = 24;  // vertices a lane walks before handing a polygon to a workgroup
  int longest_items = 2;  // triangles per thread of k_longest (1, 2 or 4)
  uint32_t long_tip_min = kBigGrid64;  // long cycles up to which the long-cycle path only copies its list
  int32_t emit_lds_max = 1536;  // output polygons of an emitter tile staged in LDS (its tile + 512)
  uint32_t gen_wave_max = kGenWaveMax;  // declined short polygons up to which each gets a wave
  int32_t lds_max = 4096;               // region size limit of the 1024-thread LDS workgroup
  int32_t mem_max = (int32_t)kMemRegionMax;  // region size limit of the global-memory workgroup
  void* gen_ws = nullptr;  // work space of polylla_gen_grid
  size_t gen_ws_cap = 0;
  int walk_blocks = 1280;  // persistent grid of the walk kernel (swept at 10M: 768 516, 1024 474, 1280 462, 1536 474 us)
  // second stream: the workgroup region kernel runs beside the per-lane one
  // (they touch disjoint regions); fork and join through events
  hipStream_t side = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
  // event profiling
  int prof = 0;  // POLYLLA_PROFILE_* mode
  std::vector<hipEvent_t> ev_pool;
  struct Rec {
    int kernel;
    hipEvent_t a, b;
  };
  std::vector<Rec> recs;
};

namespace {

constexpr int64_t kGenGridMax = 18000;  // 6 g^2 half-edge ids stay below 2^31
constexpr int64_t kTile = 2048;  // triangles per tile of k_label
constexpr size_t kMaxProfiled = 8192;
constexpr int64_t kScanTileHost = 1024;   // polygons per tile of k_scan_emit
constexpr int64_t kWalkBlocks = 2048;     // persistent grid of k_walk
constexpr int64_t kStageChunkHost = 4096; // staging ints a walk wave reserves at a time

enum KernelId {
  KR_RESET, KR_LONGEST, KR_LABEL, KR_COMPACT, KR_PACK, KR_WALK, KR_GENERAL, KR_BIG, KR_HUGE, KR_SCAN, KR_VALIDATE,
  KR_BATCH, KR_BIGW, KR_TIP, KR_SEEDS, KR_GENW, KR_GREBASE, KR_LEPP, KR_PREP, KR_TIPL, KR_N
};
const char* kKernelNames[KR_N] = {"k_reset",         "k_longest",       "k_label",          "k_compact_seeds",
                                  "k_pack_walk",     "k_walk",          "k_general_small",  "k_general_big",
                                  "k_general_huge",  "k_scan_emit",     "k_validate",       "k_batch",
                                  "k_general_big_wg", "k_tip",           "k_seeds",          "k_general_wave",
                                  "k_group_rebase",  "k_lepp",          "k_repair_prep",
                                  "k_tip_long"};

// Event pair around one kernel launch when profiling is on.
struct Prof {
  polylla_ctx* c;
  hipStream_t s;
  int id;
  hipEvent_t b = nullptr;
  Prof(polylla_ctx* c_, hipStream_t s_, int id_) : c(c_), s(s_), id(id_) {
    if (!c->prof || (c->prof == POLYLLA_PROFILE_WALK && id != KR_WALK) || c->recs.size() >= kMaxProfiled ||
        c->ev_pool.size() < 2 * (c->recs.size() + 1))
      return;
    hipEvent_t a = c->ev_pool[2 * c->recs.size()];
    b = c->ev_pool[2 * c->recs.size() + 1];
    (void)hipEventRecord(a, s);
    c->recs.push_back({id, a, b});
  }
  ~Prof() {
    if (b) (void)hipEventRecord(b, s);
  }
};

template <typename T>
int dalloc(T** p, int64_t n) {
  *p = nullptr;
  if (n <= 0) n = 1;
  if (hipMalloc((void**)p, sizeof(T) * (size_t)n) != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    return POLYLLA_ENOMEM;
  }
  return POLYLLA_OK;
}

template <typename T>
void dfree(T** p) {
  if (*p) (void)hipFree(*p);
  *p = nullptr;
}

void free_scratch(polylla_ctx* c) {
  if (c->own.block) (void)hipFree(c->own.block);
  c->own = Scratch{};
}

// Staging and arena chunk tails of the launch grids (the walk's waves, two
// launches of the one-wave region kernel, one of the 1024-thread kernel).
int64_t stage_tails(int walk_grid, int g64, int g1024) {
  return 4 * (int64_t)walk_grid * kStageChunkHost + 2 * (int64_t)g64 * kBigStageChunk64 +
         (int64_t)g1024 * kBigStageChunk1024 + ((int64_t)1 << 20);
}
int64_t arena_tails(int g64, int g1024) {
  return 2 * (int64_t)g64 * kBigArenaChunk64 + (int64_t)g1024 * kBigArenaChunk1024 + 4096;
}

// Carves the scratch arrays for meshes of up to T triangles and V vertices
// out of `base` (every slice 256-byte aligned) and returns the bytes used;
// with base == nullptr only the size is computed. Offsets into the staging
// and arena arrays stay below 2^31.
size_t carve(Scratch& S, uint8_t* base, int64_t T, int64_t V, int walk_grid, int g64, int g1024,
             int64_t mem_km_max) {
  size_t off = 0;
  auto take = [&](auto*& ptr, int64_t n) {
    using E = std::remove_reference_t<decltype(*ptr)>;
    off = (off + 255) & ~(size_t)255;
    ptr = base ? reinterpret_cast<E*>(base + off) : nullptr;
    off += sizeof(E) * (size_t)std::max<int64_t>(n, 1);
  };
  S.cap_t = T;
  S.cap_v = V;
  S.walk_grid = walk_grid;
  S.grid64 = g64;
  S.grid1024 = g1024;
  const int64_t ntiles = (T + kTile - 1) / kTile + 1;
  // polygon vertices (<= 3T) and the general paths' staging, plus chunk tails
  S.stage_cap = std::min<int64_t>(5 * T + stage_tails(walk_grid, g64, g1024), ((int64_t)1 << 31) - 1);
  S.arena_cap = std::min<int64_t>(6 * T + arena_tails(g64, g1024), ((int64_t)1 << 31) - 1);
  S.n_status_label = ntiles;
  S.n_status = ntiles + (T + kScanTileHost - 1) / kScanTileHost + 1;
  // region lists, each sized for the most regions that can reach it on a
  // valid mesh (a region's cycle holds distinct frontier half-edges, at most
  // 3T in all, and its triangles are its own):
  S.huge_cap = 3 * T / 32 + 64;  // beyond the LDS limit (>= 32 triangles or half-edges)
  S.lane_cap = 3 * T / 32 + 64;  // beyond the global-memory limit (>= 32)
  S.over_cap = T / 32 + 64;      // beyond 128 triangles or half-edges: under 3T / 128 + T / 128
  S.rest_cap = 3 * T / 4 + 64;   // declined short cycles: a repeated vertex needs 4 half-edges
  S.lrest_cap = T + 64;          // long cycles: at most one per triangle (the walk cap may be as low as 1)
  S.mem_km = std::min<int64_t>(T, mem_km_max);
  take(S.status, S.n_status);
  take(S.lg, T);
  take(S.wk, 3 * T);
  take(S.seeds, T);
  take(S.deferred, T);
  take(S.huge, S.huge_cap);
  take(S.lane, S.lane_cap);
  take(S.mem_store, kMemGrid * mem_words(S.mem_km));
  take(S.over, S.over_cap);
  take(S.rest, S.rest_cap);
  take(S.lrest, S.lrest_cap);
  take(S.poly_arrays, 5 * T);
  take(S.stage, S.stage_cap);
  take(S.arena, S.arena_cap);
  take(S.he_s, 3 * T);
  take(S.tri_s, T);
  take(S.vtx_s, V);
  return (off + 255) & ~(size_t)255;
}

void free_group(polylla_ctx* c) {
  dfree(&c->g_twin);
  dfree(&c->g_origin);
  dfree(&c->g_off);
  dfree(&c->g_verts);
  dfree(&c->g_start);
  dfree(&c->g_counts);
  dfree(&c->g_poly);
  dfree(&c->g_base);
  c->g_cap_he = c->g_cap_m = 0;
}

// Scratch of batched calls for groups of up to n_he half-edges and n_m meshes.
int ensure_group(polylla_ctx* c, int64_t n_he, int64_t n_m) {
  if (n_he <= c->g_cap_he && n_m <= c->g_cap_m && c->g_base) return POLYLLA_OK;
  const int64_t H = std::max({n_he, c->g_cap_he, (int64_t)3072}), M = std::max({n_m, c->g_cap_m, (int64_t)64});
  if (hipSetDevice(c->device) != hipSuccess) return POLYLLA_EHIP;
  (void)hipDeviceSynchronize();
  free_group(c);
  const int64_t T = H / 3;
  int rc = POLYLLA_OK;
  if ((rc = dalloc(&c->g_twin, H)) || (rc = dalloc(&c->g_origin, H)) || (rc = dalloc(&c->g_off, T + 1)) ||
      (rc = dalloc(&c->g_verts, 3 * T)) || (rc = dalloc(&c->g_start, T)) || (rc = dalloc(&c->g_counts, 2)) ||
      (rc = dalloc(&c->g_poly, M + 1)) || (rc = dalloc(&c->g_base, 4))) {
    free_group(c);
    return rc;
  }
  c->g_cap_he = H;
  c->g_cap_m = M;
  return POLYLLA_OK;
}

int ensure(polylla_ctx* c, int64_t nt, int64_t nv) {
  if (c->sc != &c->own) return POLYLLA_EINTERNAL;  // a no-alloc call never reaches here
  if (nt <= c->own.cap_t && nv <= c->own.cap_v && c->own.block) return POLYLLA_OK;
  int64_t T = std::max(nt, c->own.cap_t), V = std::max(nv, c->own.cap_v);
  if (hipSetDevice(c->device) != hipSuccess) return POLYLLA_EHIP;
  (void)hipDeviceSynchronize();
  free_scratch(c);
  T = std::max<int64_t>(T, 1024);
  V = std::max<int64_t>(V, 1024);
  Scratch S;
  const size_t bytes = carve(S, nullptr, T, V, (int)kWalkBlocks, kBigGrid64, kBigGrid1024, kMemRegionMax);
  void* block = nullptr;
  if (hipMalloc(&block, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return POLYLLA_ENOMEM;
  }
  carve(S, static_cast<uint8_t*>(block), T, V, (int)kWalkBlocks, kBigGrid64, kBigGrid1024, kMemRegionMax);
  S.block = block;
  c->own = S;
  return POLYLLA_OK;
}

PolyState poly_state(polylla_ctx* c) {
  PolyState ps;
  ps.rec = reinterpret_cast<int4*>(c->sc->poly_arrays);
  ps.prec = c->sc->poly_arrays + 4 * c->sc->cap_t;
  return ps;
}

int check_tri(const polylla_tri* t) {
  if (!t) return POLYLLA_EINVAL;
  if (t->n_vertices < 0 || t->n_halfedges < 0) return POLYLLA_EINVAL;
  if (t->n_halfedges % 3) return POLYLLA_ELAYOUT;
  if (t->n_halfedges >= ((int64_t)1 << 31) - 64 || t->n_vertices >= ((int64_t)1 << 31)) return POLYLLA_EINVAL;
  if (t->n_halfedges > 0 && (!t->xy || !t->twin || !t->origin)) return POLYLLA_EINVAL;
  return POLYLLA_OK;
}

int check_polys(const polylla_polys* p, bool need_start) {
  if (!p || !p->offsets || !p->counts) return POLYLLA_EINVAL;
  if (p->cap_polys < 0 || p->cap_verts < 0) return POLYLLA_EINVAL;
  if (p->cap_verts > 0 && !p->verts) return POLYLLA_EINVAL;
  if (need_start && !p->start) return POLYLLA_EINVAL;
  return POLYLLA_OK;
}

int launched() { return hipGetLastError() == hipSuccess ? POLYLLA_OK : POLYLLA_EHIP; }

int grid_for(int64_t n, int64_t per_block, int64_t cap) {
  int64_t g = (n + per_block - 1) / per_block;
  return (int)std::max<int64_t>(1, std::min<int64_t>(g, cap));
}

void reset(polylla_ctx* c, hipStream_t s, const int64_t* n_from, int keep = 0) {
  Prof p(c, s, KR_RESET);
  hipLaunchKernelGGL(k_reset, dim3(grid_for(c->sc->n_status, 256, 4096)), dim3(256), 0, s, c->cnt, c->sc->status,
                     c->sc->n_status, n_from, keep);
}

// Seed counts per label tile (first ntiles words of the status array) and
// their sums per group of 64 tiles (the next ntiles / 64 + 1 words, zeroed by
// k_reset).
uint32_t* tile_counts(polylla_ctx* c) { return reinterpret_cast<uint32_t*>(c->sc->status); }
uint32_t* tile_groups(polylla_ctx* c, int64_t T) { return tile_counts(c) + (T + kTile - 1) / kTile; }

void launch_seeds(polylla_ctx* c, int64_t T, const uint8_t* tri, hipStream_t s) {
  Prof p(c, s, KR_SEEDS);
  hipLaunchKernelGGL(k_seeds, dim3((T + kTile - 1) / kTile), dim3(256), 0, s, T, tri, tile_counts(c),
                     tile_groups(c, T), c->sc->seeds, c->cnt);
}

// LabelMax with the context's triangles per thread; the grid also covers the
// vertex labels it clears
void launch_longest(polylla_ctx* c, const polylla_tri* t, int64_t T, uint8_t* vtx, hipStream_t s) {
  const int k = c->longest_items;
  const int grid = grid_for(std::max((T + k - 1) / k, vtx ? t->n_vertices : (int64_t)0), 256, 1 << 20);
  if (k == 1)
    hipLaunchKernelGGL(k_longest<1>, dim3(grid), dim3(256), 0, s, T, t->n_vertices, t->xy, t->origin, t->twin,
                       c->sc->lg, vtx, c->cnt);
  else if (k == 4)
    hipLaunchKernelGGL(k_longest<4>, dim3(grid), dim3(256), 0, s, T, t->n_vertices, t->xy, t->origin, t->twin,
                       c->sc->lg, vtx, c->cnt);
  else
    hipLaunchKernelGGL(k_longest<2>, dim3(grid), dim3(256), 0, s, T, t->n_vertices, t->xy, t->origin, t->twin,
                       c->sc->lg, vtx, c->cnt);
}

int run_label(polylla_ctx* c, const polylla_tri* t, uint8_t* he, uint8_t* tri, uint8_t* vtx, hipStream_t s) {
  const int64_t T = t->n_halfedges / 3;
  {
    Prof p(c, s, KR_LONGEST);
    launch_longest(c, t, T, vtx, s);
  }
  if (T > 0) {
    Prof p(c, s, KR_LABEL);
    // 16-byte loads of twin and origin need aligned arrays (the label stores
    // adapt to the alignment of he and tri)
    const bool vec = ((uintptr_t)t->twin % 16 == 0) && ((uintptr_t)t->origin % 16 == 0);
    hipLaunchKernelGGL(k_label<true>, dim3((T + kTile - 1) / kTile), dim3(256), 0, s, T, t->twin, c->sc->lg, he, tri,
                       t->origin, c->sc->wk, tile_counts(c), tile_groups(c, T), c->cnt, vec, t->fixed);
  }
  if (T > 0) launch_seeds(c, T, tri, s);
  return launched();
}

// Walk + general path + scan + emit over the list `list` of seeds (from_seeds)
// or start half-edges; n (device) polygons already in cnt->n_seeds.
int run_build(polylla_ctx* c, const polylla_tri* t, const int32_t* list, bool from_seeds, bool repair,
              uint8_t* he, uint8_t* vtx, polylla_polys* out, hipStream_t s, const polylla_polys* prep_in = nullptr,
              const BatchEmit* be = nullptr) {
  const int64_t T = t->n_halfedges / 3;
  const int32_t nhe = (int32_t)t->n_halfedges;
  PolyState ps = poly_state(c);
  if (prep_in) {
    // repair of built polygons: only those with a tip are walked again
    Prof p(c, s, KR_PREP);
    hipLaunchKernelGGL(k_repair_prep, dim3(grid_for(T, 256, 4096)), dim3(256), 0, s, prep_in->offsets, prep_in->verts,
                       prep_in->start, c->sc->stage, c->sc->stage_cap, ps, c->sc->deferred, c->sc->cap_t, c->walk_cap,
                       c->cnt);
  } else {
    Prof p(c, s, KR_WALK);
    const int gw = std::min(c->walk_blocks, c->sc->walk_grid);  // persistent: waves take seeds from per-XCD queues
    if (!from_seeds) return POLYLLA_EINTERNAL;  // a list of start half-edges is only repaired (prep_in)
    hipLaunchKernelGGL(k_walk<true>, dim3(gw), dim3(256), 0, s, list, nhe, c->sc->wk, c->sc->stage,
                       c->sc->stage_cap, ps, c->sc->deferred, c->sc->cap_t, c->walk_cap, c->cnt);
  }
  // the long regions (workgroup kernels, caller's stream) and the flagged
  // short polygons (tip path and per-lane kernels, second stream) in
  // parallel. The 1024-thread region kernel needs whole compute units (all
  // their LDS and registers): it stays on the caller's stream and the second
  // stream forks only after the one-wave instance before it, so that its few
  // workgroups are dispatched before the tip path's blocks spread over every
  // compute unit.
  hipStream_t sl = s, ss = c->side;
  // long regions: the long-cycle tip path first (cycles of up to 32 frontier
  // half-edges with no repeated vertex or one tip, when there are more long
  // cycles than one-wave workgroups), one wave per region next
  // (regions of up to 128 triangles and frontier half-edges), then 1024
  // threads per region for the rest; when there are at most `few` of them,
  // all go to the 1024-thread instance
  const uint32_t few = 128;
  {
    Prof p(c, sl, KR_TIPL);
    Counters* k = c->cnt;
    // up to one long cycle per one-wave workgroup (the default): those
    // workgroups take them all at once (the long-cycle path only copies the list)
    const uint32_t tipl_min = c->long_tip_min;
    const int gl = 1536;  // (six workgroups of 24 KB of LDS per compute unit), grid-stride
    if (repair)
      hipLaunchKernelGGL(k_tip_long<true>, dim3(gl), dim3(64), 0, sl, nhe, t->n_vertices, t->twin, t->origin, c->sc->wk,
                         he, vtx, c->sc->stage, c->sc->stage_cap, c->sc->arena, c->sc->arena_cap, ps, c->sc->deferred,
                         c->sc->cap_t, &k->n_big, few, tipl_min, c->sc->lrest, c->sc->lrest_cap, &k->n_lrest, k);
    else
      hipLaunchKernelGGL(k_tip_long<false>, dim3(gl), dim3(64), 0, sl, nhe, t->n_vertices, t->twin, t->origin, c->sc->wk,
                         he, vtx, c->sc->stage, c->sc->stage_cap, c->sc->arena, c->sc->arena_cap, ps, c->sc->deferred,
                         c->sc->cap_t, &k->n_big, few, tipl_min, c->sc->lrest, c->sc->lrest_cap, &k->n_lrest, k);
  }
  {
    Prof p(c, sl, KR_BIG);
    Counters* k = c->cnt;
    const int gm = c->sc->grid64;  // persistent: one-wave blocks take regions round-robin
    if (repair)
      hipLaunchKernelGGL((k_general_big<true, 64, 128, 128, 8>), dim3(gm), dim3(64), 0, sl, list, from_seeds, nhe,
                         t->n_vertices, t->twin, t->origin, c->sc->wk, he, vtx, c->sc->stage, c->sc->stage_cap, c->sc->arena,
                         c->sc->arena_cap, ps, c->sc->lrest, false, c->sc->lrest_cap, &k->n_lrest, &k->big_ticket, c->sc->over,
                         c->sc->over_cap, &k->n_over, nullptr, (int64_t)0, &k->n_big, few, UINT32_MAX, 128, k);
    else
      hipLaunchKernelGGL((k_general_big<false, 64, 128, 128, 8>), dim3(gm), dim3(64), 0, sl, list, from_seeds,
                         nhe, t->n_vertices, t->twin, t->origin, c->sc->wk, he, vtx, c->sc->stage, c->sc->stage_cap, c->sc->arena,
                         c->sc->arena_cap, ps, c->sc->lrest, false, c->sc->lrest_cap, &k->n_lrest, &k->big_ticket, c->sc->over,
                         c->sc->over_cap, &k->n_over, nullptr, (int64_t)0, &k->n_big, few, UINT32_MAX, 128, k);
  }
  if (hipEventRecord(c->fork, s) != hipSuccess || hipStreamWaitEvent(c->side, c->fork, 0) != hipSuccess)
    return POLYLLA_EHIP;
  {
    Prof p(c, ss, KR_TIP);
    const int gt = 2048;  // two waves per 64 short polygons with a repeat, grid-stride
    if (repair)
      hipLaunchKernelGGL(k_tip<true>, dim3(gt), dim3(128), 0, ss, nhe, t->n_vertices, t->twin, t->origin, c->sc->wk, he, vtx,
                         c->sc->stage, c->sc->stage_cap, c->sc->arena, c->sc->arena_cap, ps, c->sc->deferred, c->sc->rest, c->sc->rest_cap,
                         c->cnt);
    else
      hipLaunchKernelGGL(k_tip<false>, dim3(gt), dim3(128), 0, ss, nhe, t->n_vertices, t->twin, t->origin, c->sc->wk, he, vtx,
                         c->sc->stage, c->sc->stage_cap, c->sc->arena, c->sc->arena_cap, ps, c->sc->deferred, c->sc->rest, c->sc->rest_cap,
                         c->cnt);
  }
  // short polygons the tip path declines: up to gen_wave_max of them one wave
  // each (latency), more one lane each (throughput); each kernel reads the
  // count and the one not meant for it returns at once
  {
    Prof p(c, ss, KR_GENW);
    Counters* k = c->cnt;
    if (repair)
      hipLaunchKernelGGL((k_general_big<true, 64, 128, 128, 8>), dim3(c->sc->grid64), dim3(64), 0, ss, list, from_seeds,
                         nhe, t->n_vertices, t->twin, t->origin, c->sc->wk, he, vtx, c->sc->stage, c->sc->stage_cap, c->sc->arena,
                         c->sc->arena_cap, ps, c->sc->rest, false, (int64_t)0, &k->n_gen, nullptr, c->sc->huge, c->sc->huge_cap,
                         &k->n_fallback, nullptr, (int64_t)0, nullptr, 0u, c->gen_wave_max, 128, k);
    else
      hipLaunchKernelGGL((k_general_big<false, 64, 128, 128, 8>), dim3(c->sc->grid64), dim3(64), 0, ss, list, from_seeds,
                         nhe, t->n_vertices, t->twin, t->origin, c->sc->wk, he, vtx, c->sc->stage, c->sc->stage_cap, c->sc->arena,
                         c->sc->arena_cap, ps, c->sc->rest, false, (int64_t)0, &k->n_gen, nullptr, c->sc->huge, c->sc->huge_cap,
                         &k->n_fallback, nullptr, (int64_t)0, nullptr, 0u, c->gen_wave_max, 128, k);
  }
  {
    Prof p(c, ss, KR_GENERAL);
    const int gg = 2048;
    if (repair)
      hipLaunchKernelGGL(k_general_small<true>, dim3(gg), dim3(64), 0, ss, list, from_seeds, nhe, t->n_vertices,
                         t->twin, t->origin, c->sc->wk, he, vtx, c->sc->stage, c->sc->stage_cap, c->sc->arena, c->sc->arena_cap, ps,
                         c->sc->rest, &c->cnt->n_gen, c->gen_wave_max, c->cnt);
    else
      hipLaunchKernelGGL(k_general_small<false>, dim3(gg), dim3(64), 0, ss, list, from_seeds, nhe, t->n_vertices,
                         t->twin, t->origin, c->sc->wk, he, vtx, c->sc->stage, c->sc->stage_cap, c->sc->arena, c->sc->arena_cap, ps,
                         c->sc->rest, &c->cnt->n_gen, c->gen_wave_max, c->cnt);
  }
  if (hipEventRecord(c->join, ss) != hipSuccess) return POLYLLA_EHIP;
  {
    Prof p(c, sl, KR_BIGW);
    Counters* k = c->cnt;
    const int gb = c->sc->grid1024;  // persistent: blocks take the remaining long regions by ticket
    if (repair)
      hipLaunchKernelGGL((k_general_big<true, 1024, 4096, 4096, 13>), dim3(gb), dim3(1024), 0, sl, list,
                         from_seeds, nhe, t->n_vertices, t->twin, t->origin, c->sc->wk, he, vtx, c->sc->stage, c->sc->stage_cap,
                         c->sc->arena, c->sc->arena_cap, ps, c->sc->over, false, (int64_t)0, &k->n_over, &k->over_ticket, c->sc->huge,
                         c->sc->huge_cap, &k->n_fallback, c->sc->deferred, c->sc->cap_t, &k->n_big, few, UINT32_MAX,
                         c->lds_max, k);
    else
      hipLaunchKernelGGL((k_general_big<false, 1024, 4096, 4096, 13>), dim3(gb), dim3(1024), 0, sl, list,
                         from_seeds, nhe, t->n_vertices, t->twin, t->origin, c->sc->wk, he, vtx, c->sc->stage, c->sc->stage_cap,
                         c->sc->arena, c->sc->arena_cap, ps, c->sc->over, false, (int64_t)0, &k->n_over, &k->over_ticket, c->sc->huge,
                         c->sc->huge_cap, &k->n_fallback, c->sc->deferred, c->sc->cap_t, &k->n_big, few, UINT32_MAX,
                         c->lds_max, k);
  }
  if (hipStreamWaitEvent(s, c->join, 0) != hipSuccess) return POLYLLA_EHIP;
  {
    Prof p(c, s, KR_HUGE);
    // regions beyond the LDS instance: a workgroup each with the region in
    // global memory; beyond that, one lane each
    const int32_t kcap = (int32_t)std::min<int64_t>(c->sc->mem_km, c->mem_max);
    const int32_t lcap = 2 * kcap;
    if (repair)
      hipLaunchKernelGGL(k_general_huge<true>, dim3(kMemGrid), dim3(1024), 0, s, list, from_seeds, nhe,
                         t->n_vertices, t->twin, t->origin, c->sc->wk, he, vtx, c->sc->stage, c->sc->stage_cap, c->sc->arena,
                         c->sc->arena_cap, ps, c->sc->huge, c->sc->huge_cap, c->sc->lane, c->sc->lane_cap, c->sc->mem_store, c->sc->mem_km,
                         kcap, lcap, c->cnt);
    else
      hipLaunchKernelGGL(k_general_huge<false>, dim3(kMemGrid), dim3(1024), 0, s, list, from_seeds, nhe,
                         t->n_vertices, t->twin, t->origin, c->sc->wk, he, vtx, c->sc->stage, c->sc->stage_cap, c->sc->arena,
                         c->sc->arena_cap, ps, c->sc->huge, c->sc->huge_cap, c->sc->lane, c->sc->lane_cap, c->sc->mem_store, c->sc->mem_km,
                         kcap, lcap, c->cnt);
  }
  {
    Prof p(c, s, KR_SCAN);
    const int64_t ntiles = (T + kScanTileHost - 1) / kScanTileHost + 1;
    if (be)
      hipLaunchKernelGGL(k_scan_emit<true>, dim3(ntiles), dim3(256), 0, s, ps, c->sc->status + c->sc->n_status_label,
                         c->sc->stage, c->sc->arena, (int32_t*)nullptr, (int32_t*)nullptr, (int32_t*)nullptr,
                         (int64_t*)nullptr, (int64_t)0, (int64_t)0, c->cnt, *be, c->emit_lds_max);
    else
      hipLaunchKernelGGL(k_scan_emit<false>, dim3(ntiles), dim3(256), 0, s, ps, c->sc->status + c->sc->n_status_label,
                         c->sc->stage, c->sc->arena, out->offsets, out->verts, out->start, out->counts, out->cap_polys,
                         out->cap_verts, c->cnt, BatchEmit{}, c->emit_lds_max);
  }
  return launched();
}

// Label, build and repair of one mesh (label arrays NULL: context scratch);
// keep != 0 keeps the error word and batch sums of earlier groups.
int mesh_run(polylla_ctx* c, const polylla_tri* t, uint8_t* he, uint8_t* tri, uint8_t* vtx, polylla_polys* out,
             hipStream_t s, int keep, const BatchEmit* be = nullptr) {
  he = he ? he : c->sc->he_s;
  tri = tri ? tri : c->sc->tri_s;
  vtx = vtx ? vtx : c->sc->vtx_s;
  reset(c, s, nullptr, keep);
  int rc = run_label(c, t, he, tri, vtx, s);
  if (rc) return rc;
  return run_build(c, t, c->sc->seeds, true, true, he, vtx, out, s, nullptr, be);
}

}  // namespace

extern "C" {

int polylla_ctx_create(polylla_ctx** out, int device) {
  if (!out) return POLYLLA_EINVAL;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return POLYLLA_EINVAL;
  if (hipSetDevice(device) != hipSuccess) return POLYLLA_EHIP;
  if (device >= kMaxDevices) return POLYLLA_EINVAL;
  {
    // the device address of this device's no-alloc scratch, once per device
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    if (!g_noalloc_ptr[device]) {
      void* p = nullptr;
      if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
        (void)hipGetLastError();
        return POLYLLA_EHIP;
      }
      g_noalloc_ptr[device] = p;
    }
  }
  polylla_ctx* c = new polylla_ctx();
  c->device = device;
  if (dalloc(&c->cnt, 1)) {
    delete c;
    return POLYLLA_ENOMEM;
  }
  if (hipMemset(c->cnt, 0, sizeof(Counters)) != hipSuccess ||
      hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&c->fork, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&c->join, hipEventDisableTiming) != hipSuccess) {
    if (c->join) (void)hipEventDestroy(c->join);
    if (c->fork) (void)hipEventDestroy(c->fork);
    if (c->side) (void)hipStreamDestroy(c->side);
    dfree(&c->cnt);
    delete c;
    return POLYLLA_EHIP;
  }
  *out = c;
  return POLYLLA_OK;
}

void polylla_ctx_destroy(polylla_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  (void)hipDeviceSynchronize();
  free_scratch(c);
  free_group(c);
  if (c->gen_ws) (void)hipFree(c->gen_ws);
  dfree(&c->cnt);
  for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
  (void)hipEventDestroy(c->join);
  (void)hipEventDestroy(c->fork);
  (void)hipStreamDestroy(c->side);
  delete c;
}

int polylla_reserve(polylla_ctx* c, int64_t n_halfedges, int64_t n_vertices) {
  if (!c || n_halfedges < 0 || n_vertices < 0) return POLYLLA_EINVAL;
  return ensure(c, n_halfedges / 3, n_vertices);
}

int polylla_reserve_batch(polylla_ctx* c, int64_t n_halfedges, int64_t n_vertices, int64_t n_meshes) {
  if (!c || n_halfedges < 0 || n_vertices < 0 || n_meshes < 0) return POLYLLA_EINVAL;
  // the largest group a batch of this size forms (unless one mesh alone is larger)
  const int64_t H = std::min(n_halfedges, c->group_he);
  const int64_t V = std::min<int64_t>(n_vertices, ((int64_t)1 << 31) - 1);
  int rc = ensure(c, H / 3, V);
  if (rc) return rc;
  return ensure_group(c, H, std::max<int64_t>(n_meshes, 1));
}

int polylla_label(polylla_ctx* c, const polylla_tri* t, polylla_labels* l, hipStream_t s) {
  if (!c || !l) return POLYLLA_EINVAL;
  int rc = check_tri(t);
  if (rc) return rc;
  const int64_t T = t->n_halfedges / 3;
  if (T > 0 && (!l->he || !l->tri)) return POLYLLA_EINVAL;
  if ((rc = ensure(c, T, t->n_vertices))) return rc;
  if (hipSetDevice(c->device) != hipSuccess) return POLYLLA_EHIP;
  reset(c, s, nullptr);
  return run_label(c, t, l->he, l->tri, l->vtx, s);
}

int polylla_build(polylla_ctx* c, const polylla_tri* t, polylla_labels* l, polylla_polys* out, hipStream_t s) {
  if (!c || !l) return POLYLLA_EINVAL;
  int rc = check_tri(t);
  if (rc) return rc;
  if ((rc = check_polys(out, true))) return rc;
  const int64_t T = t->n_halfedges / 3;
  if (T > 0 && (!l->he || !l->tri || !l->vtx)) return POLYLLA_EINVAL;
  if ((rc = ensure(c, T, t->n_vertices))) return rc;
  if (hipSetDevice(c->device) != hipSuccess) return POLYLLA_EHIP;
  reset(c, s, nullptr);
  if (T > 0) {
    Prof p(c, s, KR_COMPACT);
    hipLaunchKernelGGL(k_label<false>, dim3((T + kTile - 1) / kTile), dim3(256), 0, s, T, t->twin, c->sc->lg, l->he,
                       l->tri, t->origin, c->sc->wk, tile_counts(c), tile_groups(c, T), c->cnt, false,
                       (const uint8_t*)nullptr);
  }
  if (T > 0) launch_seeds(c, T, l->tri, s);
  if (T > 0) {
    Prof p(c, s, KR_PACK);
    hipLaunchKernelGGL(k_pack_walk, dim3(grid_for(3 * T, 256, 1 << 16)), dim3(256), 0, s, 3 * T, l->he, t->twin,
                       t->origin, c->sc->wk);
  }
  return run_build(c, t, c->sc->seeds, true, false, l->he, l->vtx, out, s);
}

int polylla_repair(polylla_ctx* c, const polylla_tri* t, polylla_labels* l, const polylla_polys* in,
                   polylla_polys* out, hipStream_t s) {
  if (!c || !l) return POLYLLA_EINVAL;
  int rc = check_tri(t);
  if (rc) return rc;
  if ((rc = check_polys(in, true)) || (rc = check_polys(out, false))) return rc;
  const int64_t T = t->n_halfedges / 3;
  if (T > 0 && (!l->he || !l->vtx)) return POLYLLA_EINVAL;
  if ((rc = ensure(c, T, t->n_vertices))) return rc;
  if (hipSetDevice(c->device) != hipSuccess) return POLYLLA_EHIP;
  reset(c, s, in->counts);
  if (T > 0) {
    Prof p(c, s, KR_PACK);
    hipLaunchKernelGGL(k_pack_walk, dim3(grid_for(3 * T, 256, 1 << 16)), dim3(256), 0, s, 3 * T, l->he, t->twin,
                       t->origin, c->sc->wk);
  }
  return run_build(c, t, in->start, false, true, l->he, l->vtx, out, s, in);
}

int polylla_mesh(polylla_ctx* c, const polylla_tri* t, polylla_labels* l, polylla_polys* out, hipStream_t s) {
  if (!c) return POLYLLA_EINVAL;
  int rc = check_tri(t);
  if (rc) return rc;
  if ((rc = check_polys(out, false))) return rc;
  const int64_t T = t->n_halfedges / 3;
  if ((rc = ensure(c, T, t->n_vertices))) return rc;
  if (hipSetDevice(c->device) != hipSuccess) return POLYLLA_EHIP;
  c->last_batched = false;
  return mesh_run(c, t, l ? l->he : nullptr, l ? l->tri : nullptr, l ? l->vtx : nullptr, out, s, 0);
}

int polylla_lepp(polylla_ctx* c, const polylla_tri* t, int32_t* terminal, int32_t* length, hipStream_t s) {
  if (!c) return POLYLLA_EINVAL;
  int rc = check_tri(t);
  if (rc) return rc;
  const int64_t T = t->n_halfedges / 3;
  if (T > 0 && (!terminal || !length)) return POLYLLA_EINVAL;
  if ((rc = ensure(c, T, t->n_vertices))) return rc;
  if (hipSetDevice(c->device) != hipSuccess) return POLYLLA_EHIP;
  c->last_batched = false;
  reset(c, s, nullptr);
  if (T == 0) return launched();
  Scratch* S = c->sc;
  {
    Prof p(c, s, KR_LONGEST);  // LabelMax: the Max byte of every triangle
    launch_longest(c, t, T, nullptr, s);
  }
  // path states in two int4 arrays over the staging (>= 5T ints) and arena
  // (>= 6T ints) scratch, the unfinished paths listed in the seed array
  int4* sa = reinterpret_cast<int4*>(S->stage);
  int4* sb = reinterpret_cast<int4*>(S->arena);
  uint32_t* n_list = &c->cnt->n_lepp;
  Prof p(c, s, KR_LEPP);
  hipLaunchKernelGGL(k_lepp_chase, dim3((T + 255) / 256), dim3(256), 0, s, T, S->lg, t->twin, t->fixed, terminal,
                     length, sa, S->seeds, n_list, c->cnt);
  // every round doubles the path length covered: 2^26 * 32 triangles at most
  constexpr int kRounds = 26;
  for (int r = 0; r < kRounds; ++r) {
    hipLaunchKernelGGL(k_lepp_jump, dim3(grid_for(T, 256, 1024)), dim3(256), 0, s, terminal, length,
                       (const int4*)(r % 2 ? sb : sa), r % 2 ? sa : sb, S->seeds, n_list);
  }
  hipLaunchKernelGGL(k_lepp_finish, dim3(grid_for(T, 256, 1024)), dim3(256), 0, s, terminal, length,
                     (const int4*)(kRounds % 2 ? sb : sa), S->seeds, n_list, c->cnt);
  return launched();
}

int polylla_mesh_mixed(polylla_ctx* c, const polylla_tri* t, const int32_t* twin_host, const int32_t* origin_host,
                       uint8_t* he_host, polylla_polys* out, double* seconds, hipStream_t s) {
  using clock = std::chrono::steady_clock;
  const auto t0 = clock::now();
  if (!c || !he_host || !twin_host || !origin_host) return POLYLLA_EINVAL;
  int rc = check_tri(t);
  if (rc) return rc;
  if ((rc = check_polys(out, false))) return rc;
  const int64_t H = t->n_halfedges, T = H / 3;
  if ((rc = ensure(c, T, t->n_vertices))) return rc;
  if ((rc = ensure_group(c, std::max<int64_t>(H, 3), 1))) return rc;
  if (hipSetDevice(c->device) != hipSuccess) return POLYLLA_EHIP;
  c->last_batched = false;
  // label and traversal on the device, the polygons before repair into scratch CSR
  Scratch* S = c->sc;
  polylla_polys pre{c->g_off, c->g_verts, c->g_start, c->g_counts, std::max<int64_t>(T, 1),
                    std::max<int64_t>(H, 3)};
  reset(c, s, nullptr);
  if ((rc = run_label(c, t, S->he_s, S->tri_s, S->vtx_s, s))) return rc;
  if ((rc = run_build(c, t, S->seeds, true, false, S->he_s, S->vtx_s, &pre, s))) return rc;
  if ((rc = polylla_status(c, s))) return rc;
  const auto t1 = clock::now();
  int64_t cnt[2] = {0, 0};
  if (hipMemcpy(cnt, c->g_counts, sizeof(cnt), hipMemcpyDeviceToHost) != hipSuccess) return POLYLLA_EHIP;
  const int64_t F = cnt[0], Sv = cnt[1];
  std::vector<int32_t> off((size_t)F + 1), verts((size_t)std::max<int64_t>(Sv, 1)), start((size_t)std::max<int64_t>(F, 1));
  if (hipMemcpy(he_host, S->he_s, (size_t)H, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(off.data(), c->g_off, sizeof(int32_t) * (size_t)(F + 1), hipMemcpyDeviceToHost) != hipSuccess ||
      (Sv > 0 && hipMemcpy(verts.data(), c->g_verts, sizeof(int32_t) * (size_t)Sv, hipMemcpyDeviceToHost) != hipSuccess) ||
      (F > 0 && hipMemcpy(start.data(), c->g_start, sizeof(int32_t) * (size_t)F, hipMemcpyDeviceToHost) != hipSuccess))
    return POLYLLA_EHIP;
  const auto t2 = clock::now();
  // the reparation phase, sequential on the host
  int64_t st[2];
  rc = host_repair(H, twin_host, origin_host, he_host, F, off.data(), verts.data(), start.data(), out->offsets,
                   out->verts, out->start, out->cap_polys, out->cap_verts, out->counts, st);
  const auto t3 = clock::now();
  if (seconds) {
    seconds[0] = std::chrono::duration<double>(t1 - t0).count();
    seconds[1] = std::chrono::duration<double>(t2 - t1).count();
    seconds[2] = std::chrono::duration<double>(t3 - t2).count();
  }
  return rc;
}

int polylla_mesh_noalloc(polylla_ctx* c, const polylla_tri* t, polylla_labels* l, polylla_polys* out,
                         hipStream_t s) {
  if (!c) return POLYLLA_EINVAL;
  int rc = check_tri(t);
  if (rc) return rc;
  if ((rc = check_polys(out, false))) return rc;
  const int64_t T = t->n_halfedges / 3;
  if (T > kNoallocMaxTri || t->n_vertices > kNoallocMaxVtx) return POLYLLA_ETOOBIG;
  void* base = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    base = g_noalloc_ptr[c->device];
  }
  if (!base) return POLYLLA_EHIP;
  // the scratch arrays as slices of this device's static array (the same
  // layout as a context's own scratch, sized for this mesh and the smaller
  // launch grids used here)
  Scratch view;
  const int64_t Tv = std::max<int64_t>(T, 1024), Vv = std::max<int64_t>(t->n_vertices, 1024);
  if (carve(view, nullptr, Tv, Vv, kNoallocWalkGrid, kNoallocGrid64, kNoallocGrid1024, kNoallocMemKm) >
      kNoallocBytes)
    return POLYLLA_ETOOBIG;
  carve(view, static_cast<uint8_t*>(base), Tv, Vv, kNoallocWalkGrid, kNoallocGrid64, kNoallocGrid1024,
        kNoallocMemKm);
  if (hipSetDevice(c->device) != hipSuccess) return POLYLLA_EHIP;
  const int prof = c->prof;  // event records would grow a host vector
  c->prof = POLYLLA_PROFILE_OFF;
  c->sc = &view;
  c->last_batched = false;
  rc = mesh_run(c, t, l ? l->he : nullptr, l ? l->tri : nullptr, l ? l->vtx : nullptr, out, s, 0);
  c->sc = &c->own;
  c->prof = prof;
  return rc;
}

int polylla_mesh_batched(polylla_ctx* c, const polylla_batch* b, polylla_labels* l, polylla_batch_out* out,
                         hipStream_t s) {
  if (!c || !b || !out || b->n_meshes < 0) return POLYLLA_EINVAL;
  const int64_t n = b->n_meshes;
  if (!b->vtx_off || !b->he_off || !b->vtx_off_host || !b->he_off_host || !out->offsets || !out->poly_off ||
      !out->counts || out->cap_polys < 0 || out->cap_verts < 0 || (out->cap_verts > 0 && !out->verts))
    return POLYLLA_EINVAL;
  const int64_t* ho = b->he_off_host;
  const int64_t* vo = b->vtx_off_host;
  if (ho[0] != 0 || vo[0] != 0) return POLYLLA_EINVAL;
  for (int64_t m = 0; m < n; ++m) {
    const int64_t dh = ho[m + 1] - ho[m], dv = vo[m + 1] - vo[m];
    if (dh < 0 || dv < 0) return POLYLLA_EINVAL;
    if (dh % 3) return POLYLLA_ELAYOUT;
    if (dh >= ((int64_t)1 << 31) - 64 || dv >= ((int64_t)1 << 31)) return POLYLLA_EINVAL;
  }
  if (ho[n] > 0 && (!b->xy || !b->twin || !b->origin)) return POLYLLA_EINVAL;
  // groups of consecutive meshes [first[k], first[k + 1]) of at most group_he
  // half-edges (a larger mesh alone) and fewer than 2^31 vertices
  std::vector<int64_t> first;
  int64_t max_he = 0, max_v = 0, max_m = 1;
  for (int64_t m = 0; m < n;) {
    first.push_back(m);
    int64_t e = m + 1;
    while (e < n && ho[e + 1] - ho[m] <= c->group_he && vo[e + 1] - vo[m] < ((int64_t)1 << 31)) ++e;
    max_he = std::max(max_he, ho[e] - ho[m]);
    max_v = std::max(max_v, vo[e] - vo[m]);
    max_m = std::max(max_m, e - m);
    m = e;
  }
  first.push_back(n);
  int rc = ensure(c, max_he / 3, max_v);
  if (rc) return rc;
  if ((rc = ensure_group(c, max_he, max_m))) return rc;
  if (hipSetDevice(c->device) != hipSuccess) return POLYLLA_EHIP;
  c->last_batched = true;
  {
    Prof p(c, s, KR_BATCH);
    hipLaunchKernelGGL(k_batch_begin, dim3(1), dim3(64), 0, s, c->g_base);
  }
  const size_t ng = first.size() - 1;
  if (ng == 0) {  // no meshes: F = 0, offsets[0] = 0, poly_off[0] = 0
    reset(c, s, nullptr);
    hipLaunchKernelGGL(k_group_advance, dim3(1), dim3(64), 0, s, (const int64_t*)c->g_base + 3, c->g_base, true, n,
                       out->offsets, out->poly_off, out->counts, out->cap_polys, out->cap_verts,
                       (const Counters*)c->cnt);
    return launched();
  }
  for (size_t k = 0; k < ng; ++k) {
    const int64_t m0 = first[k], m1 = first[k + 1], nm = m1 - m0;
    const int64_t h0 = ho[m0], H = ho[m1] - h0, v0 = vo[m0], V = vo[m1] - v0;
    if (H > 0) {
      Prof p(c, s, KR_GREBASE);
      hipLaunchKernelGGL(k_group_rebase, dim3(grid_for(H, 256, 1 << 16)), dim3(256), 0, s, b->twin, b->origin,
                         c->g_twin, c->g_origin, nm, b->he_off + m0, b->vtx_off + m0);
    }
    polylla_tri tg{V, H, b->xy + 2 * v0, c->g_twin, nullptr, c->g_origin, b->fixed ? b->fixed + h0 : nullptr};
    polylla_polys pg{nullptr, nullptr, nullptr, c->g_counts, H / 3, H};
    uint8_t* he = (l && l->he) ? l->he + h0 : nullptr;
    uint8_t* tri = (l && l->tri) ? l->tri + h0 / 3 : nullptr;
    uint8_t* vtx = (l && l->vtx) ? l->vtx + v0 : nullptr;
    // the emitter writes the group's polygons into the caller's CSR itself
    const BatchEmit be{c->sc->seeds, nm, b->he_off + m0, b->vtx_off + m0, c->g_base, out->offsets, out->verts,
                       out->start, out->poly_off + m0, out->cap_polys, out->cap_verts, c->g_counts};
    if ((rc = mesh_run(c, &tg, he, tri, vtx, &pg, s, k > 0 ? 1 : 0, &be))) return rc;
    {
      Prof p(c, s, KR_BATCH);
      hipLaunchKernelGGL(k_accumulate, dim3(1), dim3(64), 0, s, c->cnt);
      hipLaunchKernelGGL(k_batch_empty, dim3(grid_for(nm, 256, 4096)), dim3(256), 0, s, nm, b->he_off + m0, c->g_base,
                         c->g_counts, out->poly_off + m0, (const Counters*)c->cnt);
    }
    {
      Prof p(c, s, KR_BATCH);
      hipLaunchKernelGGL(k_group_advance, dim3(1), dim3(64), 0, s, c->g_counts, c->g_base, k + 1 == ng, n,
                         out->offsets, out->poly_off, out->counts, out->cap_polys, out->cap_verts,
                         (const Counters*)c->cnt);
    }
  }
  {
    Prof p(c, s, KR_BATCH);
    hipLaunchKernelGGL(k_batch_close, dim3(grid_for(n + 1, 256, 4096)), dim3(256), 0, s, c->g_base, n,
                       out->poly_off);
  }
  return launched();
}

int polylla_gen_grid(polylla_ctx* c, int64_t g, double jitter, uint64_t seed, double* xy, int32_t* twin,
                     int32_t* origin, int64_t cap_halfedges, int64_t* n_halfedges, int32_t* flip_rounds,
                     hipStream_t s) {
  if (!c || !xy || !twin || !origin || !n_halfedges) return POLYLLA_EINVAL;
  if (g < 2 || g > kGenGridMax || !(jitter >= 0.0 && jitter < 0.5)) return POLYLLA_EINVAL;
  if (cap_halfedges < 6 * g * g) return POLYLLA_ECAPACITY;
  if (hipSetDevice(c->device) != hipSuccess) return POLYLLA_EHIP;
  const size_t need = gen_ws_bytes(g);
  if (need > c->gen_ws_cap) {
    if (hipStreamSynchronize(s) != hipSuccess) return POLYLLA_EHIP;
    if (c->gen_ws) (void)hipFree(c->gen_ws);
    c->gen_ws = nullptr;
    c->gen_ws_cap = 0;
    if (hipMalloc(&c->gen_ws, need) != hipSuccess) {
      (void)hipGetLastError();
      c->gen_ws = nullptr;
      return POLYLLA_ENOMEM;
    }
    c->gen_ws_cap = need;
  }
  c->last_batched = false;
  hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, s, c->cnt, (uint64_t*)nullptr, (int64_t)0,
                     (const int64_t*)nullptr, 0);
  int64_t T = 0;
  int rounds = 0;
  int rc = gen_grid_run(g, jitter, seed, xy, twin, origin, cap_halfedges / 3, c->gen_ws, c->cnt, s, &T, &rounds);
  const int st = polylla_status(c, s);
  if (rc == POLYLLA_OK) rc = st;
  if (rc) return rc;
  *n_halfedges = 3 * T;
  if (flip_rounds) *flip_rounds = rounds;
  return POLYLLA_OK;
}

int polylla_validate(polylla_ctx* c, const polylla_tri* t, hipStream_t s) {
  if (!c) return POLYLLA_EINVAL;
  int rc = check_tri(t);
  if (rc) return rc;
  if (t->n_halfedges > 0 && !t->next) return POLYLLA_EINVAL;
  if (hipSetDevice(c->device) != hipSuccess) return POLYLLA_EHIP;
  hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, s, c->cnt, (uint64_t*)nullptr, (int64_t)0,
                     (const int64_t*)nullptr, 0);
  Prof pv(c, s, KR_VALIDATE);
  hipLaunchKernelGGL(k_validate, dim3(grid_for(t->n_halfedges, 256, 1 << 16)), dim3(256), 0, s, t->n_halfedges,
                     t->n_vertices, t->twin, t->next, t->origin, t->fixed, c->cnt);
  if ((rc = launched())) return rc;
  return polylla_status(c, s);
}

int polylla_status(polylla_ctx* c, hipStream_t s) {
  if (!c) return POLYLLA_EINVAL;
  if (hipSetDevice(c->device) != hipSuccess) return POLYLLA_EHIP;
  if (hipStreamSynchronize(s) != hipSuccess) return POLYLLA_EHIP;
  Counters h;
  if (hipMemcpy(&h, c->cnt, sizeof(Counters), hipMemcpyDeviceToHost) != hipSuccess) return POLYLLA_EHIP;
  c->last = h;
  if (h.error) {
    int32_t zero = 0;
    if (hipMemcpy(&c->cnt->error, &zero, sizeof(zero), hipMemcpyHostToDevice) != hipSuccess) return POLYLLA_EHIP;
  }
  return h.error;
}

int polylla_stats(polylla_ctx* c, int64_t* out, int n) {
  if (!c || !out || n < 0) return POLYLLA_EINVAL;
  int64_t v[7] = {c->last.n_seeds, c->last.n_deferred, c->last.n_tips, c->last.n_splits,
                  c->last.n_big,   c->last.n_fallback, c->last.n_lane};
  if (c->last_batched)
    for (int i = 0; i < 7; ++i) v[i] = (int64_t)c->last.acc[i];
  int k = std::min(n, 7);
  for (int i = 0; i < k; ++i) out[i] = v[i];
  return k;
}

int polylla_set_param(polylla_ctx* c, int param, int64_t value) {
  if (!c) return POLYLLA_EINVAL;
  switch (param) {
    case POLYLLA_PARAM_WALK_CAP:
      if (value < 1 || value > 24) return POLYLLA_EINVAL;
      c->walk_cap = (int)value;
      return POLYLLA_OK;
    case POLYLLA_PARAM_WALK_BLOCKS:
      if (value < 8 || value > kWalkBlocks || value % 8) return POLYLLA_EINVAL;
      c->walk_blocks = (int)value;
      return POLYLLA_OK;
    case POLYLLA_PARAM_GEN_WAVE_MAX:
      if (value < 0 || value > UINT32_MAX - 1) return POLYLLA_EINVAL;
      c->gen_wave_max = (uint32_t)value;
      return POLYLLA_OK;
    case POLYLLA_PARAM_REGION_LDS_MAX:
      if (value < 32 || value > 4096) return POLYLLA_EINVAL;
      c->lds_max = (int32_t)value;
      return POLYLLA_OK;
    case POLYLLA_PARAM_REGION_MEM_MAX:
      if (value < 32 || value > kMemRegionMax) return POLYLLA_EINVAL;
      c->mem_max = (int32_t)value;
      return POLYLLA_OK;
    case POLYLLA_PARAM_BATCH_GROUP_HE:
      if (value < 3 || value > kGroupHeMax) return POLYLLA_EINVAL;
      c->group_he = value;
      return POLYLLA_OK;
    case POLYLLA_PARAM_LONGEST_ITEMS:
      if (value != 1 && value != 2 && value != 4) return POLYLLA_EINVAL;
      c->longest_items = (int)value;
      return POLYLLA_OK;
    case POLYLLA_PARAM_LONG_TIP_MIN:
      if (value < 0 || value > UINT32_MAX - 1) return POLYLLA_EINVAL;
      c->long_tip_min = (uint32_t)value;
      return POLYLLA_OK;
    case POLYLLA_PARAM_EMIT_LDS_MAX:
      if (value < 0 || value > kScanTileHost + 512) return POLYLLA_EINVAL;
      c->emit_lds_max = (int32_t)value;
      return POLYLLA_OK;
    default:
      return POLYLLA_EINVAL;
  }
}

int polylla_profile(polylla_ctx* c, int enable) {
  if (!c || enable < 0 || enable > POLYLLA_PROFILE_WALK) return POLYLLA_EINVAL;
  if (hipSetDevice(c->device) != hipSuccess) return POLYLLA_EHIP;
  if (enable) {
    (void)hipDeviceSynchronize();
    while (c->ev_pool.size() < 2 * kMaxProfiled) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return POLYLLA_EHIP;
      c->ev_pool.push_back(e);
    }
    c->recs.clear();
  }
  c->prof = enable;
  return POLYLLA_OK;
}

int polylla_profile_read(polylla_ctx* c, char* names, double* ms, int64_t* launches, int n) {
  if (!c || n < 0 || (n > 0 && (!names || !ms || !launches))) return POLYLLA_EINVAL;
  if (hipSetDevice(c->device) != hipSuccess) return POLYLLA_EHIP;
  if (hipDeviceSynchronize() != hipSuccess) return POLYLLA_EHIP;
  double sum[KR_N] = {0};
  int64_t cnt[KR_N] = {0};
  for (const auto& r : c->recs) {
    float t = 0.f;
    if (hipEventElapsedTime(&t, r.a, r.b) != hipSuccess) return POLYLLA_EHIP;
    sum[r.kernel] += t;
    cnt[r.kernel] += 1;
  }
  int w = 0;
  for (int k = 0; k < KR_N && w < n; ++k) {
    if (!cnt[k]) continue;
    strncpy(names + 32 * w, kKernelNames[k], 31);
    names[32 * w + 31] = 0;
    ms[w] = sum[k];
    launches[w] = cnt[k];
    ++w;
  }
  return w;
}

const char* polylla_strerror(int code) {
  switch (code) {
    case POLYLLA_OK: return "ok";
    case POLYLLA_EINVAL: return "invalid argument";
    case POLYLLA_ELAYOUT: return "half-edge layout: n_halfedges % 3 != 0 or next not grouped";
    case POLYLLA_ETOPO: return "invalid topology: index out of range or twin inconsistent";
    case POLYLLA_ECAPACITY: return "output capacity too small";
    case POLYLLA_ENOMEM: return "device scratch allocation failed";
    case POLYLLA_EHIP: return "HIP runtime error";
    case POLYLLA_EDEGEN: return "walk bound exceeded (not a valid triangulation)";
    case POLYLLA_EINTERNAL: return "internal error: device scan did not complete";
    case POLYLLA_ETOOBIG: return "mesh larger than the no-alloc scratch (262144 triangles, 262144 vertices)";
    default: return "unknown error";
  }
}

}  // extern "C"
