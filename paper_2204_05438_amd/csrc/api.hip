// Host side of libpolylla: contexts, scratch, argument checks and the kernel
// sequence of every entry point declared in include/polylla.h.
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "common.h"

namespace polylla {

__global__ void k_reset(Counters*, uint64_t*, int64_t, const int64_t*);
__global__ void k_longest(int64_t, int64_t, const double*, const int32_t*, const int32_t*, uint8_t*, uint8_t*,
                          Counters*);
template <bool COMPUTE>
__global__ void k_label(int64_t, const int32_t*, const uint8_t*, uint8_t*, uint8_t*, const int32_t*, int32_t*,
                        uint32_t*, uint32_t*, Counters*, bool);
__global__ void k_seeds(int64_t, const uint8_t*, const uint32_t*, const uint32_t*, int32_t*, Counters*);
__global__ void k_pack_walk(int64_t, const uint8_t*, const int32_t*, const int32_t*, int32_t*);
template <bool FROM_SEEDS>
__global__ void k_walk(const int32_t*, int32_t, const int32_t*, int32_t*, int64_t, PolyState, int32_t*, int64_t, int,
                       Counters*);
template <bool REPAIR>
__global__ void k_general_small(const int32_t*, bool, int32_t, int64_t, const int32_t*, const int32_t*,
                                const int32_t*, uint8_t*, uint8_t*, int32_t*, int64_t, int32_t*, int64_t, PolyState,
                                const int32_t*, const uint32_t*, uint32_t, Counters*);
template <bool REPAIR>
__global__ void k_tip(int32_t, int64_t, const int32_t*, const int32_t*, uint8_t*, uint8_t*, int32_t*, int64_t,
                      int32_t*, int64_t, PolyState, const int32_t*, int32_t*, int64_t, Counters*);
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
__global__ void k_scan_emit(PolyState, uint64_t*, const int32_t*, const int32_t*, int32_t*, int32_t*, int32_t*,
                            int64_t*, int64_t, int64_t, Counters*);
__global__ void k_validate(int64_t, int64_t, const int32_t*, const int32_t*, const int32_t*, Counters*);
__global__ void k_rebase(int32_t*, int32_t*, int64_t, const int64_t*, const int64_t*);
__global__ void k_batch_offsets(int64_t, const int64_t*, const int32_t*, const int32_t*, const int64_t*, int64_t,
                                int64_t, int64_t*);

}  // namespace polylla

using namespace polylla;

// default number of declined short polygons up to which each gets a wave
constexpr uint32_t kGenWaveMax = 2 * polylla::kBigGrid64;

struct polylla_ctx {
  int device = 0;
  Counters* cnt = nullptr;
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
  int32_t* poly_arrays = nullptr;  // per-polygon records: 4 ints + 1 int per polygon (PolyState)
  int32_t* stage = nullptr;
  int64_t stage_cap = 0;
  int32_t* arena = nullptr;
  int64_t arena_cap = 0;
  uint64_t* status = nullptr;
  int64_t n_status = 0;
  uint8_t* he_s = nullptr;
  uint8_t* tri_s = nullptr;
  uint8_t* vtx_s = nullptr;
  Counters last{};
  int walk_cap = 24;  // vertices a lane walks before handing a polygon to a workgroup
  uint32_t gen_wave_max = kGenWaveMax;  // declined short polygons up to which each gets a wave
  int32_t lds_max = 4096;               // region size limit of the 1024-thread LDS workgroup
  int32_t mem_max = (int32_t)kMemRegionMax;  // region size limit of the global-memory workgroup
  int walk_blocks = 640;  // persistent grid of the walk kernel (swept at 10M: 512 851, 640 782, 768 791 us)
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

constexpr int64_t kTile = 2048;  // triangles per tile of k_label
constexpr size_t kMaxProfiled = 8192;
constexpr int64_t kScanTileHost = 2048;   // polygons per tile of k_scan_emit
constexpr int64_t kWalkBlocks = 2048;     // persistent grid of k_walk
constexpr int64_t kWalkWaves = kWalkBlocks * 4;
constexpr int64_t kStageChunkHost = 4096; // staging ints a walk wave reserves at a time
// unused tails of the staging and arena chunks of the region workgroups (two
// launches of the one-wave instance, one of the 1024-thread instance)
constexpr int64_t kBigStageTails = 2 * (int64_t)kBigGrid64 * kBigStageChunk64 + (int64_t)kBigGrid1024 * kBigStageChunk1024;
constexpr int64_t kBigArenaTails = 2 * (int64_t)kBigGrid64 * kBigArenaChunk64 + (int64_t)kBigGrid1024 * kBigArenaChunk1024;

enum KernelId {
  KR_RESET, KR_LONGEST, KR_LABEL, KR_COMPACT, KR_PACK, KR_WALK, KR_GENERAL, KR_BIG, KR_HUGE, KR_SCAN, KR_VALIDATE,
  KR_BATCH, KR_BIGW, KR_TIP, KR_SEEDS, KR_GENW, KR_N
};
const char* kKernelNames[KR_N] = {"k_reset",         "k_longest",       "k_label",          "k_compact_seeds",
                                  "k_pack_walk",     "k_walk",          "k_general_small",  "k_general_big",
                                  "k_general_huge",  "k_scan_emit",     "k_validate",       "k_batch_offsets",
                                  "k_general_big_wg", "k_tip",           "k_seeds",          "k_general_wave"};

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
  dfree(&c->lg);
  dfree(&c->wk);
  dfree(&c->seeds);
  dfree(&c->deferred);
  dfree(&c->huge);
  dfree(&c->lane);
  dfree(&c->mem_store);
  dfree(&c->over);
  dfree(&c->rest);
  dfree(&c->poly_arrays);
  dfree(&c->stage);
  dfree(&c->arena);
  dfree(&c->status);
  dfree(&c->he_s);
  dfree(&c->tri_s);
  dfree(&c->vtx_s);
  c->cap_t = c->cap_v = 0;
}

int ensure(polylla_ctx* c, int64_t nt, int64_t nv) {
  if (nt <= c->cap_t && nv <= c->cap_v && c->lg) return POLYLLA_OK;
  int64_t T = std::max(nt, c->cap_t), V = std::max(nv, c->cap_v);
  if (hipSetDevice(c->device) != hipSuccess) return POLYLLA_EHIP;
  (void)hipDeviceSynchronize();
  free_scratch(c);
  T = std::max<int64_t>(T, 1024);
  V = std::max<int64_t>(V, 1024);
  int rc = POLYLLA_OK;
  const int64_t ntiles = (T + kTile - 1) / kTile + 1;
  // polygon vertices (<= 3T) and the general paths' staging, plus the unused
  // tail of the last staging chunk of every walk wave. Offsets stay int32.
  c->stage_cap = std::min<int64_t>(5 * T + kWalkWaves * kStageChunkHost + kBigStageTails + ((int64_t)1 << 20),
                                   ((int64_t)1 << 31) - 1);
  c->arena_cap = 6 * T + kBigArenaTails + 4096;
  c->n_status = 2 * ntiles;
  if ((rc = dalloc(&c->lg, T)) || (rc = dalloc(&c->wk, 3 * T)) || (rc = dalloc(&c->seeds, T)) || (rc = dalloc(&c->deferred, T)) || (rc = dalloc(&c->huge, c->huge_cap = 3 * T / 32 + 64)) ||
      (rc = dalloc(&c->lane, c->lane_cap = 3 * T / 32 + 64)) ||
      (rc = dalloc(&c->mem_store, kMemGrid * mem_words(c->mem_km = std::min<int64_t>(T, kMemRegionMax)))) ||
      (rc = dalloc(&c->over, c->over_cap = T / 32 + 64)) ||
      (rc = dalloc(&c->rest, c->rest_cap = T / 3 + 64)) ||
      (rc = dalloc(&c->poly_arrays, 5 * T)) || (rc = dalloc(&c->stage, c->stage_cap)) ||
      (rc = dalloc(&c->arena, c->arena_cap)) || (rc = dalloc(&c->status, c->n_status)) ||
      (rc = dalloc(&c->he_s, 3 * T)) || (rc = dalloc(&c->tri_s, T)) || (rc = dalloc(&c->vtx_s, V))) {
    free_scratch(c);
    return rc;
  }
  c->cap_t = T;
  c->cap_v = V;
  return POLYLLA_OK;
}

PolyState poly_state(polylla_ctx* c) {
  PolyState ps;
  ps.rec = reinterpret_cast<int4*>(c->poly_arrays);
  ps.prec = c->poly_arrays + 4 * c->cap_t;
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

void reset(polylla_ctx* c, hipStream_t s, const int64_t* n_from) {
  Prof p(c, s, KR_RESET);
  hipLaunchKernelGGL(k_reset, dim3(grid_for(c->n_status, 256, 4096)), dim3(256), 0, s, c->cnt, c->status,
                     c->n_status, n_from);
}

// Seed counts per label tile (first ntiles words of the status array) and
// their sums per group of 64 tiles (the next ntiles / 64 + 1 words, zeroed by
// k_reset).
uint32_t* tile_counts(polylla_ctx* c) { return reinterpret_cast<uint32_t*>(c->status); }
uint32_t* tile_groups(polylla_ctx* c, int64_t T) { return tile_counts(c) + (T + kTile - 1) / kTile; }

void launch_seeds(polylla_ctx* c, int64_t T, const uint8_t* tri, hipStream_t s) {
  Prof p(c, s, KR_SEEDS);
  hipLaunchKernelGGL(k_seeds, dim3((T + kTile - 1) / kTile), dim3(256), 0, s, T, tri, tile_counts(c),
                     tile_groups(c, T), c->seeds, c->cnt);
}

int run_label(polylla_ctx* c, const polylla_tri* t, uint8_t* he, uint8_t* tri, uint8_t* vtx, hipStream_t s) {
  const int64_t T = t->n_halfedges / 3;
  {
    Prof p(c, s, KR_LONGEST);
    // two triangles per thread (and one vertex to clear)
    hipLaunchKernelGGL(k_longest, dim3(grid_for(std::max((T + 1) / 2, t->n_vertices), 256, 1 << 20)), dim3(256), 0,
                       s, T, t->n_vertices, t->xy, t->origin, t->twin, c->lg, vtx, c->cnt);
  }
  if (T > 0) {
    Prof p(c, s, KR_LABEL);
    // 16-byte loads of twin and 4-byte label stores need aligned arrays
    const bool vec = ((uintptr_t)t->twin % 16 == 0) && ((uintptr_t)t->origin % 16 == 0) && ((uintptr_t)he % 4 == 0) &&
                     ((uintptr_t)tri % 4 == 0);
    hipLaunchKernelGGL(k_label<true>, dim3((T + kTile - 1) / kTile), dim3(256), 0, s, T, t->twin, c->lg, he, tri,
                       t->origin, c->wk, tile_counts(c), tile_groups(c, T), c->cnt, vec);
  }
  if (T > 0) launch_seeds(c, T, tri, s);
  return launched();
}

// Walk + general path + scan + emit over the list `list` of seeds (from_seeds)
// or start half-edges; n (device) polygons already in cnt->n_seeds.
int run_build(polylla_ctx* c, const polylla_tri* t, const int32_t* list, bool from_seeds, bool repair,
              uint8_t* he, uint8_t* vtx, polylla_polys* out, hipStream_t s) {
  const int64_t T = t->n_halfedges / 3;
  const int32_t nhe = (int32_t)t->n_halfedges;
  PolyState ps = poly_state(c);
  {
    Prof p(c, s, KR_WALK);
    const int gw = c->walk_blocks;  // persistent: waves take seeds from per-XCD queues
    if (from_seeds)
      hipLaunchKernelGGL(k_walk<true>, dim3(gw), dim3(256), 0, s, list, nhe, c->wk, c->stage,
                         c->stage_cap, ps, c->deferred, c->cap_t, c->walk_cap, c->cnt);
    else
      hipLaunchKernelGGL(k_walk<false>, dim3(gw), dim3(256), 0, s, list, nhe, c->wk, c->stage,
                         c->stage_cap, ps, c->deferred, c->cap_t, c->walk_cap, c->cnt);
  }
  // the long regions (workgroup kernel, side stream) and the short ones
  // (per-lane kernel, caller's stream) in parallel
  if (hipEventRecord(c->fork, s) != hipSuccess || hipStreamWaitEvent(c->side, c->fork, 0) != hipSuccess)
    return POLYLLA_EHIP;
  // long regions: one wave per region first (regions of up to 128 triangles
  // and frontier half-edges), then 1024 threads per region for the rest; when
  // there are at most `few` of them, all go to the 1024-thread instance
  const uint32_t few = 128;
  {
    Prof p(c, c->side, KR_BIG);
    Counters* k = c->cnt;
    const int gm = kBigGrid64;  // persistent: one-wave blocks take regions round-robin
    if (repair)
      hipLaunchKernelGGL((k_general_big<true, 64, 128, 128, 8>), dim3(gm), dim3(64), 0, c->side, list, from_seeds, nhe,
                         t->n_vertices, t->twin, t->origin, c->wk, he, vtx, c->stage, c->stage_cap, c->arena,
                         c->arena_cap, ps, c->deferred, true, c->cap_t, &k->n_big, &k->big_ticket, c->over,
                         c->over_cap, &k->n_over, nullptr, (int64_t)0, &k->n_big, few, UINT32_MAX, 128, k);
    else
      hipLaunchKernelGGL((k_general_big<false, 64, 128, 128, 8>), dim3(gm), dim3(64), 0, c->side, list, from_seeds,
                         nhe, t->n_vertices, t->twin, t->origin, c->wk, he, vtx, c->stage, c->stage_cap, c->arena,
                         c->arena_cap, ps, c->deferred, true, c->cap_t, &k->n_big, &k->big_ticket, c->over,
                         c->over_cap, &k->n_over, nullptr, (int64_t)0, &k->n_big, few, UINT32_MAX, 128, k);
  }
  {
    Prof p(c, c->side, KR_BIGW);
    Counters* k = c->cnt;
    const int gb = kBigGrid1024;  // persistent: blocks take the remaining long regions by ticket
    if (repair)
      hipLaunchKernelGGL((k_general_big<true, 1024, 4096, 4096, 13>), dim3(gb), dim3(1024), 0, c->side, list,
                         from_seeds, nhe, t->n_vertices, t->twin, t->origin, c->wk, he, vtx, c->stage, c->stage_cap,
                         c->arena, c->arena_cap, ps, c->over, false, (int64_t)0, &k->n_over, &k->over_ticket, c->huge,
                         c->huge_cap, &k->n_fallback, c->deferred, c->cap_t, &k->n_big, few, UINT32_MAX,
                         c->lds_max, k);
    else
      hipLaunchKernelGGL((k_general_big<false, 1024, 4096, 4096, 13>), dim3(gb), dim3(1024), 0, c->side, list,
                         from_seeds, nhe, t->n_vertices, t->twin, t->origin, c->wk, he, vtx, c->stage, c->stage_cap,
                         c->arena, c->arena_cap, ps, c->over, false, (int64_t)0, &k->n_over, &k->over_ticket, c->huge,
                         c->huge_cap, &k->n_fallback, c->deferred, c->cap_t, &k->n_big, few, UINT32_MAX,
                         c->lds_max, k);
  }
  if (hipEventRecord(c->join, c->side) != hipSuccess) return POLYLLA_EHIP;
  {
    Prof p(c, s, KR_TIP);
    const int gt = 2048;  // one lane per short polygon with a repeat, grid-stride
    if (repair)
      hipLaunchKernelGGL(k_tip<true>, dim3(gt), dim3(64), 0, s, nhe, t->n_vertices, t->twin, t->origin, he, vtx,
                         c->stage, c->stage_cap, c->arena, c->arena_cap, ps, c->deferred, c->rest, c->rest_cap,
                         c->cnt);
    else
      hipLaunchKernelGGL(k_tip<false>, dim3(gt), dim3(64), 0, s, nhe, t->n_vertices, t->twin, t->origin, he, vtx,
                         c->stage, c->stage_cap, c->arena, c->arena_cap, ps, c->deferred, c->rest, c->rest_cap,
                         c->cnt);
  }
  // short polygons the tip path declines: up to gen_wave_max of them one wave
  // each (latency), more one lane each (throughput); each kernel reads the
  // count and the one not meant for it returns at once
  {
    Prof p(c, s, KR_GENW);
    Counters* k = c->cnt;
    if (repair)
      hipLaunchKernelGGL((k_general_big<true, 64, 128, 128, 8>), dim3(kBigGrid64), dim3(64), 0, s, list, from_seeds,
                         nhe, t->n_vertices, t->twin, t->origin, c->wk, he, vtx, c->stage, c->stage_cap, c->arena,
                         c->arena_cap, ps, c->rest, false, (int64_t)0, &k->n_gen, nullptr, c->huge, c->huge_cap,
                         &k->n_fallback, nullptr, (int64_t)0, nullptr, 0u, c->gen_wave_max, 128, k);
    else
      hipLaunchKernelGGL((k_general_big<false, 64, 128, 128, 8>), dim3(kBigGrid64), dim3(64), 0, s, list, from_seeds,
                         nhe, t->n_vertices, t->twin, t->origin, c->wk, he, vtx, c->stage, c->stage_cap, c->arena,
                         c->arena_cap, ps, c->rest, false, (int64_t)0, &k->n_gen, nullptr, c->huge, c->huge_cap,
                         &k->n_fallback, nullptr, (int64_t)0, nullptr, 0u, c->gen_wave_max, 128, k);
  }
  {
    Prof p(c, s, KR_GENERAL);
    const int gg = 2048;
    if (repair)
      hipLaunchKernelGGL(k_general_small<true>, dim3(gg), dim3(64), 0, s, list, from_seeds, nhe, t->n_vertices,
                         t->twin, t->origin, c->wk, he, vtx, c->stage, c->stage_cap, c->arena, c->arena_cap, ps,
                         c->rest, &c->cnt->n_gen, c->gen_wave_max, c->cnt);
    else
      hipLaunchKernelGGL(k_general_small<false>, dim3(gg), dim3(64), 0, s, list, from_seeds, nhe, t->n_vertices,
                         t->twin, t->origin, c->wk, he, vtx, c->stage, c->stage_cap, c->arena, c->arena_cap, ps,
                         c->rest, &c->cnt->n_gen, c->gen_wave_max, c->cnt);
  }
  if (hipStreamWaitEvent(s, c->join, 0) != hipSuccess) return POLYLLA_EHIP;
  {
    Prof p(c, s, KR_HUGE);
    // regions beyond the LDS instance: a workgroup each with the region in
    // global memory; beyond that, one lane each
    const int32_t kcap = (int32_t)std::min<int64_t>(c->mem_km, c->mem_max);
    const int32_t lcap = 2 * kcap;
    if (repair)
      hipLaunchKernelGGL(k_general_huge<true>, dim3(kMemGrid), dim3(1024), 0, s, list, from_seeds, nhe,
                         t->n_vertices, t->twin, t->origin, c->wk, he, vtx, c->stage, c->stage_cap, c->arena,
                         c->arena_cap, ps, c->huge, c->huge_cap, c->lane, c->lane_cap, c->mem_store, c->mem_km,
                         kcap, lcap, c->cnt);
    else
      hipLaunchKernelGGL(k_general_huge<false>, dim3(kMemGrid), dim3(1024), 0, s, list, from_seeds, nhe,
                         t->n_vertices, t->twin, t->origin, c->wk, he, vtx, c->stage, c->stage_cap, c->arena,
                         c->arena_cap, ps, c->huge, c->huge_cap, c->lane, c->lane_cap, c->mem_store, c->mem_km,
                         kcap, lcap, c->cnt);
  }
  {
    Prof p(c, s, KR_SCAN);
    const int64_t ntiles = (T + kScanTileHost - 1) / kScanTileHost + 1;
    hipLaunchKernelGGL(k_scan_emit, dim3(ntiles), dim3(256), 0, s, ps, c->status + c->n_status / 2, c->stage,
                       c->arena, out->offsets, out->verts, out->start, out->counts, out->cap_polys,
                       out->cap_verts, c->cnt);
  }
  return launched();
}

}  // namespace

extern "C" {

int polylla_ctx_create(polylla_ctx** out, int device) {
  if (!out) return POLYLLA_EINVAL;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return POLYLLA_EINVAL;
  if (hipSetDevice(device) != hipSuccess) return POLYLLA_EHIP;
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
    hipLaunchKernelGGL(k_label<false>, dim3((T + kTile - 1) / kTile), dim3(256), 0, s, T, t->twin, c->lg, l->he,
                       l->tri, t->origin, c->wk, tile_counts(c), tile_groups(c, T), c->cnt, false);
  }
  if (T > 0) launch_seeds(c, T, l->tri, s);
  if (T > 0) {
    Prof p(c, s, KR_PACK);
    hipLaunchKernelGGL(k_pack_walk, dim3(grid_for(3 * T, 256, 1 << 16)), dim3(256), 0, s, 3 * T, l->he, t->twin,
                       t->origin, c->wk);
  }
  return run_build(c, t, c->seeds, true, false, l->he, l->vtx, out, s);
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
                       t->origin, c->wk);
  }
  return run_build(c, t, in->start, false, true, l->he, l->vtx, out, s);
}

int polylla_mesh(polylla_ctx* c, const polylla_tri* t, polylla_labels* l, polylla_polys* out, hipStream_t s) {
  if (!c) return POLYLLA_EINVAL;
  int rc = check_tri(t);
  if (rc) return rc;
  if ((rc = check_polys(out, false))) return rc;
  const int64_t T = t->n_halfedges / 3;
  if ((rc = ensure(c, T, t->n_vertices))) return rc;
  if (hipSetDevice(c->device) != hipSuccess) return POLYLLA_EHIP;
  uint8_t* he = (l && l->he) ? l->he : c->he_s;
  uint8_t* tri = (l && l->tri) ? l->tri : c->tri_s;
  uint8_t* vtx = (l && l->vtx) ? l->vtx : c->vtx_s;
  reset(c, s, nullptr);
  if ((rc = run_label(c, t, he, tri, vtx, s))) return rc;
  return run_build(c, t, c->seeds, true, true, he, vtx, out, s);
}

int polylla_mesh_batched(polylla_ctx* c, const polylla_tri* t, int64_t n_meshes, const int64_t* vtx_off,
                         polylla_labels* l, polylla_polys* out, int64_t* poly_off, hipStream_t s) {
  if (!c || n_meshes < 0 || (n_meshes > 0 && (!vtx_off || !poly_off))) return POLYLLA_EINVAL;
  int rc = polylla_mesh(c, t, l, out, s);
  if (rc) return rc;
  if (n_meshes >= 0 && poly_off) {
    Prof p(c, s, KR_BATCH);
    hipLaunchKernelGGL(k_batch_offsets, dim3(grid_for(n_meshes + 1, 256, 4096)), dim3(256), 0, s, n_meshes,
                       vtx_off, out->offsets, out->verts, out->counts, out->cap_polys, out->cap_verts, poly_off);
  }
  return launched();
}

int polylla_rebase(int32_t* twin, int32_t* origin, int64_t n_meshes, const int64_t* he_off, const int64_t* vtx_off,
                   hipStream_t s) {
  if (n_meshes < 0 || (n_meshes > 0 && (!twin || !origin || !he_off || !vtx_off))) return POLYLLA_EINVAL;
  if (n_meshes == 0) return POLYLLA_OK;
  hipLaunchKernelGGL(k_rebase, dim3(4096), dim3(256), 0, s, twin, origin, n_meshes, he_off, vtx_off);
  return launched();
}

int polylla_validate(polylla_ctx* c, const polylla_tri* t, hipStream_t s) {
  if (!c) return POLYLLA_EINVAL;
  int rc = check_tri(t);
  if (rc) return rc;
  if (t->n_halfedges > 0 && !t->next) return POLYLLA_EINVAL;
  if (hipSetDevice(c->device) != hipSuccess) return POLYLLA_EHIP;
  hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, s, c->cnt, (uint64_t*)nullptr, (int64_t)0,
                     (const int64_t*)nullptr);
  Prof pv(c, s, KR_VALIDATE);
  hipLaunchKernelGGL(k_validate, dim3(grid_for(t->n_halfedges, 256, 1 << 16)), dim3(256), 0, s, t->n_halfedges,
                     t->n_vertices, t->twin, t->next, t->origin, c->cnt);
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
  const int64_t v[7] = {c->last.n_seeds,  c->last.n_deferred, c->last.n_tips, c->last.n_splits,
                        c->last.n_big,    c->last.n_fallback, c->last.n_lane};
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
    default: return "unknown error";
  }
}

}  // extern "C"
