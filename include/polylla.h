/*
 * polylla.h -- C ABI of the MI355X (gfx950) terminal-edge-region polygonal
 * mesher: label -> build -> repair, after Salinas, Ojeda, Hitschfeld and
 * Ortiz-Bernardin, "GPU parallel algorithm for the generation of polygonal
 * meshes based on terminal-edge regions" (SIAM IMR 2022, arXiv 2204.05438).
 *
 * Conventions for every call below
 * ---------------------------------
 *  - Pointers inside polylla_tri / polylla_labels / polylla_polys are DEVICE
 *    pointers owned by the caller; the library never frees or reallocates them.
 *  - Calls enqueue work on `stream` and return without waiting. Host-side
 *    argument errors are returned immediately; errors found by the kernels
 *    (bad indices, exhausted capacity) are recorded in the context and read
 *    with polylla_status(), which waits for the stream.
 *  - Device scratch is owned by the context and grows on demand (hipMalloc on
 *    the first call at a larger size; see polylla_reserve()). Calls sharing a
 *    context must be ordered on one stream; use one context per stream.
 *  - Output is deterministic: the same input gives byte-identical output.
 *
 * Input triangulation (the paper's Vertex, Triangle and Neighbor arrays, in
 * half-edge form; section "Data structure")
 * ----------------------------------------------------------------------
 *  half-edge h belongs to triangle t = h / 3 and runs from origin[h] to
 *  origin[next[h]]; next[3t+i] == 3t + (i+1) % 3 (grouped layout; the hot path
 *  relies on it and does not read `next`, polylla_validate() checks it);
 *  triangles are counter-clockwise; twin[h] is the opposite half-edge of the
 *  same edge, -1 on the boundary. n_halfedges must be a multiple of 3 and below
 *  2^31; vertex ids below 2^31.
 *
 * Labels (Label phase, Algorithm 2; Reparation phase, Algorithm 4)
 * ----------------------------------------------------------------
 *  he[h]  bit 1 LONGEST  : h is the longest edge of its triangle. Squared
 *                           lengths in IEEE binary64 without contraction; equal
 *                           lengths are ordered by the edge key min(h, twin[h])
 *                           (h on the boundary), smaller key wins.
 *         bit 2 FRONTIER : boundary edge, or longest edge of neither triangle,
 *                           or an edge opened by the repair.
 *         bit 4 TERMINAL : longest edge of both triangles, or a boundary edge
 *                           that is the longest edge of its triangle.
 *         bit 8 BORDER   : twin[h] == -1.
 *         bit 16 BARRIER : frontier edge whose two half-edges lie on the same
 *                           polygon before repair (set by build / repair / mesh).
 *         bit 32 REPAIRED: frontier edge opened by the repair.
 *         bit 64 CONSTRAINED: a side of a segment of the input (polylla_tri.fixed).
 *                           A segment bounds the domain on both of its sides,
 *                           so each side is labelled like a boundary edge:
 *                           FRONTIER always, TERMINAL (and its triangle a
 *                           SEED) where it is the longest edge of its triangle.
 *                           The paper meshes such inputs (its guinea-pig PSLG);
 *                           holes are triangles absent from the input.
 *  tri[t] bit 1 SEED     : t is the lower-index triangle of a terminal edge (or
 *                           the triangle of a boundary terminal edge).
 *  vtx[v] bit 1 TIP      : v is a barrier-edge tip before repair.
 *
 * Polygons (the paper's Mesh and Position arrays, as CSR)
 * -------------------------------------------------------
 *  polygon p has vertices verts[offsets[p] .. offsets[p+1]), counter-clockwise,
 *  rotated to its lexicographically smallest vertex sequence (so it starts at
 *  its smallest vertex id). start[p] is the half-edge leaving verts[offsets[p]]
 *  along the cycle. Polygons are listed in increasing seed-triangle order; the
 *  pieces of a repaired polygon take its place, ordered by their (first,
 *  second) vertex. counts[0] = number of polygons F, counts[1] = sum of their
 *  lengths (= n_tri + 2F). cap_polys >= n_tri and cap_verts >= 3 * n_tri are
 *  always enough; smaller capacities are checked on the device (ECAPACITY).
 *
 * Repair reading (Algorithm 4 leaves it open): the tips of a polygon are
 * handled in increasing vertex id. At tip v with barrier half-edge c0 (leaving
 * v) and degree d, the edge opened is c_{floor(d/2)} where c_{j+1} =
 * next[twin[c_j]] (clockwise about v). A tip whose vertex already lies on an
 * edge opened for a smaller tip is no longer a tip and is skipped.
 */
#ifndef POLYLLA_H
#define POLYLLA_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* return codes */
#define POLYLLA_OK 0
#define POLYLLA_EINVAL (-1)    /* null pointer, negative size, size limit exceeded */
#define POLYLLA_ELAYOUT (-2)   /* n_halfedges % 3 != 0 or next not grouped */
#define POLYLLA_ETOPO (-3)     /* index out of range, twin not an involution (device) */
#define POLYLLA_ECAPACITY (-4) /* output capacity too small (device) */
#define POLYLLA_ENOMEM (-5)    /* scratch allocation failed */
#define POLYLLA_EHIP (-6)      /* a HIP runtime call failed */
#define POLYLLA_EDEGEN (-7)    /* walk bound exceeded: input not a valid triangulation */
#define POLYLLA_EINTERNAL (-8) /* a device-wide scan did not complete (library bug) */
#define POLYLLA_ETOOBIG (-9)   /* mesh larger than polylla_mesh_noalloc takes */

/* label bits */
#define POLYLLA_LONGEST 1u
#define POLYLLA_FRONTIER 2u
#define POLYLLA_TERMINAL 4u
#define POLYLLA_BORDER 8u
#define POLYLLA_BARRIER 16u
#define POLYLLA_REPAIRED 32u
#define POLYLLA_CONSTRAINED 64u
#define POLYLLA_SEED 1u
#define POLYLLA_TIP 1u

typedef struct polylla_ctx polylla_ctx;

typedef struct {
  int64_t n_vertices;
  int64_t n_halfedges;
  const double *xy;       /* [2 * n_vertices], x0 y0 x1 y1 ... */
  const int32_t *twin;    /* [n_halfedges], -1 on the boundary */
  const int32_t *next;    /* [n_halfedges], grouped (see above); may be NULL except for polylla_validate */
  const int32_t *origin;  /* [n_halfedges] */
  const uint8_t *fixed;   /* [n_halfedges] or NULL: nonzero on both half-edges of a segment of an input
                             planar straight-line graph (see CONSTRAINED below) */
} polylla_tri;

typedef struct {
  uint8_t *he;   /* [n_halfedges] */
  uint8_t *tri;  /* [n_halfedges / 3] */
  uint8_t *vtx;  /* [n_vertices] */
} polylla_labels;

typedef struct {
  int32_t *offsets;   /* [cap_polys + 1] */
  int32_t *verts;     /* [cap_verts] */
  int32_t *start;     /* [cap_polys]; may be NULL for polylla_mesh outputs */
  int64_t *counts;    /* [2] device: F, sum of lengths */
  int64_t cap_polys;
  int64_t cap_verts;
} polylla_polys;

/* Create a context bound to HIP device `device`. */
int polylla_ctx_create(polylla_ctx **out, int device);
/* Release a context and its scratch (waits for the device). */
void polylla_ctx_destroy(polylla_ctx *ctx);
/* Pre-allocate scratch for meshes up to n_halfedges / n_vertices (optional). */
int polylla_reserve(polylla_ctx *ctx, int64_t n_halfedges, int64_t n_vertices);
/* Pre-allocate scratch for batches (polylla_mesh_batched) of up to
 * n_halfedges and n_vertices in total and n_meshes meshes (optional: a
 * batched call grows the scratch to its own size). */
int polylla_reserve_batch(polylla_ctx *ctx, int64_t n_halfedges, int64_t n_vertices, int64_t n_meshes);

/* Label phase (Algorithm 2: LabelMax, LabelSeed, LabelFrontier): writes
 * LONGEST, FRONTIER, TERMINAL, BORDER for every half-edge, SEED for every
 * triangle and clears vtx. BARRIER, REPAIRED and TIP are left clear. */
int polylla_label(polylla_ctx *ctx, const polylla_tri *tri, polylla_labels *labels, hipStream_t stream);

/* Traversal phase (Algorithm 3 with PolyConstruction): one polygon per seed,
 * before repair. Reads the labels written by polylla_label; adds BARRIER and
 * TIP. `out->start` must not be NULL (polylla_repair needs it). */
int polylla_build(polylla_ctx *ctx, const polylla_tri *tri, polylla_labels *labels,
                  polylla_polys *out, hipStream_t stream);

/* Reparation phase (Algorithm 4, run until no barrier-edge tip remains):
 * `in` must be the output of polylla_build on the same labels, which must not
 * have been repaired before. Adds FRONTIER | REPAIRED on the opened edges.
 * Polygons of `in` without a tip are copied as they are; only those with one
 * are walked again. `in` and `out` must not overlap. */
int polylla_repair(polylla_ctx *ctx, const polylla_tri *tri, polylla_labels *labels,
                   const polylla_polys *in, polylla_polys *out, hipStream_t stream);

/* Algorithm 1 in one call: label, build and repair. `labels` may be NULL
 * (then labels live in context scratch). Same result as the three calls. */
int polylla_mesh(polylla_ctx *ctx, const polylla_tri *tri, polylla_labels *labels,
                 polylla_polys *out, hipStream_t stream);

/* Longest-edge propagation path of every triangle (Rivara's Lepp, the basis of
 * the Lepp-based algorithms the paper's conclusions name as the next use of
 * its label kernels; it reuses LabelMax, Algorithm 2). Lepp(t) starts at t and
 * steps to the neighbour across the current triangle's longest edge (the
 * LONGEST order above) until that edge is also the neighbour's longest edge,
 * a terminal edge, or is a boundary or segment side. terminal (device
 * int32 [n_tri]) receives the key of that edge (its smaller half-edge; the
 * half-edge itself on a boundary or segment side), length (device int32
 * [n_tri]) the number of triangles on the path. All the triangles of one
 * terminal-edge region end at its terminal edge. Paths longer than 32
 * triangles are finished by pointer jumping over the unfinished ones. */
int polylla_lepp(polylla_ctx *ctx, const polylla_tri *tri, int32_t *terminal, int32_t *length, hipStream_t stream);

/* Algorithm 1 in the paper's "mixed" configuration (section "GPU parallel
 * algorithm": the reparation phase gains little in parallel, so the sequential
 * version of it is used): label and traversal run on the device as in
 * polylla_label + polylla_build, then the polygons before repair and the edge
 * labels are copied to the host, where the polygons with barrier-edge tips are
 * repaired one by one (Algorithm 4 repeated until no tip is left, in the
 * repair reading above). The result equals polylla_mesh's. Synchronous: waits
 * for `stream`. tri holds device arrays; twin_host and origin_host are host
 * copies of tri->twin and tri->origin; he_host (host, [n_halfedges]) receives
 * the final half-edge labels; `out` holds HOST arrays (offsets, verts, start
 * may be NULL, counts). seconds (host, [3], may be NULL) receives the time of
 * the device part, of the copies to the host and of the host repair. Returns
 * host errors, device errors of the device part (as polylla_status), or
 * ECAPACITY / EDEGEN from the host repair. */
int polylla_mesh_mixed(polylla_ctx *ctx, const polylla_tri *tri, const int32_t *twin_host, const int32_t *origin_host,
                       uint8_t *he_host, polylla_polys *out, double *seconds, hipStream_t stream);

/* polylla_mesh for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same result as polylla_mesh (same kernels) with all scratch in a static
 * device array of the library (64 MiB per GPU, held from the library's load
 * until the process ends) instead of the context's scratch. The call itself
 * allocates nothing; `ctx` supplies the device, the counters read by
 * polylla_status, the tuning parameters and its second stream. Meshes of up
 * to 262144 triangles and 262144 vertices; larger ones return POLYLLA_ETOOBIG
 * at once. `labels` may be NULL (labels then live in the static array too).
 * Every call on a GPU shares that GPU's array and it keeps the last call's
 * contents, so calls that overlap on one GPU (other streams or contexts)
 * race; order them. Event profiling is off during the call. */
int polylla_mesh_noalloc(polylla_ctx *ctx, const polylla_tri *tri, polylla_labels *labels, polylla_polys *out,
                         hipStream_t stream);

/* A batch of independent triangulations stored one after another (CSR of
 * meshes, each mesh in the layout of polylla_tri). Mesh m owns vertices
 * [vtx_off[m], vtx_off[m+1]) of xy and half-edges [he_off[m], he_off[m+1])
 * of twin and origin, and its twin and origin entries are LOCAL to the mesh:
 * vertex ids count from the mesh's first vertex, half-edge ids (and twin)
 * from its first half-edge. The offsets are int64, so a batch may hold more
 * than 2^31 half-edges in total; each mesh holds fewer than 2^31 - 64
 * half-edges (a multiple of 3) and fewer than 2^31 vertices. The offsets are
 * given twice: on the device (read by the kernels) and on the host (the
 * library splits the batch into launches from them, so a captured HIP graph
 * replays the same launches); both copies must hold the same values. */
typedef struct {
  int64_t n_meshes;
  const int64_t *vtx_off;       /* device [n_meshes + 1], vtx_off[0] == 0, non-decreasing */
  const int64_t *he_off;        /* device [n_meshes + 1], he_off[0] == 0, non-decreasing, multiples of 3 */
  const int64_t *vtx_off_host;  /* host copy of vtx_off */
  const int64_t *he_off_host;   /* host copy of he_off */
  const double *xy;             /* device [2 * vtx_off[n_meshes]] */
  const int32_t *twin;          /* device [he_off[n_meshes]], local, -1 on the boundary */
  const int32_t *origin;        /* device [he_off[n_meshes]], local */
  const uint8_t *fixed;         /* device [he_off[n_meshes]] or NULL: segment flags as in polylla_tri */
} polylla_batch;

/* Polygons of a batch: one CSR over all meshes, meshes in order, each mesh's
 * polygons as polylla_mesh gives them for that mesh alone. Offsets are int64;
 * vertex ids (verts) and half-edge ids (start) are LOCAL to the polygon's
 * mesh. poly_off[m] is the first polygon of mesh m and poly_off[n_meshes] = F
 * (all -1 when the output capacity was too small). cap_polys >= total
 * triangles and cap_verts >= 3 * total triangles are always enough. */
typedef struct {
  int64_t *offsets;   /* device [cap_polys + 1] */
  int32_t *verts;     /* device [cap_verts] */
  int32_t *start;     /* device [cap_polys], may be NULL */
  int64_t *poly_off;  /* device [n_meshes + 1] */
  int64_t *counts;    /* device [2]: F, sum of lengths */
  int64_t cap_polys;
  int64_t cap_verts;
} polylla_batch_out;

/* Algorithm 1 on every mesh of a batch in one call on one stream. Terminal-
 * edge regions never cross a mesh boundary, so the library runs the label,
 * traversal and repair kernels once over a group of consecutive meshes at a
 * time (as many as keep its int32 scratch indices in range, by default up to
 * 2^30 - 2^24 half-edges; POLYLLA_PARAM_BATCH_GROUP_HE lowers it): the
 * group's twin and origin are first rewritten into scratch with indices over
 * the group, and its polygons are written into `out` with the mesh-local ids
 * restored. `labels` (NULL allowed) holds the label arrays of the whole
 * batch (he [he_off[n]], tri [he_off[n] / 3], vtx [vtx_off[n]]). The same
 * results as n_meshes calls of polylla_mesh, up to the offsets of the CSR.
 * Scratch grows on the first call at a given size; a call of the same size
 * can then be captured in a HIP graph. Host-side errors: EINVAL (null
 * pointers, offsets not increasing, a mesh too large), ELAYOUT (a mesh's
 * half-edges not a multiple of 3); device-side ones as for polylla_mesh. */
int polylla_mesh_batched(polylla_ctx *ctx, const polylla_batch *batch, polylla_labels *labels,
                         polylla_batch_out *out, hipStream_t stream);

/* On-device input (so that a caller with no host mesh sends nothing over
 * PCIe): writes the Delaunay triangulation of a jittered g x g point grid
 * into device arrays in the layout above. Point of cell (i, j), 0 <= i, j < g:
 * ((i + 0.5 + jitter (2u - 1)) / g, (j + 0.5 + jitter (2w - 1)) / g), with
 * u, w in [0, 1) the top 53 bits of SplitMix64 (Steele, Lea and Flood 2014)
 * at counters 2c and 2c + 1, c = j g + i, seeded by `seed`, then rounded to
 * the nearest multiple of 2^-28 (so the orientation and in-circle tests are
 * exact integers). The triangulation is unique for points with no four on a
 * circle. Vertex ids: 32 x 32 tiles of grid points in tile-row order (row by
 * row within a tile), so that neighbouring triangles have nearby ids;
 * triangles: two per grid cell in the same tiled order, then those that fill
 * the dents of the boundary; the arrays are otherwise what any Delaunay
 * triangulation of the points in this layout holds, up to the numbering.
 * Arguments: 2 <= g <= 18000; 0 <= jitter < 0.5 (cells stay convex
 * quadrilaterals); xy (device, [2 g^2] doubles); twin, origin (device,
 * [cap_halfedges] int32, cap_halfedges >= 6 g^2, else ECAPACITY);
 * n_halfedges (host) receives 3 x the triangle count (2 g^2 - 2 - hull
 * vertices); flip_rounds (host, may be NULL) the number of rounds of parallel
 * edge flips. Synchronous: waits for `stream` (the flip rounds are launched in
 * batches and a count is read on the host after each). Allocates a work space
 * of about 50 g^2 bytes, kept by the context.
 * Errors: EINVAL for bad arguments, ENOMEM, EDEGEN if the flips do not end,
 * EINTERNAL on a work-space overflow. */
int polylla_gen_grid(polylla_ctx *ctx, int64_t g, double jitter, uint64_t seed, double *xy, int32_t *twin,
                     int32_t *origin, int64_t cap_halfedges, int64_t *n_halfedges, int32_t *flip_rounds,
                     hipStream_t stream);

/* Full input check on the device (layout of next, index ranges, twin
 * involution and endpoints). Waits for the stream; returns the first error. */
int polylla_validate(polylla_ctx *ctx, const polylla_tri *tri, hipStream_t stream);

/* Waits for `stream` and returns the first device-side error recorded by the
 * context since the previous polylla_status call (then clears it). */
int polylla_status(polylla_ctx *ctx, hipStream_t stream);

/* Diagnostics of the last build / repair / mesh call, after polylla_status:
 * out[0] seeds, out[1] short polygons with a tip or a repeated vertex (one
 * lane each), out[2] tips, out[3] opened edges, out[4] long polygons (one
 * workgroup each), out[5] regions beyond the LDS of the 1024-thread
 * workgroup (one workgroup each, region kept in global memory), out[6]
 * regions beyond that path's store as well (one lane each). Returns the
 * number of values written (<= n). */
int polylla_stats(polylla_ctx *ctx, int64_t *out, int n);

/* Tuning parameters of a context (defaults are the tuned values).
 * POLYLLA_PARAM_WALK_CAP (1..24, default 24): the longest cycle one lane walks
 * and stages by itself; longer polygons are built by a whole workgroup. Small
 * values route more polygons through the cooperative kernel (used by tests).
 * Returns POLYLLA_EINVAL for an unknown parameter or a value out of range. */
#define POLYLLA_PARAM_WALK_CAP 1
/* POLYLLA_PARAM_WALK_BLOCKS (8..2048, multiple of 8): workgroups of 256
 * threads of the walk kernel; fewer keep the polygons in flight within each
 * XCD's L2, more hide more latency. Default 1280; at most six per compute
 * unit are resident (1536), so a larger grid only adds workgroups that find
 * no work. */
#define POLYLLA_PARAM_WALK_BLOCKS 2
/* POLYLLA_PARAM_GEN_WAVE_MAX (0..2^32-2, default 8192): the short polygons
 * with a repeated vertex that the single-tip path declines are repaired one
 * wave per polygon when there are at most this many (lowest latency), else
 * one lane per polygon (highest throughput). */
#define POLYLLA_PARAM_GEN_WAVE_MAX 3
/* POLYLLA_PARAM_REGION_LDS_MAX (32..4096, default 4096): regions with more
 * triangles or frontier half-edges than this are not built by the 1024-thread
 * workgroup out of LDS but by the global-memory workgroup path. Lower values
 * exercise that path (used by tests). */
#define POLYLLA_PARAM_REGION_LDS_MAX 4
/* POLYLLA_PARAM_REGION_MEM_MAX (32..65536, default 65536): regions with more
 * triangles than this, or more than twice as many frontier half-edges, are
 * not built by the global-memory workgroup path but one lane each. Its store
 * holds min(triangles of the mesh, 65536) triangles per workgroup (8
 * workgroups, about 260 bytes per triangle of capacity). */
#define POLYLLA_PARAM_REGION_MEM_MAX 5
/* POLYLLA_PARAM_BATCH_GROUP_HE (3..2^30 - 2^24, default 2^30 - 2^24): the
 * most half-edges polylla_mesh_batched runs in one group of consecutive
 * meshes (a larger mesh forms a group of its own). Lower values split a
 * batch into more groups (used by tests). */
#define POLYLLA_PARAM_BATCH_GROUP_HE 6
/* POLYLLA_PARAM_LONGEST_ITEMS (1, 2 or 4, default 2): triangles per thread of
 * the longest-edge kernel (LabelMax): each thread issues the loads of that many
 * triangles before it uses any. */
#define POLYLLA_PARAM_LONGEST_ITEMS 7
/* POLYLLA_PARAM_LONG_TIP_MIN (0..2^32-2, default 4096, the one-wave region
 * workgroups): with more cycles longer than the walk cap than this, the
 * long-cycle tip path walks each again (up to 32 frontier half-edges) and
 * finishes those without a repeated vertex or with one tip; with at most this
 * many, every long cycle gets a one-wave region workgroup at once, which is
 * sooner. Lower values exercise the long-cycle path (used by tests). */
#define POLYLLA_PARAM_LONG_TIP_MIN 8
/* POLYLLA_PARAM_EMIT_LDS_MAX (0..1536, default 1536): the most output
 * polygons of one emitter tile (1024 polygon records) whose offsets and start
 * half-edges are staged in LDS and stored coalesced; a tile with more writes
 * them directly. Lower values exercise the direct path (used by tests). */
#define POLYLLA_PARAM_EMIT_LDS_MAX 9
int polylla_set_param(polylla_ctx *ctx, int param, int64_t value);

/* Per-kernel GPU timing with HIP events, for benchmarks (off by default).
 * polylla_profile(ctx, POLYLLA_PROFILE_ALL) clears earlier records and records
 * an event pair on the launching stream around every kernel launched by later
 * calls (up to 8192 launches); POLYLLA_PROFILE_WALK does the same for the walk
 * kernel only (two events per call, so that timing a whole call is barely
 * disturbed); POLYLLA_PROFILE_OFF stops recording. Other values:
 * POLYLLA_EINVAL. polylla_profile_read waits for the device and fills, for up
 * to n kernels, the kernel name (NUL-terminated, 32 bytes per entry in
 * `names`), the summed milliseconds and the number of launches; it returns the
 * number of kernels written. */
#define POLYLLA_PROFILE_OFF 0
#define POLYLLA_PROFILE_ALL 1
#define POLYLLA_PROFILE_WALK 2
int polylla_profile(polylla_ctx *ctx, int enable);
int polylla_profile_read(polylla_ctx *ctx, char *names, double *ms, int64_t *launches, int n);

const char *polylla_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* POLYLLA_H */
