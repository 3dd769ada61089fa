// On-device input generation: a jittered g x g point grid and its Delaunay
// triangulation built on the GPU, written straight into the arrays the
// mesher reads (no host generation, no host-to-device copy).
//
// Points: cell (i, j) holds ((i + 0.5 + jitter * (2u - 1)) / g,
// (j + 0.5 + jitter * (2u' - 1)) / g) with u, u' from the counter-based
// SplitMix64 generator (seed, 2c) and (seed, 2c + 1), c = j g + i, snapped to
// multiples of 2^-28 like the host generator (so orientation and in-circle
// tests are exact in 64/128-bit integers). jitter < 0.5 keeps every row
// x-monotone and every column y-monotone, so every cell quad is a simple
// polygon and one of its diagonals splits it into two counter-clockwise
// triangles.
//
// Triangulation: (1) every cell splits its quad (the Delaunay diagonal when
// both are valid); (2) the four boundary chains are made convex one side per
// thread (a monotone-chain scan that fills every dent with a triangle), and
// a last scan over the four chains' hulls fills the corners; (3) parallel
// Lawson flips: every round each edge that fails the in-circle test claims
// its two triangles and their (up to) four neighbours with a hashed
// priority, the edges holding all their claims flip at once (no two flips
// touch the same triangle or a neighbour of one), until no edge fails. The
// result is the Delaunay triangulation of the points (unique for points with
// no four on a circle).
//
// Numbering: vertices and cells in 32 x 32 tiles of cells (tile rows, tiles
// within a row, rows within a tile), two triangles per cell in cell order,
// then the triangles filling the boundary dents; a tile of cells is 2048
// triangles, the label kernels' tile.
#include <algorithm>
#include <vector>

#include "common.h"

namespace polylla {

constexpr int kGenTile = 32;
constexpr int64_t kLatScale = (int64_t)1 << 28;

__host__ __device__ inline uint64_t splitmix64(uint64_t seed, uint64_t k) {
  uint64_t z = seed + (k + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// vertex (and cell) id of grid position (i, j) in the tiled numbering
__device__ __forceinline__ int64_t grid_id(int64_t i, int64_t j, int64_t g) {
  const int64_t tj = j / kGenTile, ti = i / kGenTile;
  const int64_t hj = min<int64_t>(kGenTile, g - kGenTile * tj), wi = min<int64_t>(kGenTile, g - kGenTile * ti);
  return kGenTile * g * tj + (int64_t)kGenTile * hj * ti + (j - kGenTile * tj) * wi + (i - kGenTile * ti);
}

// cell id of cell (i, j) of the (g-1) x (g-1) cells
__device__ __forceinline__ int64_t cell_id(int64_t i, int64_t j, int64_t g) { return grid_id(i, j, g - 1); }

__device__ __forceinline__ int64_t orient(int64_t ax, int64_t ay, int64_t bx, int64_t by, int64_t cx, int64_t cy) {
  return (bx - ax) * (cy - ay) - (by - ay) * (cx - ax);  // |terms| < 2^57
}

// > 0 when d lies inside the circle through a, b, c (counter-clockwise):
// first in binary64 with the static error bound of Shewchuk's incircle
// predicate (Adaptive Precision Floating-Point Arithmetic and Fast Robust
// Geometric Predicates, 1997: |error| <= (10 + 96 eps) eps x the permanent;
// the coordinate differences here are exact), then exactly in 128-bit
// integers when the rounded value is within the bound.
__device__ int incircle_exact(const int64_t* p, int32_t a, int32_t b, int32_t c, int32_t d);

__device__ __forceinline__ int incircle(const int64_t* p, int32_t a, int32_t b, int32_t c, int32_t d) {
  const double adx = (double)(p[2 * a] - p[2 * d]), ady = (double)(p[2 * a + 1] - p[2 * d + 1]);
  const double bdx = (double)(p[2 * b] - p[2 * d]), bdy = (double)(p[2 * b + 1] - p[2 * d + 1]);
  const double cdx = (double)(p[2 * c] - p[2 * d]), cdy = (double)(p[2 * c + 1] - p[2 * d + 1]);
  const double bdxcdy = bdx * cdy, cdxbdy = cdx * bdy, cdxady = cdx * ady, adxcdy = adx * cdy;
  const double adxbdy = adx * bdy, bdxady = bdx * ady;
  const double alift = adx * adx + ady * ady, blift = bdx * bdx + bdy * bdy, clift = cdx * cdx + cdy * cdy;
  const double det = alift * (bdxcdy - cdxbdy) + blift * (cdxady - adxcdy) + clift * (adxbdy - bdxady);
  const double perm = (fabs(bdxcdy) + fabs(cdxbdy)) * alift + (fabs(cdxady) + fabs(adxcdy)) * blift +
                      (fabs(adxbdy) + fabs(bdxady)) * clift;
  const double eps = 0x1.0p-53;
  const double bound = (10.0 + 96.0 * eps) * eps * perm;
  if (det > bound) return 1;
  if (-det > bound) return -1;
  return incircle_exact(p, a, b, c, d);
}

__device__ int incircle_exact(const int64_t* p, int32_t a, int32_t b, int32_t c, int32_t d) {
  const int64_t adx = p[2 * a] - p[2 * d], ady = p[2 * a + 1] - p[2 * d + 1];
  const int64_t bdx = p[2 * b] - p[2 * d], bdy = p[2 * b + 1] - p[2 * d + 1];
  const int64_t cdx = p[2 * c] - p[2 * d], cdy = p[2 * c + 1] - p[2 * d + 1];
  const __int128 al = (__int128)adx * adx + (__int128)ady * ady;
  const __int128 bl = (__int128)bdx * bdx + (__int128)bdy * bdy;
  const __int128 cl = (__int128)cdx * cdx + (__int128)cdy * cdy;
  const __int128 det = al * ((__int128)bdx * cdy - (__int128)bdy * cdx) -
                       bl * ((__int128)adx * cdy - (__int128)ady * cdx) +
                       cl * ((__int128)adx * bdy - (__int128)ady * bdx);
  return det > 0 ? 1 : (det < 0 ? -1 : 0);
}

__global__ __launch_bounds__(256) void k_gen_points(int64_t g, double jitter, uint64_t seed, double* __restrict__ xy,
                                                    int64_t* __restrict__ lat) {
  const int64_t n = g * g;
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = c / g, i = c - j * g;
    const double u = (double)(splitmix64(seed, 2 * (uint64_t)c) >> 11) * 0x1.0p-53;
    const double w = (double)(splitmix64(seed, 2 * (uint64_t)c + 1) >> 11) * 0x1.0p-53;
    const double jx = jitter * (2.0 * u - 1.0), jy = jitter * (2.0 * w - 1.0);
    const double x = ((double)i + 0.5 + jx) / (double)g;
    const double y = ((double)j + 0.5 + jy) / (double)g;
    double qx = __builtin_rint(x * (double)kLatScale), qy = __builtin_rint(y * (double)kLatScale);
    qx = qx < 0.0 ? 0.0 : (qx > (double)kLatScale ? (double)kLatScale : qx);
    qy = qy < 0.0 ? 0.0 : (qy > (double)kLatScale ? (double)kLatScale : qy);
    const int64_t v = grid_id(i, j, g);
    lat[2 * v] = (int64_t)qx;
    lat[2 * v + 1] = (int64_t)qy;
    xy[2 * v] = qx / (double)kLatScale;
    xy[2 * v + 1] = qy / (double)kLatScale;
  }
}

// Every cell's two triangles. Cell quad a = (i, j), b = (i+1, j), c = (i+1,
// j+1), d = (i, j+1), counter-clockwise. Diagonal ac: triangles (a, b, c),
// (a, c, d); diagonal bd: (a, b, d), (b, c, d). diag[cell] = 0 for ac, 1 for bd.
__global__ __launch_bounds__(256) void k_gen_cells(int64_t g, const int64_t* __restrict__ lat,
                                                   int32_t* __restrict__ origin, uint8_t* __restrict__ diag,
                                                   Counters* cnt) {
  const int64_t nc = (g - 1) * (g - 1);
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nc; k += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = k / (g - 1), i = k - j * (g - 1);
    const int32_t a = (int32_t)grid_id(i, j, g), b = (int32_t)grid_id(i + 1, j, g);
    const int32_t c = (int32_t)grid_id(i + 1, j + 1, g), d = (int32_t)grid_id(i, j + 1, g);
    const int64_t* p = lat;
    const bool ac = orient(p[2 * a], p[2 * a + 1], p[2 * b], p[2 * b + 1], p[2 * c], p[2 * c + 1]) > 0 &&
                    orient(p[2 * a], p[2 * a + 1], p[2 * c], p[2 * c + 1], p[2 * d], p[2 * d + 1]) > 0;
    const bool bd = orient(p[2 * a], p[2 * a + 1], p[2 * b], p[2 * b + 1], p[2 * d], p[2 * d + 1]) > 0 &&
                    orient(p[2 * b], p[2 * b + 1], p[2 * c], p[2 * c + 1], p[2 * d], p[2 * d + 1]) > 0;
    // both valid: the Delaunay one (d outside the circle of a, b, c)
    const bool use_ac = ac && (!bd || incircle(p, a, b, c, d) <= 0);
    if (!ac && !bd) set_error(cnt, POLYLLA_EDEGEN);
    const int64_t t0 = 2 * cell_id(i, j, g), t1 = t0 + 1;
    int32_t* o0 = origin + 3 * t0;
    int32_t* o1 = origin + 3 * t1;
    if (use_ac) {
      o0[0] = a; o0[1] = b; o0[2] = c;
      o1[0] = a; o1[1] = c; o1[2] = d;
    } else {
      o0[0] = a; o0[1] = b; o0[2] = d;
      o1[0] = b; o1[1] = c; o1[2] = d;
    }
    diag[cell_id(i, j, g)] = use_ac ? 0 : 1;
  }
}

// half-edges of a cell's sides (see k_gen_cells): bottom a->b, right b->c,
// top c->d, left d->a, and the diagonal pair
__device__ __forceinline__ int32_t side_he(int64_t t0, bool bd, int side) {
  const int32_t h0 = (int32_t)(3 * t0), h1 = h0 + 3;
  switch (side) {
    case 0: return h0;                   // bottom
    case 1: return bd ? h1 : h0 + 1;     // right
    case 2: return h1 + 1;               // top
    default: return bd ? h0 + 2 : h1 + 2;  // left
  }
}

__global__ __launch_bounds__(256) void k_gen_twins(int64_t g, const uint8_t* __restrict__ diag,
                                                   int32_t* __restrict__ twin) {
  const int64_t n1 = g - 1, nc = n1 * n1;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nc; k += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = k / n1, i = k - j * n1;
    const int64_t cid = cell_id(i, j, g);
    const bool bd = diag[cid] != 0;
    const int64_t t0 = 2 * cid;
    const int32_t h0 = (int32_t)(3 * t0), h1 = h0 + 3;
    // the diagonal
    if (bd) {
      twin[h0 + 1] = h1 + 2;
      twin[h1 + 2] = h0 + 1;
    } else {
      twin[h0 + 2] = h1;
      twin[h1] = h0 + 2;
    }
    // bottom with the top of (i, j-1); right with the left of (i+1, j); the
    // neighbours set the other two sides
    if (j > 0) {
      const int64_t nb = cell_id(i, j - 1, g);
      twin[side_he(t0, bd, 0)] = side_he(2 * nb, diag[nb] != 0, 2);
    } else {
      twin[side_he(t0, bd, 0)] = -1;
    }
    if (i + 1 < n1) {
      const int64_t nb = cell_id(i + 1, j, g);
      twin[side_he(t0, bd, 1)] = side_he(2 * nb, diag[nb] != 0, 3);
    } else {
      twin[side_he(t0, bd, 1)] = -1;
    }
    if (j + 1 < n1) {
      const int64_t nb = cell_id(i, j + 1, g);
      twin[side_he(t0, bd, 2)] = side_he(2 * nb, diag[nb] != 0, 0);
    } else {
      twin[side_he(t0, bd, 2)] = -1;
    }
    if (i > 0) {
      const int64_t nb = cell_id(i - 1, j, g);
      twin[side_he(t0, bd, 3)] = side_he(2 * nb, diag[nb] != 0, 1);
    } else {
      twin[side_he(t0, bd, 3)] = -1;
    }
  }
}

// One side of the grid's boundary ring, traversed with the domain on its
// left: bottom (i, 0) left to right, right (g-1, j) bottom to top, top
// (i, g-1) right to left, left (0, j) top to bottom. Vertex k of side s, and
// the boundary half-edge from vertex k to vertex k+1 (its twin is -1).
__device__ __forceinline__ void ring_pos(int s, int64_t k, int64_t g, int64_t* i, int64_t* j) {
  switch (s) {
    case 0: *i = k; *j = 0; break;
    case 1: *i = g - 1; *j = k; break;
    case 2: *i = g - 1 - k; *j = g - 1; break;
    default: *i = 0; *j = g - 1 - k; break;
  }
}

__device__ __forceinline__ int32_t ring_he(int s, int64_t k, int64_t g, const uint8_t* diag) {
  int64_t i, j;
  switch (s) {
    case 0: i = k; j = 0; break;              // cell (k, 0), bottom side
    case 1: i = g - 2; j = k; break;          // cell (g-2, k), right side
    case 2: i = g - 2 - k; j = g - 2; break;  // cell (g-2-k, g-2), top side
    default: i = 0; j = g - 2 - k; break;     // cell (0, g-2-k), left side
  }
  const int64_t cid = cell_id(i, j, g);
  return side_he(2 * cid, diag[cid] != 0, s);
}

// Triangles filling the dents of the boundary live in a pocket store while
// they are made: segment s (the four sides, then the corner scan) holds up
// to seg_cap triangles, numbered from a virtual base above every final
// triangle; k_gen_pack later moves them behind the grid's triangles.
struct Pockets {
  int32_t* origin;   // [5 seg_cap * 3]
  int32_t* twin;     // [5 seg_cap * 3]
  uint32_t* count;   // [5]
  int64_t seg_cap;
  int32_t vbase;     // first virtual half-edge id
  __device__ __forceinline__ void set_twin(int32_t* twin_grid, int32_t h, int32_t v) const {
    if (h >= vbase) twin[h - vbase] = v;
    else twin_grid[h] = v;
  }
};

// Monotone-chain scan over the chain v[0..n) with boundary half-edges ve[k]
// (v[k] -> v[k+1]), domain on the left: a vertex b making a right turn with
// its stack neighbours a and c lies in a dent, which the triangle (a, c, b)
// fills (its edges c->b and b->a face the chain edges b->c and a->b, its
// edge a->c is the new boundary). S and E receive the hull chain and its
// boundary half-edges; returns its length.
__device__ int64_t fill_chain(int32_t* S, int32_t* E, const int32_t* v, const int32_t* ve, int64_t n,
                              const int64_t* lat, int32_t* twin, const Pockets& P, int seg, Counters* cnt) {
  int64_t m = 0;
  uint32_t used = 0;  // the segment's triangles (one thread owns the segment)
  for (int64_t k = 0; k < n; ++k) {
    const int32_t c = v[k];
    if (k > 0) {
      int32_t ec = ve[k - 1];
      while (m >= 2) {
        const int32_t a = S[m - 2], b = S[m - 1];
        if (orient(lat[2 * a], lat[2 * a + 1], lat[2 * b], lat[2 * b + 1], lat[2 * c], lat[2 * c + 1]) >= 0) break;
        const uint32_t q = used++;
        if ((int64_t)q >= P.seg_cap) {
          set_error(cnt, POLYLLA_EINTERNAL);
          P.count[seg] = used;
          return m;
        }
        const int64_t slot = seg * P.seg_cap + q;
        const int32_t h = P.vbase + (int32_t)(3 * slot);
        P.origin[3 * slot] = a;
        P.origin[3 * slot + 1] = c;
        P.origin[3 * slot + 2] = b;
        P.twin[3 * slot] = -1;
        P.twin[3 * slot + 1] = ec;
        P.set_twin(twin, ec, h + 1);
        P.twin[3 * slot + 2] = E[m - 2];
        P.set_twin(twin, E[m - 2], h + 2);
        ec = h;
        --m;
      }
      E[m - 1] = ec;
    }
    S[m++] = c;
  }
  P.count[seg] = used;
  return m;
}

// k_gen_sides with the side in LDS (g <= kGenSideLds): the points' lattice
// coordinates (< 2^29, int32), the boundary half-edges and the scans' stacks
// (side positions and hull half-edges) live in LDS. The side is cut into
// chunks of kGenChunk edges; one thread per chunk runs the scan on it, then
// one thread runs it again over the chunks' hulls in order (the hull of the
// whole chain is the hull of its chunks' hulls, and the second scan fills the
// dents between them), writing its stack in place over the chunks' stacks it
// has already read. The two points on top of a stack stay in registers.
constexpr int64_t kGenSideLds = 3200;  // 5 int32 per point and 2 per chunk: < 64 KB of LDS
constexpr int32_t kGenChunk = 64;

__device__ __forceinline__ int32_t side_vertex(int s, int64_t k, int64_t g) {
  int64_t i, j;
  ring_pos(s, k, g, &i, &j);
  return (int32_t)grid_id(i, j, g);
}

// one pop of the scan: point b = S[m-1] lies in a dent of the chain a -> b -> c
// (a = S[m-2], c at position pc, ec the half-edge b -> c): triangle (a, c, b)
// fills it (see fill_chain); returns its a -> c half-edge, or -1 when the
// segment is full
__device__ __forceinline__ int32_t side_pop(int s, int64_t g, int32_t pa, int32_t pb, int32_t pc, int32_t ec,
                                            int32_t eab, uint32_t q, int32_t* twin, const Pockets& P,
                                            Counters* cnt) {
  if ((int64_t)q >= P.seg_cap) {
    set_error(cnt, POLYLLA_EINTERNAL);
    return -1;
  }
  const int64_t slot = s * P.seg_cap + q;
  const int32_t h = P.vbase + (int32_t)(3 * slot);
  P.origin[3 * slot] = side_vertex(s, pa, g);
  P.origin[3 * slot + 1] = side_vertex(s, pc, g);
  P.origin[3 * slot + 2] = side_vertex(s, pb, g);
  P.twin[3 * slot] = -1;
  P.twin[3 * slot + 1] = ec;
  P.set_twin(twin, ec, h + 1);
  P.twin[3 * slot + 2] = eab;
  P.set_twin(twin, eab, h + 2);
  return h;
}

__global__ __launch_bounds__(256) void k_gen_sides_lds(int64_t g, const int64_t* __restrict__ lat,
                                                       const uint8_t* __restrict__ diag,
                                                       int32_t* __restrict__ twin, int32_t* __restrict__ wsp,
                                                       int64_t* __restrict__ hull_len, Pockets P, Counters* cnt) {
  extern __shared__ int32_t sm[];
  const int s = blockIdx.x;
  if (s >= 4) return;
  const int32_t nch = (int32_t)((g - 1 + kGenChunk - 1) / kGenChunk);  // chunks of kGenChunk edges
  int32_t* px = sm;
  int32_t* py = px + g;
  int32_t* ve = py + g;
  int32_t* S = ve + g;                          // stacks: side positions, chunk c at c (kGenChunk + 1)
  int32_t* E = S + nch * (kGenChunk + 1);       // and hull half-edges
  int32_t* mc = E + nch * (kGenChunk + 1);      // hull length of each chunk
  __shared__ uint32_t s_used;
  __shared__ int32_t s_m;
  if (threadIdx.x == 0) s_used = 0;
  for (int64_t k = threadIdx.x; k < g; k += blockDim.x) {
    const int32_t v = side_vertex(s, k, g);
    px[k] = (int32_t)lat[2 * v];
    py[k] = (int32_t)lat[2 * v + 1];
    if (k + 1 < g) ve[k] = ring_he(s, k, g, diag);
  }
  __syncthreads();
  // level 1: one thread per chunk (positions c C .. min(c C + C, g - 1))
  for (int32_t c = threadIdx.x; c < nch; c += blockDim.x) {
    int32_t* Sc = S + c * (kGenChunk + 1);
    int32_t* Ec = E + c * (kGenChunk + 1);
    const int32_t k0 = c * kGenChunk, k1 = (int32_t)min<int64_t>(k0 + kGenChunk, g - 1);
    int32_t m = 0;
    int64_t ax = 0, ay = 0, bx = 0, by = 0;  // points Sc[m-2], Sc[m-1]
    bool ok = true;
    for (int32_t k = k0; k <= k1 && ok; ++k) {
      const int64_t cx = px[k], cy = py[k];
      if (k > k0) {
        int32_t ec = ve[k - 1];
        while (m >= 2 && orient(ax, ay, bx, by, cx, cy) < 0) {
          ec = side_pop(s, g, Sc[m - 2], Sc[m - 1], k, ec, Ec[m - 2], atomicAdd(&s_used, 1u), twin, P, cnt);
          if (ec < 0) {
            ok = false;
            break;
          }
          --m;
          bx = ax;
          by = ay;
          if (m >= 2) {
            ax = px[Sc[m - 2]];
            ay = py[Sc[m - 2]];
          }
        }
        Ec[m - 1] = ec;
      }
      Sc[m++] = k;
      ax = bx;
      ay = by;
      bx = cx;
      by = cy;
    }
    mc[c] = m;
  }
  __syncthreads();
  // level 2: the chunks' hulls in order (a chunk's first point is the
  // previous chunk's last), the stack written in place from the start
  if (threadIdx.x == 0) {
    uint32_t used = s_used;
    int32_t m = 0;
    int64_t ax = 0, ay = 0, bx = 0, by = 0;
    bool ok = true;
    for (int32_t c = 0; c < nch && ok; ++c) {
      const int32_t base = c * (kGenChunk + 1), mcc = mc[c];
      for (int32_t kk = c == 0 ? 0 : 1; kk < mcc && ok; ++kk) {
        const int32_t pk = S[base + kk];
        const int64_t cx = px[pk], cy = py[pk];
        if (m > 0) {
          int32_t ec = E[base + kk - 1];
          while (m >= 2 && orient(ax, ay, bx, by, cx, cy) < 0) {
            ec = side_pop(s, g, S[m - 2], S[m - 1], pk, ec, E[m - 2], used++, twin, P, cnt);
            if (ec < 0) {
              ok = false;
              break;
            }
            --m;
            bx = ax;
            by = ay;
            if (m >= 2) {
              ax = px[S[m - 2]];
              ay = py[S[m - 2]];
            }
          }
          E[m - 1] = ec;
        }
        S[m++] = pk;
        ax = bx;
        ay = by;
        bx = cx;
        by = cy;
      }
    }
    P.count[s] = used;
    s_m = m;
    hull_len[s] = m;
  }
  __syncthreads();
  // the hull chain for the corner scan: vertex ids and half-edges
  const int32_t m = s_m;
  int32_t* hs = wsp + (int64_t)s * 4 * g + 2 * g;
  int32_t* he = hs + g;
  for (int32_t k = threadIdx.x; k < m; k += blockDim.x) {
    hs[k] = side_vertex(s, S[k], g);
    if (k + 1 < m) he[k] = E[k];
  }
}

__global__ void k_gen_sides(int64_t g, const int64_t* __restrict__ lat, const uint8_t* __restrict__ diag,
                            int32_t* __restrict__ twin, int32_t* __restrict__ wsp, int64_t* __restrict__ hull_len,
                            Pockets P, Counters* cnt) {
  // one thread per side; its work space: chain vertices, chain half-edges,
  // hull vertices, hull half-edges (g ints each)
  const int s = blockIdx.x;
  if (threadIdx.x != 0 || s >= 4) return;
  int32_t* v = wsp + (int64_t)s * 4 * g;
  int32_t* ve = v + g;
  int32_t* S = ve + g;
  int32_t* E = S + g;
  for (int64_t k = 0; k < g; ++k) {
    int64_t i, j;
    ring_pos(s, k, g, &i, &j);
    v[k] = (int32_t)grid_id(i, j, g);
    if (k + 1 < g) ve[k] = ring_he(s, k, g, diag);
  }
  hull_len[s] = fill_chain(S, E, v, ve, g, lat, twin, P, s, cnt);
}

// The four sides' hulls joined into one ring (a side's last vertex is the
// next side's first) and scanned again once around it, from the lowest (then
// leftmost) ring vertex, which lies on the convex hull, back to it.
__global__ void k_gen_corners(int64_t g, const int64_t* __restrict__ lat, int32_t* __restrict__ twin,
                              int32_t* __restrict__ wsp, const int64_t* __restrict__ hull_len, Pockets P,
                              Counters* cnt) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  int32_t* rv = wsp + 16 * g;      // ring: vertices, half-edges
  int32_t* re = rv + 4 * g;
  int32_t* v = re + 4 * g;         // the chain from the start round to it again
  int32_t* ve = v + 4 * g + 1;
  int32_t* S = ve + 4 * g + 1;
  int32_t* E = S + 4 * g + 1;
  int64_t n = 0;
  for (int s = 0; s < 4; ++s) {
    const int32_t* hs = wsp + (int64_t)s * 4 * g + 2 * g;
    const int32_t* he = hs + g;
    for (int64_t k = 0; k + 1 < hull_len[s]; ++k) {
      rv[n] = hs[k];
      re[n] = he[k];
      ++n;
    }
  }
  if (n < 3) {
    set_error(cnt, POLYLLA_EINTERNAL);
    return;
  }
  int64_t best = 0;
  for (int64_t k = 1; k < n; ++k) {
    const int32_t a = rv[k], b = rv[best];
    if (lat[2 * a + 1] < lat[2 * b + 1] || (lat[2 * a + 1] == lat[2 * b + 1] && lat[2 * a] < lat[2 * b])) best = k;
  }
  for (int64_t k = 0; k <= n; ++k) {
    v[k] = rv[(best + k) % n];
    if (k < n) ve[k] = re[(best + k) % n];
  }
  fill_chain(S, E, v, ve, n + 1, lat, twin, P, 4, cnt);
}

// The pocket triangles behind the grid's (tri_base onwards), segment by
// segment, their virtual half-edge ids replaced everywhere.
__device__ __forceinline__ int32_t pocket_final(int32_t h, const Pockets& P, const uint32_t* pre, int64_t tri_base) {
  if (h < P.vbase) return h;
  const int64_t slot = (h - P.vbase) / 3, r = (h - P.vbase) - 3 * slot;
  const int64_t seg = slot / P.seg_cap, q = slot - seg * P.seg_cap;
  return (int32_t)(3 * (tri_base + pre[seg] + q) + r);
}

__global__ __launch_bounds__(256) void k_gen_pack(Pockets P, int64_t tri_base, int64_t cap_tri,
                                                  int32_t* __restrict__ origin, int32_t* __restrict__ twin,
                                                  int64_t* __restrict__ n_tri, Counters* cnt) {
  uint32_t pre[6];
  pre[0] = 0;
  for (int s = 0; s < 5; ++s) pre[s + 1] = pre[s] + (uint32_t)min<int64_t>(P.count[s], P.seg_cap);
  if (tri_base + pre[5] > cap_tri) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      *n_tri = 0;
      set_error(cnt, POLYLLA_EINTERNAL);
    }
    return;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) *n_tri = tri_base + pre[5];
  for (int s = 0; s < 5; ++s) {
    const uint32_t cs = pre[s + 1] - pre[s];
    for (uint32_t q = blockIdx.x * blockDim.x + threadIdx.x; q < cs; q += gridDim.x * blockDim.x) {
      const int64_t slot = s * P.seg_cap + q;
      const int64_t t = tri_base + pre[s] + q;
      for (int r = 0; r < 3; ++r) {
        origin[3 * t + r] = P.origin[3 * slot + r];
        const int32_t tw = P.twin[3 * slot + r];
        const int32_t f = tw < 0 ? -1 : pocket_final(tw, P, pre, tri_base);
        twin[3 * t + r] = f;
        if (f >= 0 && tw < P.vbase) twin[tw] = (int32_t)(3 * t + r);  // a grid half-edge facing this triangle
      }
    }
  }
}

// Structural check before the flips (which index through twin): twins are an
// involution between half-edges of opposite direction, origins are vertex
// ids, triangles are counter-clockwise. The triangle count is read on the
// device (the launch covers its bound).
__global__ __launch_bounds__(256) void k_gen_check(const int64_t* __restrict__ n_tri, int64_t nv,
                                                   const int32_t* __restrict__ twin,
                                                   const int32_t* __restrict__ origin,
                                                   const int64_t* __restrict__ lat, Counters* cnt) {
  const int64_t nh = 3 * *n_tri;
  for (int64_t h = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; h < nh; h += (int64_t)gridDim.x * blockDim.x) {
    const int32_t hn = he_next((int32_t)h);
    const int32_t a = origin[h], b = origin[hn], c = origin[he_next(hn)];
    if (a < 0 || a >= nv || b < 0 || b >= nv || c < 0 || c >= nv) {
      set_error(cnt, POLYLLA_EINTERNAL);
      continue;
    }
    if (h % 3 == 0 &&
        orient(lat[2 * a], lat[2 * a + 1], lat[2 * b], lat[2 * b + 1], lat[2 * c], lat[2 * c + 1]) <= 0)
      set_error(cnt, POLYLLA_EINTERNAL);
    const int32_t tw = twin[h];
    if (tw == -1) continue;
    if (tw < 0 || tw >= nh || twin[tw] != (int32_t)h || origin[tw] != b) set_error(cnt, POLYLLA_EINTERNAL);
  }
}

// ---- parallel Lawson flips
//
// Round r: every failing edge joins the round's list and claims its two
// triangles and their (up to) four neighbours with a priority whose top bits
// are the round (so claims of earlier rounds never win and the claims need no
// clearing); the listed edges that hold all six claims flip. An edge is
// tested in round r only if one of its triangles was changed by a flip of
// round r - 1, or held an edge that failed and did not flip (their stamp is
// r; round 0 tests every edge), and only from one of its triangles. Each kernel returns at once after an error or
// once a round has found no failing edge, so the host launches rounds in
// batches and reads the counts once per batch.

__device__ __forceinline__ uint64_t flip_priority(int32_t h, uint32_t round) {
  const uint64_t mix = splitmix64(0x5DEECE66Dull + round, (uint64_t)h) >> 44;  // 20 random bits
  return ((uint64_t)round << 52) | (mix << 32) | (uint32_t)h;
}

// the half-edge h (h < twin) fails the in-circle test: the apex of its twin's
// triangle lies inside the circle of h's triangle
__device__ __forceinline__ bool fails_incircle(int32_t h, int32_t ht, const int32_t* origin, const int64_t* lat) {
  const int32_t a = origin[h], b = origin[he_next(h)], c = origin[he_next(he_next(h))];
  const int32_t d = origin[he_next(he_next(ht))];
  return incircle(lat, a, b, c, d) > 0;
}

// the rounds before r all found failing edges and no error is recorded
__device__ __forceinline__ bool round_live(const uint32_t* bad, uint32_t r, const Counters* cnt) {
  return cnt->error == 0 && (r == 0 || bad[r - 1] != 0u);
}

__global__ __launch_bounds__(256) void k_gen_claim(const int64_t* __restrict__ n_tri, const int32_t* __restrict__ twin,
                                                   const int32_t* __restrict__ origin,
                                                   const int64_t* __restrict__ lat,
                                                   const uint16_t* __restrict__ stamp, unsigned long long* claim,
                                                   int32_t* __restrict__ list, uint32_t* bad, uint32_t round,
                                                   const Counters* cnt) {
  if (!round_live(bad, round, cnt)) return;
  const int64_t nh = 3 * *n_tri;
  const int lane = threadIdx.x & 63;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  // wave-uniform loop: the failing edges of a wave join the list with one counter update
  for (int64_t h0 = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63); h0 < nh; h0 += stride) {
    const int64_t hh = h0 + lane;
    bool fail = false;
    int32_t ht = -1;
    // an edge is tested from a stamped triangle, from the smaller one when both are
    if (hh < nh && stamp[hh / 3] == round) {
      ht = twin[hh];
      if (ht >= 0) {
        const int64_t t = hh / 3, u = ht / 3;
        if (stamp[u] != round || u > t) fail = fails_incircle((int32_t)hh, ht, origin, lat);
      }
    }
    const uint64_t m = __ballot(fail);
    if (m == 0ull) continue;
    uint32_t base = 0;
    if (lane == 0) base = atomicAdd(&bad[round], (uint32_t)__popcll(m));
    base = __shfl(base, 0, 64);
    if (!fail) continue;
    const int32_t h = (int32_t)hh;
    list[base + __popcll(m & ((1ull << lane) - 1ull))] = h;
    const unsigned long long pr = flip_priority(h, round);
    const int32_t hs[4] = {he_next(h), he_next(he_next(h)), he_next(ht), he_next(he_next(ht))};
    atomicMax(&claim[h / 3], pr);
    atomicMax(&claim[ht / 3], pr);
    for (int k = 0; k < 4; ++k) {
      const int32_t nb = twin[hs[k]];
      if (nb >= 0) atomicMax(&claim[nb / 3], pr);
    }
  }
}

__global__ __launch_bounds__(256) void k_gen_flip(int32_t* __restrict__ twin, int32_t* __restrict__ origin,
                                                  const unsigned long long* __restrict__ claim,
                                                  const int32_t* __restrict__ list, uint16_t* __restrict__ stamp,
                                                  const uint32_t* bad, uint32_t round, const Counters* cnt) {
  if (cnt->error != 0) return;
  const uint32_t n = bad[round];
  const uint16_t next = (uint16_t)(round + 1);
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const int32_t h = list[i];
    const unsigned long long pr = flip_priority(h, round);
    const int32_t ht = twin[h];
    const int32_t hn = he_next(h), hp = he_next(hn), tn = he_next(ht), tp = he_next(tn);
    const int32_t nbs[4] = {twin[hn], twin[hp], twin[tn], twin[tp]};
    bool mine = claim[h / 3] == pr && claim[ht / 3] == pr;
    for (int k = 0; k < 4; ++k)
      if (nbs[k] >= 0) mine = mine && claim[nbs[k] / 3] == pr;
    if (!mine) {
      stamp[h / 3] = next;  // still failing: tested again next round
      continue;
    }
    // h = a->b in (a, b, c), ht = b->a in (b, a, d): new (c, a, d) in h's
    // triangle and (d, b, c) in ht's
    const int32_t a = origin[h], b = origin[hn], c = origin[hp], d = origin[tp];
    const int32_t t1 = 3 * (h / 3), t2 = 3 * (ht / 3);
    const int32_t tb_c = nbs[0], tc_a = nbs[1], ta_d = nbs[2], td_b = nbs[3];
    origin[t1] = c;
    origin[t1 + 1] = a;
    origin[t1 + 2] = d;
    origin[t2] = d;
    origin[t2 + 1] = b;
    origin[t2 + 2] = c;
    twin[t1] = tc_a;
    twin[t1 + 1] = ta_d;
    twin[t1 + 2] = t2 + 2;
    twin[t2] = td_b;
    twin[t2 + 1] = tb_c;
    twin[t2 + 2] = t1 + 2;
    if (tc_a >= 0) twin[tc_a] = t1;
    if (ta_d >= 0) twin[ta_d] = t1 + 1;
    if (td_b >= 0) twin[td_b] = t2;
    if (tb_c >= 0) twin[tb_c] = t2 + 1;
    stamp[h / 3] = next;
    stamp[ht / 3] = next;
  }
}

}  // namespace polylla

namespace polylla {


// Host driver (called by polylla_gen_grid). ws: device work space of
// gen_ws_bytes(g) bytes. Returns a polylla code; *n_tri receives the number
// of triangles.
constexpr int kGenMaxRounds = 4095;  // flip rounds before EDEGEN (the round is 12 bits of a claim)
constexpr int kGenFirstRounds = 12;  // rounds launched before the first read of the counts
constexpr int kGenMoreRounds = 4;    // then between reads

size_t gen_ws_bytes(int64_t g) {
  const int64_t V = g * g, Tmax = 2 * V;
  const int64_t seg = 4 * g + 8;
  size_t b = 0;
  auto add = [&](size_t n) { b += (n + 255) & ~(size_t)255; };
  add(sizeof(int64_t) * 2 * V);            // lattice coordinates
  add((size_t)V);                          // cell diagonals
  add(sizeof(unsigned long long) * Tmax);  // flip claims
  add(sizeof(int32_t) * 44 * g + 64);      // side and corner scans
  add(sizeof(int32_t) * 2 * 3 * 5 * seg);  // pocket store
  add(sizeof(uint32_t) * 16);              // pocket counts
  add(sizeof(int64_t) * 8);                // hull lengths, triangle count
  add(sizeof(uint32_t) * kGenMaxRounds);   // failing edges per flip round
  add(sizeof(uint16_t) * Tmax);            // round stamps of the triangles
  add(sizeof(int32_t) * (3 * Tmax / 2 + 64));  // the round's failing edges
  return b;
}

int gen_grid_run(int64_t g, double jitter, uint64_t seed, double* xy, int32_t* twin, int32_t* origin,
                 int64_t cap_tri, void* ws, Counters* cnt, hipStream_t s, int64_t* n_tri, int* rounds) {
  const int64_t V = g * g, Tmax = 2 * V;
  const int64_t seg = 4 * g + 8;
  uint8_t* p = static_cast<uint8_t*>(ws);
  auto take = [&](size_t n) {
    uint8_t* r = p;
    p += (n + 255) & ~(size_t)255;
    return r;
  };
  int64_t* lat = reinterpret_cast<int64_t*>(take(sizeof(int64_t) * 2 * V));
  uint8_t* diag = take((size_t)V);
  unsigned long long* claim = reinterpret_cast<unsigned long long*>(take(sizeof(unsigned long long) * Tmax));
  int32_t* wsp = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * 44 * g + 64));
  int32_t* porg = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * 2 * 3 * 5 * seg));
  uint32_t* u32 = reinterpret_cast<uint32_t*>(take(sizeof(uint32_t) * 16));
  int64_t* i64 = reinterpret_cast<int64_t*>(take(sizeof(int64_t) * 8));
  uint32_t* bad = reinterpret_cast<uint32_t*>(take(sizeof(uint32_t) * kGenMaxRounds));
  uint16_t* stamp = reinterpret_cast<uint16_t*>(take(sizeof(uint16_t) * Tmax));
  int32_t* list = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * (3 * Tmax / 2 + 64)));
  const int64_t tri_base = 2 * (g - 1) * (g - 1);
  Pockets P{porg, porg + 3 * 5 * seg, u32, seg, (int32_t)(3 * (tri_base + 8 * g + 64))};
  const int64_t* d_tri = i64 + 4;
  const int64_t cap = std::min(cap_tri, Tmax);
  const int grid = (int)std::min<int64_t>((V + 255) / 256, 1 << 16);
  const int hgrid = (int)std::min<int64_t>((3 * Tmax + 255) / 256, 1 << 16);
  if (hipMemsetAsync(u32, 0, sizeof(uint32_t) * 16, s) != hipSuccess ||
      hipMemsetAsync(bad, 0, sizeof(uint32_t) * kGenMaxRounds, s) != hipSuccess ||
      hipMemsetAsync(claim, 0, sizeof(unsigned long long) * Tmax, s) != hipSuccess ||
      hipMemsetAsync(stamp, 0, sizeof(uint16_t) * Tmax, s) != hipSuccess)
    return POLYLLA_EHIP;
  hipLaunchKernelGGL(k_gen_points, dim3(grid), dim3(256), 0, s, g, jitter, seed, xy, lat);
  hipLaunchKernelGGL(k_gen_cells, dim3(grid), dim3(256), 0, s, g, (const int64_t*)lat, origin, diag, cnt);
  hipLaunchKernelGGL(k_gen_twins, dim3(grid), dim3(256), 0, s, g, (const uint8_t*)diag, twin);
  const int64_t nch = (g - 1 + kGenChunk - 1) / kGenChunk;
  const size_t side_lds = sizeof(int32_t) * (size_t)(3 * g + 2 * nch * (kGenChunk + 1) + nch);
  if (g <= kGenSideLds)
    hipLaunchKernelGGL(k_gen_sides_lds, dim3(4), dim3(256), side_lds, s, g, (const int64_t*)lat,
                       (const uint8_t*)diag, twin, wsp, i64, P, cnt);
  else
    hipLaunchKernelGGL(k_gen_sides, dim3(4), dim3(64), 0, s, g, (const int64_t*)lat, (const uint8_t*)diag, twin,
                       wsp, i64, P, cnt);
  hipLaunchKernelGGL(k_gen_corners, dim3(1), dim3(64), 0, s, g, (const int64_t*)lat, twin, wsp,
                     (const int64_t*)i64, P, cnt);
  hipLaunchKernelGGL(k_gen_pack, dim3(64), dim3(256), 0, s, P, tri_base, cap, origin, twin, i64 + 4, cnt);
  hipLaunchKernelGGL(k_gen_check, dim3(hgrid), dim3(256), 0, s, d_tri, V, (const int32_t*)twin,
                     (const int32_t*)origin, (const int64_t*)lat, cnt);
  if (hipGetLastError() != hipSuccess) return POLYLLA_EHIP;
  // Lawson flips until every edge passes the in-circle test, rounds launched
  // in batches (a converged or failed round makes the rest return at once)
  struct {
    int64_t nt;
    uint32_t last;
    int32_t err;
  } h{};
  int r = 0;
  for (int batch = kGenFirstRounds;; batch = kGenMoreRounds) {
    for (int k = 0; k < batch; ++k, ++r) {
      hipLaunchKernelGGL(k_gen_claim, dim3(hgrid), dim3(256), 0, s, d_tri, (const int32_t*)twin,
                         (const int32_t*)origin, (const int64_t*)lat, (const uint16_t*)stamp, claim, list, bad,
                         (uint32_t)r, (const Counters*)cnt);
      hipLaunchKernelGGL(k_gen_flip, dim3(hgrid), dim3(256), 0, s, twin, origin, (const unsigned long long*)claim,
                         (const int32_t*)list, stamp, (const uint32_t*)bad, (uint32_t)r, (const Counters*)cnt);
    }
    if (hipMemcpyAsync(&h.nt, d_tri, sizeof(int64_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(&h.last, bad + r - 1, sizeof(uint32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(&h.err, &cnt->error, sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return POLYLLA_EHIP;
    if (h.err) return h.err;
    if (h.last == 0) break;
    if (r + kGenMoreRounds > kGenMaxRounds) return POLYLLA_EDEGEN;
  }
  if (h.nt <= 0 || h.nt > cap) return POLYLLA_EINTERNAL;
  // rounds that found failing edges (the first round without one ends the flips)
  std::vector<uint32_t> counts((size_t)r);
  if (hipMemcpy(counts.data(), bad, sizeof(uint32_t) * (size_t)r, hipMemcpyDeviceToHost) != hipSuccess)
    return POLYLLA_EHIP;
  int done = 0;
  while (done < r && counts[(size_t)done] != 0u) ++done;
  *n_tri = h.nt;
  if (rounds) *rounds = done;
  return hipGetLastError() == hipSuccess ? POLYLLA_OK : POLYLLA_EHIP;
}

}  // namespace polylla
