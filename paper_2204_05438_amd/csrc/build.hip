// Traversal phase (Algorithm 3, PolyConstruction) and Reparation phase
// (Algorithm 4) as gfx950 kernels.
//
// k_walk    : one lane per polygon. Walks the frontier half-edges of the
//             region from its start half-edge with the region on the left
//             (turning about each vertex through internal edges), staging the
//             vertex ids in LDS (interleaved [slot][lane], conflict free). A
//             cycle with no repeated vertex and at most kWalkCap vertices is
//             complete: it is rotated to start at its smallest vertex and
//             copied to a staging buffer at a wave-allocated slot. Every other
//             cycle (a barrier-edge tip, another repeated vertex, or a long
//             cycle) is queued for k_general.
// k_general : one lane per queued polygon, data in a global arena. Records
//             the whole cycle, marks barrier edges (frontier edges met twice),
//             finds the tips (next frontier half-edge == twin), and, when
//             repairing, opens the middle internal edge at every tip that is
//             still a tip once the smaller tips are handled; then walks the
//             pieces, each once, and sorts them by their canonical first two
//             vertices.
// k_scan_polys : single-pass decoupled look-back scan of (pieces, vertices)
//             per polygon in seed order; writes counts and the final offset.
// k_emit    : copies every polygon from staging to its place in the CSR output
//             and writes its offsets and start half-edges.
#include "common.h"
#include "scan.h"

namespace polylla {

constexpr int kWalkCap = 32;

// Start half-edge of the region of seed triangle t: its first frontier
// half-edge in local order, else the first frontier half-edge met turning
// about its vertex 0. Returns -1 on an invalid mesh.
__device__ __forceinline__ int32_t seed_start(int32_t t, int32_t nhe, const int32_t* __restrict__ twin,
                                              const uint8_t* __restrict__ he, Counters* cnt) {
  const int32_t h0 = 3 * t;
  if (t < 0 || h0 >= nhe) {
    set_error(cnt, POLYLLA_ETOPO);
    return -1;
  }
  uint8_t l0 = he[h0], l1 = he[h0 + 1], l2 = he[h0 + 2];
  if (l0 & kFrontier) return h0;
  if (l1 & kFrontier) return h0 + 1;
  if (l2 & kFrontier) return h0 + 2;
  int32_t c = h0;
  for (int32_t steps = 0; steps <= nhe; ++steps) {
    if (he[c] & kFrontier) return c;
    int32_t tw = twin[c];
    if ((uint32_t)tw >= (uint32_t)nhe) break;
    c = he_next(tw);
  }
  set_error(cnt, POLYLLA_EDEGEN);
  return -1;
}

// Next frontier half-edge of the cycle after frontier half-edge h.
__device__ __forceinline__ int32_t walk_next(int32_t h, int32_t nhe, const int32_t* __restrict__ twin,
                                             const uint8_t* __restrict__ he, Counters* cnt) {
  int32_t c = he_next(h);
  for (int32_t steps = 0; steps <= nhe; ++steps) {
    if (he[c] & kFrontier) return c;
    int32_t tw = twin[c];
    if ((uint32_t)tw >= (uint32_t)nhe) {
      set_error(cnt, POLYLLA_ETOPO);
      return -1;
    }
    c = he_next(tw);
  }
  set_error(cnt, POLYLLA_EDEGEN);
  return -1;
}

template <bool FROM_SEEDS>
__global__ __launch_bounds__(256) void k_walk(const int32_t* __restrict__ list, int32_t nhe,
                                              const int32_t* __restrict__ twin,
                                              const int32_t* __restrict__ origin,
                                              const uint8_t* __restrict__ he, int32_t* __restrict__ stage,
                                              int64_t stage_cap, PolyState ps, int32_t* __restrict__ deferred,
                                              Counters* cnt) {
  __shared__ int32_t buf[kWalkCap][256];
  const int lane = threadIdx.x & 63;
  const uint32_t R = cnt->n_seeds;
  for (int64_t base = (int64_t)blockIdx.x * 256; base < (int64_t)R; base += (int64_t)gridDim.x * 256) {
    const int64_t i = base + threadIdx.x;
    // 0 = complete here, 1 = queued for the general path, 2 = invalid input
    int state = 1;
    int32_t L = 0, minpos = 0, minhe = -1;
    if (i < (int64_t)R) {
      int32_t s = FROM_SEEDS ? seed_start(list[i], nhe, twin, he, cnt) : list[i];
      if ((uint32_t)s >= (uint32_t)nhe) {
        if (!FROM_SEEDS) set_error(cnt, POLYLLA_ETOPO);
        state = 2;
      } else {
        state = 0;
        int32_t minv = 0x7FFFFFFF;
        int32_t h = s;
        int32_t steps = 0;
        do {
          const int32_t v = origin[h];
          if (L == kWalkCap) {
            state = 1;
            break;
          }
          bool rep = false;
          for (int j = 0; j < L; ++j) rep |= (buf[j][threadIdx.x] == v);
          if (rep) {
            state = 1;
            break;
          }
          buf[L][threadIdx.x] = v;
          if (v < minv) {
            minv = v;
            minhe = h;
            minpos = L;
          }
          ++L;
          const int32_t twh = twin[h];
          int32_t c = he_next(h);
          while (!(he[c] & kFrontier)) {
            int32_t tw = twin[c];
            if ((uint32_t)tw >= (uint32_t)nhe || ++steps > nhe) {
              set_error(cnt, (uint32_t)tw >= (uint32_t)nhe ? POLYLLA_ETOPO : POLYLLA_EDEGEN);
              state = 2;
              break;
            }
            c = he_next(tw);
          }
          if (state == 2) break;
          if (c == twh) {  // barrier-edge tip at the end of h
            state = 1;
            break;
          }
          h = c;
        } while (h != s);
      }
    }
    // staging slots for complete polygons, one atomic per wave
    uint32_t need = (i < (int64_t)R && state == 0) ? (uint32_t)L : 0u;
    uint32_t incl = need;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      uint32_t t = __shfl_up(incl, o, 64);
      if (lane >= o) incl += t;
    }
    uint32_t wbase = 0;
    if (lane == 63 && incl) wbase = atomicAdd(&cnt->stage_top, incl);
    wbase = __shfl(wbase, 63, 64);
    if (i < (int64_t)R) {
      if (state == 0) {
        const int64_t off = (int64_t)wbase + incl - need;
        if (off + L > stage_cap) {
          set_error(cnt, POLYLLA_ENOMEM);
          ps.plen[i] = 0;
          ps.ppieces[i] = 0;
          ps.prec[i] = -1;
          ps.pstage[i] = 0;
        } else {
          int p = minpos;
          for (int k = 0; k < L; ++k) {
            stage[off + k] = buf[p][threadIdx.x];
            p = (p + 1 == L) ? 0 : p + 1;
          }
          ps.plen[i] = L;
          ps.ppieces[i] = 1;
          ps.pstart[i] = minhe;
          ps.prec[i] = -1;
          ps.pstage[i] = (int32_t)off;
        }
      } else if (state == 1) {
        uint32_t q = atomicAdd(&cnt->n_deferred, 1u);
        deferred[q] = (int32_t)i;
      } else {
        ps.plen[i] = 0;
        ps.ppieces[i] = 0;
        ps.prec[i] = -1;
        ps.pstage[i] = 0;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// general path

__device__ void heap_sort(int32_t* a, int32_t n) {
  auto sift = [&](int32_t root, int32_t end) {
    while (2 * root + 1 < end) {
      int32_t child = 2 * root + 1;
      if (child + 1 < end && a[child] < a[child + 1]) ++child;
      if (a[root] < a[child]) {
        int32_t tmp = a[root];
        a[root] = a[child];
        a[child] = tmp;
        root = child;
      } else {
        return;
      }
    }
  };
  for (int32_t k = n / 2 - 1; k >= 0; --k) sift(k, n);
  for (int32_t end = n - 1; end > 0; --end) {
    int32_t tmp = a[0];
    a[0] = a[end];
    a[end] = tmp;
    sift(0, end);
  }
}

// index of x in sorted a[0..n), or -1
__device__ __forceinline__ int32_t bsearch_idx(const int32_t* a, int32_t n, int32_t x) {
  int32_t lo = 0, hi = n;
  while (lo < hi) {
    int32_t mid = (lo + hi) >> 1;
    if (a[mid] < x) lo = mid + 1;
    else hi = mid;
  }
  return (lo < n && a[lo] == x) ? lo : -1;
}

// Compare the vertex sequences of length len starting at frontier half-edges
// p and q of the same cycle: -1 if p's is smaller, 0 equal, 1 greater.
__device__ int compare_rotations(int32_t p, int32_t q, int32_t len, int32_t nhe, const int32_t* __restrict__ twin,
                                 const int32_t* __restrict__ origin, const uint8_t* __restrict__ he, Counters* cnt) {
  for (int32_t k = 0; k < len; ++k) {
    int32_t a = origin[p], b = origin[q];
    if (a != b) return a < b ? -1 : 1;
    p = walk_next(p, nhe, twin, he, cnt);
    q = walk_next(q, nhe, twin, he, cnt);
    if (p < 0 || q < 0) return 0;
  }
  return 0;
}

template <bool REPAIR>
__global__ __launch_bounds__(64) void k_general(const int32_t* __restrict__ list, bool from_seeds, int32_t nhe,
                                                int64_t nv, const int32_t* __restrict__ twin,
                                                const int32_t* __restrict__ origin, uint8_t* __restrict__ he,
                                                uint8_t* __restrict__ vtx, int32_t* __restrict__ stage,
                                                int64_t stage_cap, int32_t* __restrict__ arena, int64_t arena_cap,
                                                PolyState ps, const int32_t* __restrict__ deferred,
                                                Counters* cnt) {
  const uint32_t nd = cnt->n_deferred;
  for (uint32_t j = blockIdx.x * 64 + threadIdx.x; j < nd; j += gridDim.x * 64) {
    const int32_t i = deferred[j];
    ps.plen[i] = 0;
    ps.ppieces[i] = 0;
    ps.prec[i] = -1;
    ps.pstage[i] = 0;
    const int32_t s = from_seeds ? seed_start(list[i], nhe, twin, he, cnt) : list[i];
    if ((uint32_t)s >= (uint32_t)nhe) continue;
    // cycle length
    int32_t L = 0;
    {
      int32_t h = s;
      do {
        ++L;
        h = walk_next(h, nhe, twin, he, cnt);
      } while (h >= 0 && h != s && L <= nhe);
      if (h != s) {
        set_error(cnt, POLYLLA_EDEGEN);
        continue;
      }
    }
    const uint32_t need = 2u * (uint32_t)L;
    const uint32_t a0 = atomicAdd(&cnt->arena_top, need);
    if ((int64_t)a0 + need > arena_cap) {
      set_error(cnt, POLYLLA_ENOMEM);
      continue;
    }
    int32_t* cyc = arena + a0;
    int32_t* aux = cyc + L;
    {
      int32_t h = s;
      for (int32_t k = 0; k < L; ++k) {
        cyc[k] = h;
        h = walk_next(h, nhe, twin, he, cnt);
      }
    }
    // barrier edges: edge keys that occur twice on the cycle
    for (int32_t k = 0; k < L; ++k) {
      int32_t h = cyc[k], tw = twin[h];
      aux[k] = (uint32_t)tw >= (uint32_t)nhe ? -1 : (h < tw ? h : tw);
    }
    heap_sort(aux, L);
    for (int32_t k = 1; k < L; ++k) {
      int32_t e = aux[k];
      if (e >= 0 && e == aux[k - 1]) {
        const int32_t te = twin[e];
        he[e] |= kBarrier;
        if ((uint32_t)te < (uint32_t)nhe) he[te] |= kBarrier;
      }
    }
    // tips: the next frontier half-edge is the twin of the current one
    int32_t ntip = 0;
    for (int32_t k = 0; k < L; ++k) {
      int32_t h = cyc[k], hn = cyc[k + 1 == L ? 0 : k + 1];
      if (twin[h] == hn) {
        int32_t v = origin[hn];
        if ((uint64_t)(uint32_t)v < (uint64_t)nv) vtx[v] |= kTip;
        aux[2 * ntip] = v;
        aux[2 * ntip + 1] = hn;
        ++ntip;
      }
    }
    if (ntip) atomicAdd(&cnt->n_tips, (uint32_t)ntip);
    int32_t nsplit = 0;
    if (REPAIR && ntip) {
      // middle internal edge at every tip: c_{floor(d/2)} clockwise from c0
      for (int32_t q = 0; q < ntip; ++q) {
        const int32_t c0 = aux[2 * q + 1];
        int32_t d = 0, c = c0;
        do {
          const int32_t tw = twin[c];
          if ((uint32_t)tw >= (uint32_t)nhe) {
            d = -1;
            break;
          }
          c = he_next(tw);
          ++d;
        } while (c != c0 && d <= nhe);
        if (d < 0 || c != c0) {
          set_error(cnt, POLYLLA_ETOPO);
          d = 0;
        }
        int32_t e = c0;
        for (int32_t k = 0; k < d / 2; ++k) e = he_next(twin[e]);
        aux[2 * q + 1] = e;
      }
      // tips in increasing vertex id (insertion sort of pairs)
      for (int32_t q = 1; q < ntip; ++q) {
        int32_t v = aux[2 * q], e = aux[2 * q + 1], p = q;
        while (p > 0 && aux[2 * (p - 1)] > v) {
          aux[2 * p] = aux[2 * (p - 1)];
          aux[2 * p + 1] = aux[2 * (p - 1) + 1];
          --p;
        }
        aux[2 * p] = v;
        aux[2 * p + 1] = e;
      }
      // a tip on an edge opened for a smaller live tip is no longer a tip
      for (int32_t q = 0; q < ntip; ++q) {
        const int32_t v = aux[2 * q];
        bool dead = false;
        for (int32_t p = 0; p < q && !dead; ++p) {
          if (aux[2 * p] < 0) continue;  // dead tips are stored as -1 - v
          dead = origin[he_next(aux[2 * p + 1])] == v;
        }
        if (dead) aux[2 * q] = -1 - v;
      }
      for (int32_t q = 0; q < ntip; ++q) {
        if (aux[2 * q] < 0) continue;
        int32_t e = aux[2 * q + 1];
        const int32_t te = twin[e];
        if ((uint32_t)te >= (uint32_t)nhe) {  // only reachable on an invalid mesh
          set_error(cnt, POLYLLA_ETOPO);
          aux[2 * q] = -1 - aux[2 * q];
          continue;
        }
        he[e] |= kFrontier | kRepaired;
        he[te] |= kFrontier | kRepaired;
        ++nsplit;
      }
      if (nsplit) atomicAdd(&cnt->n_splits, (uint32_t)nsplit);
    }
    if (nsplit == 0) {
      // one piece: the cycle itself, rotated to its smallest vertex sequence
      int32_t best = 0, minv = origin[cyc[0]];
      for (int32_t k = 1; k < L; ++k) {
        int32_t v = origin[cyc[k]];
        if (v < minv) {
          minv = v;
          best = k;
        }
      }
      for (int32_t k = best + 1; k < L; ++k) {
        if (origin[cyc[k]] != minv) continue;
        for (int32_t m = 1; m < L; ++m) {
          int32_t a = origin[cyc[(k + m) % L]], b = origin[cyc[(best + m) % L]];
          if (a != b) {
            if (a < b) best = k;
            break;
          }
        }
      }
      const uint32_t off = atomicAdd(&cnt->stage_top, (uint32_t)L);
      if ((int64_t)off + L > stage_cap) {
        set_error(cnt, POLYLLA_ENOMEM);
        continue;
      }
      for (int32_t k = 0; k < L; ++k) stage[off + k] = origin[cyc[(best + k) % L]];
      ps.plen[i] = L;
      ps.ppieces[i] = 1;
      ps.pstart[i] = cyc[best];
      ps.pstage[i] = (int32_t)off;
      continue;
    }
    // pieces: walk from the opened half-edges, each piece once
    const int32_t nc = 2 * nsplit;
    int32_t* cand = cyc;  // the recorded cycle is no longer needed
    {
      int32_t w = 0;
      for (int32_t q = 0; q < ntip; ++q) {
        if (aux[2 * q] < 0) continue;
        int32_t e = aux[2 * q + 1];
        cand[w++] = e;
        cand[w++] = twin[e];
      }
      heap_sort(cand, nc);
    }
    const int32_t npieces = nsplit + 1;
    const uint32_t rneed = (uint32_t)(4 * npieces + nc);
    const uint32_t r0 = atomicAdd(&cnt->arena_top, rneed);
    if ((int64_t)r0 + rneed > arena_cap) {
      set_error(cnt, POLYLLA_ENOMEM);
      continue;
    }
    int32_t* rec = arena + r0;
    int32_t* seen = rec + 4 * npieces;
    for (int32_t k = 0; k < nc; ++k) seen[k] = 0;
    int32_t np = 0, total = 0;
    bool bad = false;
    for (int32_t k = 0; k < nc && !bad; ++k) {
      if (seen[k]) continue;
      const int32_t x = cand[k];
      int32_t h = x, len = 0, minv = 0x7FFFFFFF, minh = -1, mincount = 0;
      do {
        int32_t v = origin[h];
        if (v < minv) {
          minv = v;
          minh = h;
          mincount = 1;
        } else if (v == minv) {
          ++mincount;
        }
        if (he[h] & kRepaired) {
          int32_t idx = bsearch_idx(cand, nc, h);
          if (idx >= 0) seen[idx] = 1;
        }
        ++len;
        h = walk_next(h, nhe, twin, he, cnt);
      } while (h >= 0 && h != x && len <= nhe);
      if (h != x || np >= npieces) {
        set_error(cnt, POLYLLA_EDEGEN);
        bad = true;
        break;
      }
      if (mincount > 1) {
        // pinched piece: lexicographically smallest rotation among the
        // occurrences of its smallest vertex
        int32_t best = minh, q = walk_next(minh, nhe, twin, he, cnt);
        for (int32_t m = 1; m < len && q >= 0; ++m) {
          if (origin[q] == minv && compare_rotations(q, best, len, nhe, twin, origin, he, cnt) < 0) best = q;
          q = walk_next(q, nhe, twin, he, cnt);
        }
        minh = best;
      }
      int32_t nxt = walk_next(minh, nhe, twin, he, cnt);
      rec[4 * np] = minv;
      rec[4 * np + 1] = nxt >= 0 ? origin[nxt] : 0;
      rec[4 * np + 2] = minh;
      rec[4 * np + 3] = len;
      ++np;
      total += len;
    }
    if (bad || np != npieces) {
      if (!bad) set_error(cnt, POLYLLA_EDEGEN);
      continue;
    }
    // pieces by (first, second) vertex
    for (int32_t q = 1; q < np; ++q) {
      int32_t r[4] = {rec[4 * q], rec[4 * q + 1], rec[4 * q + 2], rec[4 * q + 3]};
      int32_t p = q;
      while (p > 0 && (rec[4 * (p - 1)] > r[0] || (rec[4 * (p - 1)] == r[0] && rec[4 * (p - 1) + 1] > r[1]))) {
        for (int m = 0; m < 4; ++m) rec[4 * p + m] = rec[4 * (p - 1) + m];
        --p;
      }
      for (int m = 0; m < 4; ++m) rec[4 * p + m] = r[m];
    }
    const uint32_t off = atomicAdd(&cnt->stage_top, (uint32_t)total);
    if ((int64_t)off + total > stage_cap) {
      set_error(cnt, POLYLLA_ENOMEM);
      continue;
    }
    int32_t w = (int32_t)off;
    for (int32_t q = 0; q < np; ++q) {
      int32_t h = rec[4 * q + 2];
      for (int32_t k = 0; k < rec[4 * q + 3] && h >= 0; ++k) {
        stage[w++] = origin[h];
        h = walk_next(h, nhe, twin, he, cnt);
      }
    }
    ps.plen[i] = total;
    ps.ppieces[i] = np;
    ps.prec[i] = (int32_t)r0;
    ps.pstage[i] = (int32_t)off;
  }
}

// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_scan_polys(PolyState ps, int32_t* __restrict__ poly_off,
                                                    int32_t* __restrict__ vert_off, uint64_t* status,
                                                    int32_t* __restrict__ offsets, int64_t* __restrict__ counts,
                                                    int64_t cap_polys, int64_t cap_verts, Counters* cnt) {
  constexpr int ITEMS = 4;
  const uint32_t R = cnt->n_seeds;
  const uint32_t ntiles = (R + 256 * ITEMS - 1) / (256 * ITEMS);
  const uint32_t tile = take_tile(&cnt->tile_ticket[1]);
  if (ntiles == 0) {
    if (tile == 0 && threadIdx.x == 0) {
      counts[0] = 0;
      counts[1] = 0;
      if (cap_polys >= 0) offsets[0] = 0;
    }
    return;
  }
  if (tile >= ntiles) return;
  const int64_t i0 = ((int64_t)tile * 256 + threadIdx.x) * ITEMS;
  uint32_t a = 0, b = 0;
  int32_t np[ITEMS], nl[ITEMS];
#pragma unroll
  for (int j = 0; j < ITEMS; ++j) {
    const int64_t i = i0 + j;
    np[j] = i < R ? ps.ppieces[i] : 0;
    nl[j] = i < R ? ps.plen[i] : 0;
    a += (uint32_t)np[j];
    b += (uint32_t)nl[j];
  }
  uint2 total;
  uint2 pre = block_exclusive_scan<256>(a, b, &total);
  uint2 ex = tile_lookback(status, tile, total, cnt);
  uint32_t ra = ex.x + pre.x, rb = ex.y + pre.y;
#pragma unroll
  for (int j = 0; j < ITEMS; ++j) {
    const int64_t i = i0 + j;
    if (i < R) {
      poly_off[i] = (int32_t)ra;
      vert_off[i] = (int32_t)rb;
    }
    ra += (uint32_t)np[j];
    rb += (uint32_t)nl[j];
  }
  if (tile == ntiles - 1 && threadIdx.x == 0) {
    const int64_t F = (int64_t)ex.x + total.x, S = (int64_t)ex.y + total.y;
    counts[0] = F;
    counts[1] = S;
    if (F <= cap_polys) offsets[F] = (int32_t)S;
    if (F > cap_polys || S > cap_verts) set_error(cnt, POLYLLA_ECAPACITY);
  }
}

__global__ __launch_bounds__(256) void k_emit(PolyState ps, const int32_t* __restrict__ poly_off,
                                              const int32_t* __restrict__ vert_off,
                                              const int32_t* __restrict__ stage, const int32_t* __restrict__ arena,
                                              int32_t* __restrict__ offsets, int32_t* __restrict__ verts,
                                              int32_t* __restrict__ start, int64_t cap_polys, int64_t cap_verts,
                                              Counters* cnt) {
  const uint32_t R = cnt->n_seeds;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (int64_t)R;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t p0 = poly_off[i], v0 = vert_off[i], np = ps.ppieces[i], len = ps.plen[i];
    if (np == 0) continue;
    if ((int64_t)p0 + np > cap_polys || (int64_t)v0 + len > cap_verts) {
      set_error(cnt, POLYLLA_ECAPACITY);
      continue;
    }
    const int32_t* src = stage + ps.pstage[i];
    for (int32_t k = 0; k < len; ++k) verts[v0 + k] = src[k];
    const int32_t r = ps.prec[i];
    if (r < 0) {
      offsets[p0] = v0;
      if (start) start[p0] = ps.pstart[i];
    } else {
      const int32_t* rec = arena + r;
      int32_t acc = 0;
      for (int32_t q = 0; q < np; ++q) {
        offsets[p0 + q] = v0 + acc;
        if (start) start[p0 + q] = rec[4 * q + 2];
        acc += rec[4 * q + 3];
      }
    }
  }
}

template __global__ void k_walk<true>(const int32_t*, int32_t, const int32_t*, const int32_t*, const uint8_t*,
                                      int32_t*, int64_t, PolyState, int32_t*, Counters*);
template __global__ void k_walk<false>(const int32_t*, int32_t, const int32_t*, const int32_t*, const uint8_t*,
                                       int32_t*, int64_t, PolyState, int32_t*, Counters*);
template __global__ void k_general<true>(const int32_t*, bool, int32_t, int64_t, const int32_t*, const int32_t*,
                                         uint8_t*, uint8_t*, int32_t*, int64_t, int32_t*, int64_t, PolyState,
                                         const int32_t*, Counters*);
template __global__ void k_general<false>(const int32_t*, bool, int32_t, int64_t, const int32_t*, const int32_t*,
                                          uint8_t*, uint8_t*, int32_t*, int64_t, int32_t*, int64_t, PolyState,
                                          const int32_t*, Counters*);

}  // namespace polylla
