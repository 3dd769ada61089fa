/*
 * oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, sequential CPU reference of the terminal-edge-region polygonal mesh
 * method of Salinas, Ojeda, Hitschfeld and Ortiz-Bernardin, "GPU parallel
 * algorithm for the generation of polygonal meshes based on terminal-edge
 * regions" (SIAM IMR 2022, arXiv 2204.05438). Only the test suite, the smoke
 * check and the benchmark's CPU-baseline leg may load this library; the product
 * path never does. It shares no code, header or table with the HIP library.
 *
 * It follows Algorithm 1 of the paper (label, generate polygons, repeat the
 * repair pass while barrier-edge tips remain) phase by phase:
 *   - label phase, Algorithm 2: LabelMax (per triangle), LabelSeed (per edge),
 *     LabelFrontier (per edge), as three separate loops;
 *   - traversal phase, Algorithm 3 with the PolyConstruction function;
 *   - reparation phase, Algorithm 4, run pass after pass until no tip remains.
 * All floating point is IEEE binary64 without contraction (build with
 * -ffp-contract=off); only squared lengths are compared, no square roots.
 *
 * Readings of the paper taken here (the paper is silent or ambiguous):
 *   - longest edge ties (Algorithm 2, LabelMax): edges are totally ordered by
 *     (squared length descending, edge key ascending) where the key of an edge
 *     is its smaller half-edge index (the half-edge itself on the hull);
 *   - PolyConstruction starts at the first frontier half-edge of the seed
 *     triangle in local order 0,1,2 (or, when the triangle has none, the first
 *     frontier half-edge met rotating about its vertex 0) and walks the
 *     frontier half-edges with the region on their left, so cycles are CCW;
 *   - "consecutive vertices" of the repair are taken cyclically; among the
 *     tips of a polygon the one with the smallest vertex id is repaired first;
 *   - the "middle internal edge" at tip v: rotate clockwise about v from the
 *     barrier half-edge c0 (c_{j+1} = next(twin(c_j))); with d the degree of v
 *     the internal edges are c_1..c_{d-1} and the middle one is c_{floor(d/2)};
 *     P_a is built from the triangle of that half-edge, P_b from the triangle
 *     of its twin, and both replace the repaired polygon in place;
 *   - every output cycle is rotated to its lexicographically smallest vertex
 *     sequence (which starts at its smallest vertex id); polygons are listed
 *     in seed-triangle order, and the pieces of a repaired polygon, which
 *     take its place, by ascending first and second vertex;
 *   - a barrier edge is a frontier edge whose two half-edges lie on the same
 *     polygon before repair;
 *   - a segment of a planar straight-line graph (a constrained edge of the
 *     input, the paper's guinea-pig example) bounds the domain on both of its
 *     sides, so each side is labelled like a boundary edge: always a frontier
 *     edge, and a boundary terminal edge with its own seed triangle on each
 *     side where it is the longest edge of that side's triangle. Holes are
 *     triangles absent from the input, their rims boundary edges.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* half-edge label bits */
#define OR_LONGEST 1u
#define OR_FRONTIER 2u
#define OR_TERMINAL 4u
#define OR_BORDER 8u
#define OR_BARRIER 16u
#define OR_REPAIRED 32u
#define OR_CONSTRAINED 64u
/* triangle / vertex label bits */
#define OR_SEED 1u
#define OR_TIP 1u

/* return codes */
#define OR_OK 0
#define OR_EINVAL (-1)
#define OR_ELAYOUT (-2)
#define OR_ETOPO (-3)
#define OR_ECAPACITY (-4)
#define OR_ENOMEM (-5)
#define OR_EDEGEN (-7)

/* stats slots */
enum {
  ST_SEEDS = 0,        /* number of terminal-edge regions (seed triangles) */
  ST_TIP_POLYGONS,     /* polygons with at least one tip before repair */
  ST_TIPS,             /* distinct tip vertices before repair */
  ST_SPLITS,           /* edges turned into frontier edges by the repair */
  ST_PASSES,           /* repair passes that found a tip */
  ST_NONSIMPLE_FINAL,  /* final polygons that still repeat a vertex */
  ST_MAXLEN_PRE,
  ST_MAXLEN_FINAL,
  ST_BARRIER_EDGES,    /* barrier edges (counted once per edge) */
  ST_COUNT
};

typedef struct {
  int64_t nv, nhe, nt;
  const double *xy;
  const int32_t *twin, *next, *origin;
  const uint8_t *fixed;  /* nonzero: the edge is a segment of the input PSLG (may be NULL) */
  uint8_t *he, *tri, *vtx;
  int32_t *maxe;  /* the paper's Max array: local index of the longest edge */
} mesh_t;

static int validate(const mesh_t *m) {
  if (m->nhe % 3 != 0) return OR_ELAYOUT;
  for (int64_t h = 0; h < m->nhe; ++h) {
    if (m->next[h] != (int32_t)(h - h % 3 + (h + 1) % 3)) return OR_ELAYOUT;
  }
  for (int64_t h = 0; h < m->nhe; ++h) {
    int32_t o = m->origin[h], t = m->twin[h];
    if (o < 0 || o >= m->nv) return OR_ETOPO;
    if (t < -1 || t >= m->nhe || t == h) return OR_ETOPO;
    if (t >= 0) {
      if (m->twin[t] != h) return OR_ETOPO;
      if (m->origin[t] != m->origin[m->next[h]]) return OR_ETOPO;
      if (m->fixed && (m->fixed[h] != 0) != (m->fixed[t] != 0)) return OR_ETOPO;
    }
  }
  return OR_OK;
}

static int is_frontier(const mesh_t *m, int32_t h) { return (m->he[h] & OR_FRONTIER) != 0; }

/* a boundary side: a hull or hole edge, or a segment of the input PSLG */
static int is_bounding(const mesh_t *m, int32_t h) { return m->twin[h] < 0 || (m->fixed && m->fixed[h]); }

/* squared length of half-edge h, rounded after every operation */
static double sq_length(const mesh_t *m, int32_t h) {
  int32_t a = m->origin[h], b = m->origin[m->next[h]];
  double dx = m->xy[2 * (int64_t)b] - m->xy[2 * (int64_t)a];
  double dy = m->xy[2 * (int64_t)b + 1] - m->xy[2 * (int64_t)a + 1];
  double dx2 = dx * dx;
  double dy2 = dy * dy;
  return dx2 + dy2;
}

static int32_t edge_key(const mesh_t *m, int32_t h) {
  int32_t t = m->twin[h];
  return (t < 0 || h < t) ? h : t;
}

/* ---------------------------- label phase ---------------------------- */

/* LabelMax: for every triangle, the local index of its longest edge. */
static void label_max(mesh_t *m) {
  for (int64_t t = 0; t < m->nt; ++t) {
    int best = 0;
    double lb = sq_length(m, (int32_t)(3 * t));
    int32_t kb = edge_key(m, (int32_t)(3 * t));
    for (int i = 1; i < 3; ++i) {
      int32_t h = (int32_t)(3 * t + i);
      double l = sq_length(m, h);
      int32_t k = edge_key(m, h);
      if (l > lb || (l == lb && k < kb)) { best = i; lb = l; kb = k; }
    }
    m->maxe[t] = best;
    m->he[3 * t + best] |= OR_LONGEST;
  }
}

/* LabelSeed: terminal edges and their seed triangle (lower index); a hull edge
 * (or a side of a PSLG segment) that is the longest edge of its triangle is a
 * border terminal edge. */
static void label_seed(mesh_t *m) {
  for (int64_t h = 0; h < m->nhe; ++h) {
    int32_t tw = m->twin[h];
    int64_t ta = h / 3;
    if (is_bounding(m, (int32_t)h)) { /* each side on its own */
      if (m->maxe[ta] == h % 3) {
        m->he[h] |= OR_TERMINAL;
        m->tri[ta] |= OR_SEED;
      }
      continue;
    }
    if (tw < h) continue; /* visit each interior edge once */
    int64_t tb = tw / 3;
    if (m->maxe[ta] == h % 3 && m->maxe[tb] == tw % 3) {
      m->he[h] |= OR_TERMINAL;
      m->he[tw] |= OR_TERMINAL;
      m->tri[ta < tb ? ta : tb] |= OR_SEED;
    }
  }
}

/* LabelFrontier: an edge is a frontier edge when it is a hull edge, a PSLG
 * segment or the longest edge of neither adjacent triangle. */
static void label_frontier(mesh_t *m) {
  for (int64_t h = 0; h < m->nhe; ++h) {
    int32_t tw = m->twin[h];
    if (tw >= 0 && tw < h) continue;
    if (tw < 0) {
      m->he[h] |= OR_FRONTIER | OR_BORDER;
      continue;
    }
    if (m->fixed && m->fixed[h]) {
      m->he[h] |= OR_FRONTIER | OR_CONSTRAINED;
      m->he[tw] |= OR_FRONTIER | OR_CONSTRAINED;
      continue;
    }
    int64_t ta = h / 3, tb = tw / 3;
    if (m->maxe[ta] != h % 3 && m->maxe[tb] != tw % 3) {
      m->he[h] |= OR_FRONTIER;
      m->he[tw] |= OR_FRONTIER;
    }
  }
}

/* ------------------------- polygon construction ------------------------- */

/* PolyConstruction from triangle t: the frontier half-edges of the region of
 * t, in the order met walking CCW around the region. The state of the walk is
 * the current frontier half-edge h (triangle h/3, vertex origin[h]); after
 * storing it, the walk moves to its end vertex and turns about that vertex
 * through the internal edges of the region until the next frontier edge.
 * Returns the cycle length or a negative code. */
static int64_t poly_construction(const mesh_t *m, int64_t t, int32_t *out, int64_t cap) {
  int32_t s = -1;
  for (int i = 0; i < 3 && s < 0; ++i)
    if (is_frontier(m, (int32_t)(3 * t + i))) s = (int32_t)(3 * t + i);
  if (s < 0) {
    int32_t c = (int32_t)(3 * t);
    for (int64_t k = 0; k <= m->nhe && s < 0; ++k) {
      if (is_frontier(m, c)) s = c;
      else c = m->next[m->twin[c]];
    }
    if (s < 0) return OR_EDEGEN;
  }
  int64_t len = 0;
  int32_t h = s;
  do {
    if (len >= cap) return OR_EDEGEN;
    out[len++] = h;
    int32_t c = m->next[h];
    int64_t turns = 0;
    while (!is_frontier(m, c)) {
      c = m->next[m->twin[c]];
      if (++turns > m->nhe) return OR_EDEGEN;
    }
    h = c;
  } while (h != s);
  return len;
}

/* ------------------------------ polygon list ------------------------------ */

typedef struct {
  int64_t n, cap_n, len, cap_len;
  int64_t *off;   /* [n+1] */
  int32_t *hes;   /* half-edge cycles */
  int64_t *root;  /* index of the polygon before repair this one comes from */
} plist_t;

static int pl_init(plist_t *p, int64_t cap_n, int64_t cap_len) {
  p->n = 0; p->len = 0; p->cap_n = cap_n; p->cap_len = cap_len;
  p->off = (int64_t *)malloc(sizeof(int64_t) * (size_t)(cap_n + 1));
  p->hes = (int32_t *)malloc(sizeof(int32_t) * (size_t)(cap_len > 0 ? cap_len : 1));
  p->root = (int64_t *)malloc(sizeof(int64_t) * (size_t)(cap_n + 1));
  if (!p->off || !p->hes || !p->root) return OR_ENOMEM;
  p->off[0] = 0;
  return OR_OK;
}
static void pl_free(plist_t *p) { free(p->off); free(p->hes); free(p->root); }

static int pl_push(plist_t *p, const int32_t *c, int64_t len, int64_t root) {
  if (p->n + 1 > p->cap_n || p->len + len > p->cap_len) return OR_ECAPACITY;
  memcpy(p->hes + p->len, c, sizeof(int32_t) * (size_t)len);
  p->root[p->n] = root;
  p->len += len;
  p->n += 1;
  p->off[p->n] = p->len;
  return OR_OK;
}

/* smallest tip vertex of a cycle (v_a == v_c for consecutive v_a, v_b, v_c,
 * taken cyclically); returns -1 when there is none and the position of v_b. */
static int32_t min_tip(const mesh_t *m, const int32_t *c, int64_t len, int64_t *pos) {
  int32_t best = -1;
  for (int64_t k = 0; k < len && len >= 3; ++k) {
    int32_t va = m->origin[c[k]];
    int32_t vb = m->origin[c[(k + 1) % len]];
    int32_t vc = m->origin[c[(k + 2) % len]];
    if (va == vc && (best < 0 || vb < best)) { best = vb; *pos = (k + 1) % len; }
  }
  return best;
}

/* lexicographically smallest rotation of the vertex sequence of a cycle */
static int64_t least_rotation(const mesh_t *m, const int32_t *c, int64_t len) {
  int64_t best = 0;
  for (int64_t r = 1; r < len; ++r) {
    for (int64_t k = 0; k < len; ++k) {
      int32_t a = m->origin[c[(r + k) % len]], b = m->origin[c[(best + k) % len]];
      if (a != b) { if (a < b) best = r; break; }
    }
  }
  return best;
}

static int has_repeated_vertex(const mesh_t *m, const int32_t *c, int64_t len) {
  for (int64_t i = 0; i < len; ++i)
    for (int64_t j = i + 1; j < len; ++j)
      if (m->origin[c[i]] == m->origin[c[j]]) return 1;
  return 0;
}

/* Write a list as canonical CSR vertex cycles. Polygons keep the order of the
 * polygons before repair they come from; the pieces of one repaired polygon
 * are listed by ascending (first, second) vertex of their canonical cycle. */
static int emit(const mesh_t *m, const plist_t *p, int32_t *off, int32_t *verts, int32_t *start,
                int64_t cap_polys, int64_t cap_verts, int64_t *counts) {
  if (p->n > cap_polys || p->len > cap_verts) return OR_ECAPACITY;
  int64_t *rot = (int64_t *)malloc(sizeof(int64_t) * (size_t)(p->n + 1));
  int64_t *ord = (int64_t *)malloc(sizeof(int64_t) * (size_t)(p->n + 1));
  int32_t *k0 = (int32_t *)malloc(sizeof(int32_t) * (size_t)(p->n + 1));
  int32_t *k1 = (int32_t *)malloc(sizeof(int32_t) * (size_t)(p->n + 1));
  if (!rot || !ord || !k0 || !k1) { free(rot); free(ord); free(k0); free(k1); return OR_ENOMEM; }
  for (int64_t i = 0; i < p->n; ++i) {
    const int32_t *c = p->hes + p->off[i];
    int64_t len = p->off[i + 1] - p->off[i];
    rot[i] = least_rotation(m, c, len);
    k0[i] = m->origin[c[rot[i]]];
    k1[i] = m->origin[c[(rot[i] + 1) % len]];
    ord[i] = i;
  }
  /* insertion sort inside each group of pieces sharing a root */
  for (int64_t g = 0; g < p->n;) {
    int64_t e = g + 1;
    while (e < p->n && p->root[e] == p->root[g]) ++e;
    for (int64_t i = g + 1; i < e; ++i) {
      int64_t x = ord[i], j = i;
      while (j > g && (k0[ord[j - 1]] > k0[x] || (k0[ord[j - 1]] == k0[x] && k1[ord[j - 1]] > k1[x]))) {
        ord[j] = ord[j - 1];
        --j;
      }
      ord[j] = x;
    }
    g = e;
  }
  int64_t w = 0;
  off[0] = 0;
  for (int64_t q = 0; q < p->n; ++q) {
    int64_t i = ord[q];
    const int32_t *c = p->hes + p->off[i];
    int64_t len = p->off[i + 1] - p->off[i];
    if (start) start[q] = c[rot[i]];
    for (int64_t k = 0; k < len; ++k) verts[w++] = m->origin[c[(rot[i] + k) % len]];
    off[q + 1] = (int32_t)w;
  }
  counts[0] = p->n;
  counts[1] = w;
  free(rot); free(ord); free(k0); free(k1);
  return OR_OK;
}

/* ------------------------------ Algorithm 1 ------------------------------ */

int oracle_mesh(int64_t nv, int64_t nhe, const double *xy, const int32_t *twin,
                const int32_t *next, const int32_t *origin, const uint8_t *fixed,
                uint8_t *he_labels, uint8_t *tri_labels, uint8_t *vtx_labels,
                int32_t *pre_off, int32_t *pre_verts, int32_t *pre_start, int64_t *pre_counts,
                int32_t *off, int32_t *verts, int32_t *start, int64_t *counts,
                int64_t cap_polys, int64_t cap_verts, int64_t *stats) {
  if (nv < 0 || nhe < 0 || !he_labels || !tri_labels || !vtx_labels || !off || !verts ||
      !counts || !stats || !pre_off || !pre_verts || !pre_counts)
    return OR_EINVAL;
  if (nhe > 0 && (!xy || !twin || !next || !origin)) return OR_EINVAL;
  if (nhe >= INT32_MAX || nv >= INT32_MAX) return OR_EINVAL;
  mesh_t m;
  m.nv = nv; m.nhe = nhe; m.nt = nhe / 3;
  m.xy = xy; m.twin = twin; m.next = next; m.origin = origin; m.fixed = fixed;
  m.he = he_labels; m.tri = tri_labels; m.vtx = vtx_labels;
  for (int i = 0; i < ST_COUNT; ++i) stats[i] = 0;
  int rc = validate(&m);
  if (rc) return rc;
  memset(m.he, 0, (size_t)nhe);
  memset(m.tri, 0, (size_t)m.nt);
  memset(m.vtx, 0, (size_t)nv);
  m.maxe = (int32_t *)malloc(sizeof(int32_t) * (size_t)(m.nt + 1));
  if (!m.maxe) return OR_ENOMEM;

  /* Label phase (Algorithm 2) */
  label_max(&m);
  label_seed(&m);
  label_frontier(&m);

  /* Traversal phase (Algorithm 3): one polygon per seed triangle */
  plist_t cur, nxt;
  int32_t *buf = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nhe + 1));
  int32_t *cyc = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nhe + 1));
  int32_t *trivertex = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nv + 1));
  if (!buf || !cyc || !trivertex) { rc = OR_ENOMEM; goto done0; }
  if ((rc = pl_init(&cur, m.nt + 1, nhe + 1))) goto done0;
  if ((rc = pl_init(&nxt, m.nt + 1, nhe + 1))) { pl_free(&cur); goto done0; }
  for (int64_t t = 0; t < m.nt; ++t) {
    if (!(m.tri[t] & OR_SEED)) continue;
    stats[ST_SEEDS]++;
    int64_t len = poly_construction(&m, t, buf, nhe);
    if (len < 0) { rc = (int)len; goto done; }
    if ((rc = pl_push(&cur, buf, len, cur.n))) goto done;
  }
  if ((rc = emit(&m, &cur, pre_off, pre_verts, pre_start, cap_polys, cap_verts, pre_counts))) goto done;

  /* Barrier edges: frontier edges whose two half-edges lie on one polygon. */
  for (int64_t h = 0; h < nhe; ++h) cyc[h] = -1;
  for (int64_t i = 0; i < cur.n; ++i) {
    int64_t len = cur.off[i + 1] - cur.off[i];
    if (len > stats[ST_MAXLEN_PRE]) stats[ST_MAXLEN_PRE] = len;
    for (int64_t k = cur.off[i]; k < cur.off[i + 1]; ++k) cyc[cur.hes[k]] = (int32_t)i;
  }
  for (int64_t h = 0; h < nhe; ++h) {
    int32_t tw = twin[h];
    if (tw >= 0 && cyc[h] >= 0 && cyc[h] == cyc[tw]) {
      m.he[h] |= OR_BARRIER;
      if (h < tw) stats[ST_BARRIER_EDGES]++;
    }
  }
  /* Tips before repair */
  for (int64_t i = 0; i < cur.n; ++i) {
    const int32_t *c = cur.hes + cur.off[i];
    int64_t len = cur.off[i + 1] - cur.off[i];
    int found = 0;
    for (int64_t k = 0; k < len && len >= 3; ++k) {
      int32_t va = origin[c[k]], vb = origin[c[(k + 1) % len]], vc = origin[c[(k + 2) % len]];
      if (va == vc) {
        found = 1;
        if (!(m.vtx[vb] & OR_TIP)) stats[ST_TIPS]++;
        m.vtx[vb] |= OR_TIP;
      }
    }
    stats[ST_TIP_POLYGONS] += found;
  }

  /* Reparation phase (Algorithm 4), repeated while tips remain. The
   * Trivertex array gives one triangle incident to each vertex. */
  for (int64_t v = 0; v < nv; ++v) trivertex[v] = -1;
  for (int64_t h = 0; h < nhe; ++h)
    if (trivertex[origin[h]] < 0) trivertex[origin[h]] = (int32_t)(h / 3);
  for (;;) {
    int any = 0;
    nxt.n = 0; nxt.len = 0; nxt.off[0] = 0;
    for (int64_t i = 0; i < cur.n; ++i) {
      const int32_t *c = cur.hes + cur.off[i];
      int64_t len = cur.off[i + 1] - cur.off[i];
      int64_t pos = -1;
      int32_t vbet = min_tip(&m, c, len, &pos);
      if (vbet < 0) {
        if ((rc = pl_push(&nxt, c, len, cur.root[i]))) goto done;
        continue;
      }
      any = 1;
      /* half-edge of the Trivertex triangle leaving v_bet */
      int64_t tv = trivertex[vbet];
      int32_t c0 = -1;
      for (int k = 0; k < 3; ++k)
        if (origin[3 * tv + k] == vbet) c0 = (int32_t)(3 * tv + k);
      /* turn about v_bet to its (only) frontier edge: the barrier edge */
      for (int64_t k = 0; k <= nhe && !is_frontier(&m, c0); ++k) c0 = next[twin[c0]];
      if (!is_frontier(&m, c0)) { rc = OR_EDEGEN; goto done; }
      /* internal edges c_1..c_{d-1}, clockwise from c0 */
      int64_t d = 0;
      int32_t cj = c0;
      do {
        cj = next[twin[cj]];
        d++;
        if (d > nhe) { rc = OR_EDEGEN; goto done; }
      } while (cj != c0);
      int32_t e = c0;
      for (int64_t j = 0; j < d / 2; ++j) e = next[twin[e]];
      int32_t et = twin[e];
      m.he[e] |= OR_FRONTIER | OR_REPAIRED;
      m.he[et] |= OR_FRONTIER | OR_REPAIRED;
      stats[ST_SPLITS]++;
      int64_t la = poly_construction(&m, e / 3, buf, nhe);
      if (la < 0) { rc = (int)la; goto done; }
      if ((rc = pl_push(&nxt, buf, la, cur.root[i]))) goto done;
      int64_t lb = poly_construction(&m, et / 3, buf, nhe);
      if (lb < 0) { rc = (int)lb; goto done; }
      if ((rc = pl_push(&nxt, buf, lb, cur.root[i]))) goto done;
      if (la + lb != len + 2) { rc = OR_EDEGEN; goto done; }
      (void)pos;
    }
    plist_t tmp = cur; cur = nxt; nxt = tmp;
    if (!any) break;
    stats[ST_PASSES]++;
  }
  for (int64_t i = 0; i < cur.n; ++i) {
    int64_t len = cur.off[i + 1] - cur.off[i];
    if (len > stats[ST_MAXLEN_FINAL]) stats[ST_MAXLEN_FINAL] = len;
    stats[ST_NONSIMPLE_FINAL] += has_repeated_vertex(&m, cur.hes + cur.off[i], len);
  }
  rc = emit(&m, &cur, off, verts, start, cap_polys, cap_verts, counts);
done:
  pl_free(&cur);
  pl_free(&nxt);
done0:
  free(buf);
  free(cyc);
  free(trivertex);
  free(m.maxe);
  return rc;
}

/* ------------------------------- Lepp ------------------------------- */

/* Longest-edge propagation path of every triangle (the paper names Lepp-based
 * algorithms as the next use of its label kernels; Lepp as defined by Rivara):
 * Lepp(t) = t_0 = t, t_1, ..., t_n where t_{i+1} is the neighbour of t_i across
 * the longest edge of t_i, ending when that edge is also the longest edge of
 * t_{i+1} (a terminal edge shared by t_{n-1} and t_n) or is a boundary edge
 * (or a side of an input segment) of t_n. terminal[t] = the edge key (smaller
 * half-edge, or the boundary half-edge) of the terminal edge; length[t] = n + 1
 * triangles. Longest edges use the same (length, edge key) order as LabelMax. */
int oracle_lepp(int64_t nv, int64_t nhe, const double *xy, const int32_t *twin, const int32_t *next,
                const int32_t *origin, const uint8_t *fixed, int32_t *terminal, int32_t *length) {
  if (nv < 0 || nhe < 0 || (nhe > 0 && (!xy || !twin || !next || !origin || !terminal || !length)))
    return OR_EINVAL;
  if (nhe >= INT32_MAX || nv >= INT32_MAX) return OR_EINVAL;
  mesh_t m;
  memset(&m, 0, sizeof(m));
  m.nv = nv; m.nhe = nhe; m.nt = nhe / 3;
  m.xy = xy; m.twin = twin; m.next = next; m.origin = origin; m.fixed = fixed;
  int rc = validate(&m);
  if (rc) return rc;
  uint8_t *he = (uint8_t *)calloc((size_t)nhe + 1, 1);
  m.maxe = (int32_t *)malloc(sizeof(int32_t) * (size_t)(m.nt + 1));
  if (!he || !m.maxe) { free(he); free(m.maxe); return OR_ENOMEM; }
  m.he = he;
  label_max(&m);
  for (int64_t t = 0; t < m.nt; ++t) {
    int64_t cur = t, n = 1;
    for (;;) {
      int32_t h = (int32_t)(3 * cur + m.maxe[cur]);
      if (is_bounding(&m, h)) { terminal[t] = h; break; }
      int32_t u = twin[h];
      int64_t nb = u / 3;
      ++n;
      if (m.maxe[nb] == u % 3) { terminal[t] = h < u ? h : u; break; }
      cur = nb;
      if (n > m.nt + 1) { rc = OR_EDEGEN; goto out; }
    }
    length[t] = (int32_t)n;
  }
out:
  free(he);
  free(m.maxe);
  return rc;
}
