// Seeded input generator, native part: incremental Delaunay triangulation
// (Bowyer-Watson cavity insertion with a ghost vertex closing the convex hull)
// over points on an integer lattice.
//
// This file is input generation only. It holds none of the meshing method's
// arithmetic (no edge lengths, labels or polygons) and is shared by the test
// oracle and the GPU path as the source of their common inputs.
//
// Exactness: coordinates are integers in [0, 2^28]. orient2d fits in int64
// (|diff| <= 2^28, products <= 2^56) and incircle fits in __int128
// (lifted terms <= 2^57, 2x2 minors <= 2^57, three products < 2^116), so every
// predicate is evaluated exactly and the construction never loops on rounding.
// Degenerate cases: a point exactly on a circumcircle is not in conflict, a
// point on the open segment of a hull edge is in conflict with that hull edge's
// ghost triangle. Collinear points on the hull therefore all become vertices.
//
// C ABI (ctypes):
//   void*   mg_delaunay_run(int64_t n, const int64_t* X, const int64_t* Y,
//                           int64_t* n_tri_out, int32_t* status);
//   void    mg_delaunay_fetch(void* h, int32_t* origin, int32_t* twin);
//   void    mg_delaunay_free(void* h);
// Output layout (after fetch): triangle t has vertices origin[3t+0..2] in CCW
// order with the smallest vertex id first; triangles are sorted by
// (origin[3t], origin[3t+1]); twin[3t+i] is the half-edge index of the same
// edge in the adjacent triangle, -1 on the convex hull. Half-edge 3t+i runs
// from origin[3t+i] to origin[3t+(i+1)%3].

#include <cstdint>
#include <cstring>
#include <vector>
#include <algorithm>

namespace {

typedef __int128 i128;

struct Delaunay {
  const int64_t* X;
  const int64_t* Y;
  int32_t n;
  int32_t INF;                 // ghost vertex id (== n)
  std::vector<int32_t> v;      // 3 vertex ids per triangle slot
  std::vector<int32_t> nb;     // 3 twin half-edge ids per triangle slot
  std::vector<uint8_t> alive;
  std::vector<int32_t> free_slots;
  std::vector<uint32_t> st_in, st_out;
  std::vector<int32_t> start_of;  // per vertex (incl. ghost): new triangle starting there
  std::vector<int32_t> stack, cavity;
  struct Bd { int32_t a, b, outer; };
  std::vector<Bd> bd;
  uint32_t stamp = 0;
  int32_t last = 0;

  int64_t orient(int32_t a, int32_t b, int32_t c) const {
    return (X[b] - X[a]) * (Y[c] - Y[a]) - (Y[b] - Y[a]) * (X[c] - X[a]);
  }
  // > 0 iff d lies strictly inside the circumcircle of CCW triangle (a, b, c).
  int incircle(int32_t a, int32_t b, int32_t c, int32_t d) const {
    int64_t adx = X[a] - X[d], ady = Y[a] - Y[d];
    int64_t bdx = X[b] - X[d], bdy = Y[b] - Y[d];
    int64_t cdx = X[c] - X[d], cdy = Y[c] - Y[d];
    int64_t al = adx * adx + ady * ady;
    int64_t bl = bdx * bdx + bdy * bdy;
    int64_t cl = cdx * cdx + cdy * cdy;
    i128 m_bc = (i128)bdx * cdy - (i128)bdy * cdx;
    i128 m_ca = (i128)cdx * ady - (i128)cdy * adx;
    i128 m_ab = (i128)adx * bdy - (i128)ady * bdx;
    i128 det = (i128)al * m_bc + (i128)bl * m_ca + (i128)cl * m_ab;
    return det > 0 ? 1 : (det < 0 ? -1 : 0);
  }
  bool is_ghost(int32_t t) const {
    return v[3 * t] == INF || v[3 * t + 1] == INF || v[3 * t + 2] == INF;
  }
  // Hull edge (a -> b) of a ghost triangle; the outside lies to its left.
  void ghost_edge(int32_t t, int32_t& a, int32_t& b) const {
    const int32_t* w = &v[3 * t];
    if (w[2] == INF) { a = w[0]; b = w[1]; }
    else if (w[0] == INF) { a = w[1]; b = w[2]; }
    else { a = w[2]; b = w[0]; }
  }
  bool conflict(int32_t t, int32_t p) const {
    if (!is_ghost(t)) return incircle(v[3 * t], v[3 * t + 1], v[3 * t + 2], p) > 0;
    int32_t a, b;
    ghost_edge(t, a, b);
    int64_t o = orient(a, b, p);
    if (o != 0) return o > 0;
    // collinear with the hull edge: conflict only on the open segment
    int64_t d1 = (X[p] - X[a]) * (X[b] - X[a]) + (Y[p] - Y[a]) * (Y[b] - Y[a]);
    int64_t d2 = (X[p] - X[b]) * (X[a] - X[b]) + (Y[p] - Y[b]) * (Y[a] - Y[b]);
    return d1 > 0 && d2 > 0;
  }
  int32_t alloc() {
    int32_t t;
    if (!free_slots.empty()) { t = free_slots.back(); free_slots.pop_back(); }
    else {
      t = (int32_t)(v.size() / 3);
      v.resize(v.size() + 3); nb.resize(nb.size() + 3);
      alive.push_back(0); st_in.push_back(0); st_out.push_back(0);
    }
    alive[t] = 1;
    return t;
  }
  void link(int32_t h1, int32_t h2) { nb[h1] = h2; nb[h2] = h1; }

  // Visibility walk from `start` to a triangle in conflict with p.
  int32_t locate(int32_t p) {
    int32_t t = last;
    if (!alive[t]) t = 0;
    while (!alive[t]) ++t;
    if (is_ghost(t)) {
      int32_t a, b; ghost_edge(t, a, b);
      // the finite triangle across the hull edge
      for (int i = 0; i < 3; ++i)
        if (v[3 * t + i] == a && v[3 * t + (i + 1) % 3] == b) { t = nb[3 * t + i] / 3; break; }
    }
    uint32_t rot = (uint32_t)p;
    for (int64_t steps = 0;; ++steps) {
      if (is_ghost(t)) return t;
      bool moved = false;
      for (int k = 0; k < 3; ++k) {
        int i = (int)((k + rot) % 3);
        int32_t a = v[3 * t + i], b = v[3 * t + (i + 1) % 3];
        if (orient(a, b, p) < 0) { t = nb[3 * t + i] / 3; moved = true; break; }
      }
      if (!moved) return t;
      rot = rot * 1103515245u + 12345u;
      if (steps > 4 * (int64_t)n + 64) break;  // cannot happen on a Delaunay mesh
    }
    // Fallback: exhaustive search (never expected).
    int32_t T = (int32_t)(v.size() / 3);
    for (int32_t t2 = 0; t2 < T; ++t2)
      if (alive[t2] && conflict(t2, p)) return t2;
    return -1;
  }

  bool insert(int32_t p) {
    int32_t t0 = locate(p);
    if (t0 < 0 || !conflict(t0, p)) return false;
    ++stamp;
    stack.clear(); cavity.clear(); bd.clear();
    st_in[t0] = stamp;
    stack.push_back(t0);
    while (!stack.empty()) {
      int32_t t = stack.back(); stack.pop_back();
      cavity.push_back(t);
      for (int i = 0; i < 3; ++i) {
        int32_t he = nb[3 * t + i];
        int32_t u = he / 3;
        if (st_in[u] == stamp) continue;
        if (st_out[u] != stamp) {
          if (conflict(u, p)) { st_in[u] = stamp; stack.push_back(u); continue; }
          st_out[u] = stamp;
        }
        bd.push_back({v[3 * t + i], v[3 * t + (i + 1) % 3], he});
      }
    }
    for (int32_t t : cavity) { alive[t] = 0; free_slots.push_back(t); }
    int32_t first_new = -1;
    for (const Bd& e : bd) {
      int32_t T = alloc();
      v[3 * T] = e.a; v[3 * T + 1] = e.b; v[3 * T + 2] = p;
      link(3 * T, e.outer);
      start_of[e.a] = T;
      if (first_new < 0 || (e.a != INF && e.b != INF)) first_new = T;
    }
    for (const Bd& e : bd) {
      int32_t T = start_of[e.a];
      int32_t U = start_of[e.b];
      link(3 * T + 1, 3 * U + 2);
    }
    last = first_new;
    return true;
  }

  int run() {
    INF = n;
    start_of.assign((size_t)n + 1, -1);
    if (n < 3) return 1;
    int32_t k = -1;
    for (int32_t i = 2; i < n; ++i)
      if (orient(0, 1, i) != 0) { k = i; break; }
    if (k < 0) return 2;  // all collinear
    int32_t a = 0, b = 1, c = k;
    if (orient(a, b, c) < 0) std::swap(b, c);
    v.reserve((size_t)6 * n + 64); nb.reserve((size_t)6 * n + 64);
    int32_t T0 = alloc();
    v[0] = a; v[1] = b; v[2] = c;
    int32_t G[3];
    const int32_t w[3] = {a, b, c};
    for (int i = 0; i < 3; ++i) {
      G[i] = alloc();
      v[3 * G[i]] = w[(i + 1) % 3]; v[3 * G[i] + 1] = w[i]; v[3 * G[i] + 2] = INF;
      link(3 * T0 + i, 3 * G[i]);
    }
    for (int i = 0; i < 3; ++i) link(3 * G[i] + 2, 3 * G[(i + 1) % 3] + 1);
    last = T0;
    for (int32_t p = 2; p < n; ++p) {
      if (p == k) continue;
      if (!insert(p)) return 3;  // duplicate point or internal failure
    }
    return 0;
  }
};

struct Result {
  std::vector<int32_t> origin, twin;
};

}  // namespace

extern "C" {

void* mg_delaunay_run(int64_t n, const int64_t* X, const int64_t* Y, int64_t* n_tri_out,
                      int32_t* status) {
  Delaunay D;
  D.X = X; D.Y = Y; D.n = (int32_t)n;
  *status = D.run();
  *n_tri_out = 0;
  if (*status != 0) return nullptr;
  const int32_t S = (int32_t)(D.v.size() / 3);
  // finite triangles, rotated to start at their smallest vertex id
  std::vector<int32_t> ids;
  std::vector<int8_t> rot((size_t)S, 0);
  ids.reserve((size_t)2 * n);
  for (int32_t t = 0; t < S; ++t) {
    if (!D.alive[t] || D.is_ghost(t)) continue;
    const int32_t* w = &D.v[3 * t];
    int r = 0;
    if (w[1] < w[r]) r = 1;
    if (w[2] < w[r]) r = 2;
    rot[t] = (int8_t)r;
    ids.push_back(t);
  }
  const int64_t T = (int64_t)ids.size();
  // sort by (first vertex, second vertex): bucket by the first vertex, then
  // order each (small) bucket by the second vertex
  std::vector<int64_t> cnt((size_t)n + 1, 0);
  for (int32_t t : ids) cnt[D.v[3 * t + rot[t]] + 1]++;
  for (int64_t i = 0; i < n; ++i) cnt[i + 1] += cnt[i];
  std::vector<int32_t> order((size_t)T);
  {
    std::vector<int64_t> pos(cnt.begin(), cnt.end() - 1);
    for (int32_t t : ids) order[pos[D.v[3 * t + rot[t]]]++] = t;
  }
  for (int64_t i = 0; i < n; ++i) {
    auto b = order.begin() + cnt[i], e = order.begin() + cnt[i + 1];
    if (e - b > 1)
      std::sort(b, e, [&](int32_t p, int32_t q) {
        return D.v[3 * p + (rot[p] + 1) % 3] < D.v[3 * q + (rot[q] + 1) % 3];
      });
  }
  std::vector<int32_t> newid((size_t)S, -1);
  for (int64_t i = 0; i < T; ++i) newid[order[i]] = (int32_t)i;
  Result* R = new Result();
  R->origin.resize((size_t)3 * T);
  R->twin.resize((size_t)3 * T);
  for (int64_t i = 0; i < T; ++i) {
    int32_t t = order[i];
    int r = rot[t];
    for (int j = 0; j < 3; ++j) {
      int oj = (r + j) % 3;
      R->origin[3 * i + j] = D.v[3 * t + oj];
      int32_t he = D.nb[3 * t + oj];
      int32_t u = he / 3, ui = he % 3;
      if (D.is_ghost(u)) { R->twin[3 * i + j] = -1; continue; }
      int uj = (ui - rot[u] + 3) % 3;
      R->twin[3 * i + j] = 3 * newid[u] + uj;
    }
  }
  *n_tri_out = T;
  return R;
}

void mg_delaunay_fetch(void* h, int32_t* origin, int32_t* twin) {
  Result* R = (Result*)h;
  std::memcpy(origin, R->origin.data(), R->origin.size() * sizeof(int32_t));
  std::memcpy(twin, R->twin.data(), R->twin.size() * sizeof(int32_t));
}

void mg_delaunay_free(void* h) { delete (Result*)h; }

}  // extern "C"
