// Reparation phase (Algorithm 4, repeated as in Algorithm 1) on the host: the
// sequential half of the paper's "mixed" configuration, in which the GPU
// labels the mesh and builds the polygons and the CPU repairs the few
// non-simple ones. Host-only C++ (no device code).
//
// A polygon with barrier-edge tips is split recursively: in each piece, the
// tip with the smallest vertex id opens the middle internal edge of its fan
// (c_{floor(d/2)}, turning clockwise from the barrier half-edge leaving it),
// and the two sides are walked again from the opened edge's half-edges. The
// pieces of one polygon share no triangle, so the order in which they are
// split does not change the result. Final pieces are rotated to their
// lexicographically least vertex sequence and take their polygon's place,
// ordered by their first two vertices.
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "../../include/polylla.h"

namespace polylla {

namespace {

struct HostMesh {
  int64_t nhe;
  const int32_t* twin;
  const int32_t* origin;
  uint8_t* he;
  static int32_t next(int32_t h) { return h % 3 == 2 ? h - 2 : h + 1; }
  bool frontier(int32_t h) const { return (he[h] & POLYLLA_FRONTIER) != 0; }
  // next frontier half-edge of the cycle after frontier half-edge h (-1: invalid mesh)
  int32_t succ(int32_t h) const {
    int32_t c = next(h);
    for (int64_t steps = 0; steps <= nhe; ++steps) {
      if (frontier(c)) return c;
      const int32_t tw = twin[c];
      if (tw < 0 || tw >= nhe) return -1;
      c = next(tw);
    }
    return -1;
  }
  // the cycle of frontier half-edges from h, appended to out; false on an invalid mesh
  bool cycle(int32_t h, std::vector<int32_t>& out) const {
    const size_t first = out.size();
    int32_t c = h;
    do {
      out.push_back(c);
      c = succ(c);
      if (c < 0 || (int64_t)(out.size() - first) > nhe) return false;
    } while (c != h);
    return true;
  }
};

// Position of the smallest tip vertex of a cycle (v_{k-1} == v_{k+1}), -1 if none.
int64_t min_tip_pos(const HostMesh& m, const int32_t* c, int64_t len) {
  if (len < 3) return -1;
  int64_t best = -1;
  for (int64_t k = 0; k < len; ++k) {
    const int32_t vp = m.origin[c[(k + len - 1) % len]], vn = m.origin[c[(k + 1) % len]];
    if (vp == vn && (best < 0 || m.origin[c[k]] < m.origin[c[best]])) best = k;
  }
  return best;
}

// Start of the lexicographically least rotation of the cycle's vertex sequence.
int64_t least_rotation(const HostMesh& m, const int32_t* c, int64_t len) {
  int64_t best = 0;
  for (int64_t r = 1; r < len; ++r) {
    for (int64_t k = 0; k < len; ++k) {
      const int32_t a = m.origin[c[(r + k) % len]], b = m.origin[c[(best + k) % len]];
      if (a != b) {
        if (a < b) best = r;
        break;
      }
    }
  }
  return best;
}

struct Piece {
  int64_t at, len;  // slice of the piece buffer
  int64_t rot;
  int32_t v0, v1;
};

}  // namespace

// Repairs the polygons of a pre-repair CSR (as polylla_build writes it) and
// writes the final CSR. he gets FRONTIER | REPAIRED on the opened edges.
// stats[0] polygons repaired, stats[1] edges opened. Returns a polylla code.
int host_repair(int64_t nhe, const int32_t* twin, const int32_t* origin, uint8_t* he, int64_t F,
                const int32_t* off, const int32_t* verts, const int32_t* start, int32_t* out_off,
                int32_t* out_verts, int32_t* out_start, int64_t cap_polys, int64_t cap_verts, int64_t* counts,
                int64_t* stats) {
  HostMesh m{nhe, twin, origin, he};
  int64_t np = 0, nv = 0;
  stats[0] = stats[1] = 0;
  out_off[0] = 0;
  std::vector<int32_t> buf, fan;
  std::vector<int64_t> todo;
  std::vector<std::pair<int64_t, int64_t>> seg;
  std::vector<Piece> done;
  for (int64_t p = 0; p < F; ++p) {
    const int32_t* v = verts + off[p];
    const int64_t L = off[p + 1] - off[p];
    bool tip = false;
    for (int64_t k = 0; k < L && L >= 3 && !tip; ++k) tip = v[(k + L - 1) % L] == v[(k + 1) % L];
    if (!tip) {  // unchanged: copied
      if (np + 1 > cap_polys || nv + L > cap_verts) return POLYLLA_ECAPACITY;
      memcpy(out_verts + nv, v, sizeof(int32_t) * (size_t)L);
      if (out_start) out_start[np] = start[p];
      nv += L;
      out_off[++np] = (int32_t)nv;
      continue;
    }
    ++stats[0];
    // the polygon's half-edge cycle, then split pieces until none has a tip;
    // every piece is a slice (offset, length) of buf
    buf.clear();
    done.clear();
    seg.clear();
    if (!m.cycle(start[p], buf)) return POLYLLA_EDEGEN;
    seg.push_back({0, (int64_t)buf.size()});
    todo.assign(1, 0);
    while (!todo.empty()) {
      const int64_t at = seg[todo.back()].first, len = seg[todo.back()].second;
      todo.pop_back();
      const int64_t k = min_tip_pos(m, buf.data() + at, len);
      if (k < 0) {
        const int32_t* c = buf.data() + at;
        const int64_t r = least_rotation(m, c, len);
        done.push_back({at, len, r, m.origin[c[r]], m.origin[c[(r + 1) % len]]});
        continue;
      }
      // fan of the tip: c_0 = barrier half-edge leaving it, c_{j+1} = next(twin(c_j))
      const int32_t c0 = buf[at + k];
      fan.clear();
      int32_t x = c0;
      do {
        fan.push_back(x);
        const int32_t tw = twin[x];
        if (tw < 0 || tw >= nhe || (int64_t)fan.size() > nhe) return POLYLLA_EDEGEN;
        x = HostMesh::next(tw);
      } while (x != c0);
      const int64_t d = (int64_t)fan.size();
      if (d < 2) return POLYLLA_EDEGEN;
      const int32_t e = fan[d / 2], te = twin[e];
      if (te < 0) return POLYLLA_EDEGEN;
      he[e] |= POLYLLA_FRONTIER | POLYLLA_REPAIRED;
      he[te] |= POLYLLA_FRONTIER | POLYLLA_REPAIRED;
      ++stats[1];
      // the two sides, walked again from the opened edge's half-edges
      for (const int32_t s0 : {e, te}) {
        const int64_t a0 = (int64_t)buf.size();
        if (!m.cycle(s0, buf)) return POLYLLA_EDEGEN;
        seg.push_back({a0, (int64_t)buf.size() - a0});
        todo.push_back((int64_t)seg.size() - 1);
      }
    }
    std::sort(done.begin(), done.end(), [](const Piece& a, const Piece& b) {
      return a.v0 < b.v0 || (a.v0 == b.v0 && a.v1 < b.v1);
    });
    for (const Piece& q : done) {
      if (np + 1 > cap_polys || nv + q.len > cap_verts) return POLYLLA_ECAPACITY;
      for (int64_t j = 0; j < q.len; ++j) out_verts[nv + j] = origin[buf[q.at + (q.rot + j) % q.len]];
      if (out_start) out_start[np] = buf[q.at + q.rot];
      nv += q.len;
      out_off[++np] = (int32_t)nv;
    }
  }
  counts[0] = np;
  counts[1] = nv;
  return POLYLLA_OK;
}

}  // namespace polylla
