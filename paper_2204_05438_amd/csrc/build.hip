// Traversal phase (Algorithm 3, PolyConstruction) and Reparation phase
// (Algorithm 4) as gfx950 kernels.
//
// k_walk          : persistent lanes, one polygon each at a time. Walks the
//                   frontier half-edges of the region from its start
//                   half-edge with the region on the left (turning about each
//                   vertex through internal edges), keeping the vertex ids in
//                   LDS (interleaved [slot][lane]). A cycle with at most
//                   kWalkCap vertices that a signature filter finds free of
//                   repeated vertices is complete and is staged unrotated
//                   with the slot of its smallest vertex; the cycles it flags
//                   (every one with a tip or another repeated vertex) are
//                   queued for the tip path, longer ones for the region path.
// k_tip           : 64 flagged short polygons per workgroup of two waves:
//                   walks each cycle again from its start half-edge (one
//                   wave forwards, one backwards, half the cycle each),
//                   stages it if it has no repeated vertex after all, repairs
//                   a single tip, and leaves other cases to the region path.
// k_general_big   : the region path: a breadth-first search gathers the
//                   region into LDS as links between local edges, then
//                   barrier marking, tips, the repair and the pieces run
//                   there in parallel. One wave per region (up to 128
//                   triangles), then 1024 threads per region (up to 4096).
// k_general_small : one lane per declined short polygon when there are many.
// k_general_huge  : regions beyond 4096: the same steps by 1024 threads with
//                   the region in global memory; beyond that store, one lane
//                   per region.
// k_scan_emit     : single-pass decoupled look-back scan of (pieces,
//                   vertices) per polygon in seed order fused with the CSR
//                   write.
#include "common.h"
#include "scan.h"

namespace polylla {

constexpr int kWalkCap = 24;

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
    // label and twin are loaded together: one memory round trip per step
    const uint8_t lab = he[c];
    const int32_t tw = twin[c];
    if (lab & kFrontier) return c;
    if ((uint32_t)tw >= (uint32_t)nhe) {
      set_error(cnt, POLYLLA_ETOPO);
      return -1;
    }
    c = he_next(tw);
  }
  set_error(cnt, POLYLLA_EDEGEN);
  return -1;
}

// Three values of a triangle selected by a local index without indexing a
// register array (which would go to scratch memory).
__device__ __forceinline__ int32_t sel3(int32_t a, int32_t b, int32_t c, int i) {
  return i == 0 ? a : (i == 1 ? b : c);
}

struct alignas(4) Int3 {
  int32_t x, y, z;
};

// The walk array holds one word per half-edge: the twin of an internal
// half-edge, -1 - origin of a frontier one. A walk reads one 12-byte triple
// per triangle it enters: its next step (crossing) or its next vertex.
struct WalkRec {
  int32_t w0, w1, w2;
  __device__ __forceinline__ int32_t w(int i) const { return sel3(w0, w1, w2, i); }
  __device__ __forceinline__ void load(int32_t t, const int32_t* __restrict__ wk) {
    const Int3 a = *reinterpret_cast<const Int3*>(wk + 3 * t);
    w0 = a.x;
    w1 = a.y;
    w2 = a.z;
  }
};

// Twin triple, origin triple and frontier flags (from the walk array) of one
// triangle: three independent loads issued together.
struct TriRec {
  int32_t tw0, tw1, tw2;
  int32_t or0, or1, or2;
  uint32_t fm;  // bit i: half-edge i is a frontier edge
  __device__ __forceinline__ int32_t tw(int i) const { return sel3(tw0, tw1, tw2, i); }
  __device__ __forceinline__ int32_t org(int i) const { return sel3(or0, or1, or2, i); }
  __device__ __forceinline__ bool frontier(int i) const { return (fm >> i) & 1u; }
  __device__ __forceinline__ void load(int32_t t, const int32_t* __restrict__ twin,
                                       const int32_t* __restrict__ origin, const int32_t* __restrict__ wk) {
    const Int3 a = *reinterpret_cast<const Int3*>(twin + 3 * t);
    const Int3 b = *reinterpret_cast<const Int3*>(origin + 3 * t);
    const Int3 c = *reinterpret_cast<const Int3*>(wk + 3 * t);
    fm = (c.x < 0 ? 1u : 0u) | (c.y < 0 ? 2u : 0u) | (c.z < 0 ? 4u : 0u);
    tw0 = a.x;
    tw1 = a.y;
    tw2 = a.z;
    or0 = b.x;
    or1 = b.y;
    or2 = b.z;
  }
};

__device__ __forceinline__ int next_local(int i) { return i == 2 ? 0 : i + 1; }

// Walk states
constexpr int kSimple = 0;    // complete here
constexpr int kSmall = 1;     // short, with a tip or a repeated vertex
constexpr int kInvalid = 2;   // input error (reported)
constexpr int kLarge = 3;     // longer than kWalkCap

// Inclusive sum over the 64 lanes of a wave with DPP row shifts and row
// broadcasts (no LDS round trip); every lane of the wave must be active.
__device__ __forceinline__ uint32_t wave_incl_sum(uint32_t x) {
  const int lane = threadIdx.x & 63, rl = lane & 15;
  uint32_t t;
  t = __builtin_amdgcn_update_dpp(0u, x, 0x111, 0xf, 0xf, false);  // row_shr:1
  if (rl >= 1) x += t;
  t = __builtin_amdgcn_update_dpp(0u, x, 0x112, 0xf, 0xf, false);  // row_shr:2
  if (rl >= 2) x += t;
  t = __builtin_amdgcn_update_dpp(0u, x, 0x114, 0xf, 0xf, false);  // row_shr:4
  if (rl >= 4) x += t;
  t = __builtin_amdgcn_update_dpp(0u, x, 0x118, 0xf, 0xf, false);  // row_shr:8
  if (rl >= 8) x += t;
  t = __builtin_amdgcn_update_dpp(0u, x, 0x142, 0xf, 0xf, false);  // row_bcast:15 (rows 1, 3)
  if ((lane & 31) >= 16) x += t;
  t = __builtin_amdgcn_update_dpp(0u, x, 0x143, 0xf, 0xf, false);  // row_bcast:31 (rows 2, 3)
  if (lane >= 32) x += t;
  return x;
}

// Walk kernel as a persistent state machine: every lane walks one polygon at
// a time and takes the next one as soon as it finishes. The seed range is cut
// into one contiguous part per XCD (workgroups are dispatched to the 8 XCDs
// round-robin), each consumed in chunks of 64 seeds through its own counter,
// so the polygons in flight on an XCD are spatial neighbours that share
// cache lines in that XCD's L2. Each loop iteration advances every busy lane
// until it needs the record of the next triangle and issues that load into a
// second record buffer, so no instruction waits on a load in flight and a
// wave pays one memory round trip per iteration.
constexpr int kXcds = 8;
constexpr int32_t kStageChunk = 4096;  // staging ints a wave reserves at a time
constexpr int kRefill = 8;             // idle lanes of a wave before it hands out polygons

template <bool FROM_SEEDS>
__global__ __launch_bounds__(256) void k_walk(const int32_t* __restrict__ list, int32_t nhe,
                                              const int32_t* __restrict__ wk, int32_t* __restrict__ stage,
                                              int64_t stage_cap, PolyState ps, int32_t* __restrict__ deferred,
                                              int64_t deferred_cap, int walk_cap, Counters* cnt) {
  // (the two emission steps per triangle below rely on seed starts)
  static_assert(FROM_SEEDS, "the walk starts from seed triangles");
  __shared__ int32_t buf[kWalkCap + 1][256];  // vertex ids of the cycle, per lane (+ a spare row)
  walk_cap = walk_cap < 1 ? 1 : (walk_cap > kWalkCap ? kWalkCap : walk_cap);
  const int lane = threadIdx.x & 63;
  // per-wave queue of short polygons with a repeated vertex (see below)
  __shared__ int32_t dq[4][64];
  const int wv_id = threadIdx.x >> 6;
  int dq_n = 0;  // wave-uniform
  auto flush_deferred = [&]() {
    if (dq_n > 0) {
      uint32_t b = 0;
      if (lane == 0) b = atomicAdd(&cnt->n_deferred, (uint32_t)dq_n);
      b = __shfl(b, 0, 64);
      if (lane < dq_n) deferred[b + lane] = dq[wv_id][lane];
      dq_n = 0;
    }
  };
  const int32_t R = (int32_t)cnt->n_seeds;
  const int32_t nt = nhe / 3;
  const int xcd = blockIdx.x % kXcds;
  const int32_t part_lo = (int32_t)((int64_t)R * xcd / kXcds);
  const int32_t part_hi = (int32_t)((int64_t)R * (xcd + 1) / kXcds);
  uint32_t* ticket = &cnt->xcd_ticket[64 * xcd];
  // wave-uniform: current chunk [cbase, cbase + clen), next unused slot cpos;
  // chunk_item: list entry of slot `lane` of the chunk
  int32_t cbase = 0, clen = 0, cpos = 0, chunk_item = 0;
  bool more = true;
  int64_t sbase = 0;  // wave-uniform: free part of the wave's staging chunk
  int32_t sleft = 0;
  // lane state; the cycle's vertices are kept in LDS column buf[.][threadIdx.x]
  int32_t idx = -1;
  int32_t s = -1, t = 0, ci = 0, L = 0, minv = 0, minpos = 0, minhe = -1, steps = 0;
  // repeated-vertex filter: two 64-bit signatures of the vertices so far (bit
  // v & 63 and bit (v ^ v >> 5 ^ v >> 11) & 63). A cycle in which a vertex
  // finds both its bits set already is flagged and goes to the tip path, which
  // checks it exactly: every cycle with a repeated vertex is flagged, and
  // about one in five hundred without one.
  uint64_t sig = 0, sig2 = 0;
  bool complex = false, pending = false, fresh = false, done = false;
  int result = kSimple;
  WalkRec r, rn;
  r.w0 = r.w1 = r.w2 = 0;
  rn = r;
  for (;;) {
    if (pending) {
      r = rn;
      pending = false;
    }
    // ---- idle lanes take the next polygons, in batches of kRefill lanes
    const bool want = idx < 0;
    const uint64_t wmask = __ballot(want);
    const int nwant = __popcll(wmask);
    bool got = false;
    if (more && (nwant >= kRefill || nwant == 64)) {
      const int rank = __popcll(wmask & ((1ull << lane) - 1ull));
      const int32_t take_old = min(clen - cpos, nwant);
      const int32_t src_old = cpos + rank;
      const int32_t item_old = __shfl(chunk_item, src_old & 63, 64);
      if (want && rank < take_old) {
        idx = cbase + src_old;
        got = true;
        t = item_old;
      }
      cpos += take_old;
      if (take_old < nwant) {
        int32_t base = 0;
        if (lane == 0) base = part_lo + 64 * (int32_t)atomicAdd(ticket, 1u);
        base = __shfl(base, 0, 64);
        if (base < part_hi) {
          cbase = base;
          clen = min(64, part_hi - base);
          chunk_item = lane < clen ? list[base + lane] : 0;
          const int32_t src_new = rank - take_old;
          const int32_t item_new = __shfl(chunk_item, src_new & 63, 64);
          if (want && rank >= take_old && src_new < clen) {
            idx = cbase + src_new;
            got = true;
            t = item_new;
          }
          cpos = min(nwant - take_old, clen);
        } else {
          more = false;
          clen = cpos = 0;
        }
      }
      if (got) {
        // new polygon: t holds the list entry (seed triangle or start half-edge)
        fresh = true;
        const int32_t item = t;
        t = FROM_SEEDS ? item : item / 3;
        L = 0;
        steps = 0;
        complex = false;
        done = false;
        sig = 0;
        sig2 = 0;
        minv = 0x7FFFFFFF;
        minpos = 0;
        minhe = -1;
        result = kSimple;
        if ((uint32_t)t < (uint32_t)nt && (FROM_SEEDS || item >= 0)) {
          pending = true;  // (loaded below)
          s = FROM_SEEDS ? -1 : item;  // -1: start not found yet
          ci = FROM_SEEDS ? 0 : item - 3 * t;
        } else {
          result = kInvalid;
          done = true;
        }
      }
    }
    // ---- advance every busy lane up to its next load
    const bool busy = idx >= 0 && !pending && !done;
    if (busy && fresh && FROM_SEEDS) {
      // seed triangle: its first frontier half-edge, else turn about vertex 0
      if (r.w0 < 0) ci = 0;
      else if (r.w1 < 0) ci = 1;
      else if (r.w2 < 0) ci = 2;
      else ci = -1;
      if (r.w0 < 0 && r.w1 < 0 && r.w2 < 0) {
        // a region of one triangle: its three vertices are the whole cycle
        s = 3 * t;
        if (walk_cap < 3) {
          result = kLarge;
        } else {
          const int32_t v0 = -1 - r.w0, v1 = -1 - r.w1, v2 = -1 - r.w2;
          buf[0][threadIdx.x] = v0;
          buf[1][threadIdx.x] = v1;
          buf[2][threadIdx.x] = v2;
          L = 3;
          minpos = v1 < v0 ? (v2 < v1 ? 2 : 1) : (v2 < v0 ? 2 : 0);
          minhe = s + minpos;
          complex = v0 == v1 || v1 == v2 || v0 == v2;  // (not a triangulation)
        }
        done = true;
      } else if (ci < 0) {
        const int32_t tw = r.w0;
        if ((uint32_t)tw >= (uint32_t)nhe) {
          result = kInvalid;
          done = true;
        } else {
          t = tw / 3;
          ci = next_local(tw - 3 * t);
          pending = true;
        }
      } else {
        s = 3 * t + ci;
      }
    }
    if (busy) fresh = false;
    const bool act = busy && !pending && !done;
    {
      // In the triangle just entered, from local index ci: the frontier
      // half-edges that follow one another (their origins are the next
      // vertices of the cycle), then the first internal one, which the lane
      // crosses (turning about the current vertex). Entered across an edge,
      // a triangle has at most two such frontier half-edges before that edge
      // comes round again, and a seed triangle with three (a region of one
      // triangle) was taken whole above, so two steps suffice. Written as
      // selects on per-lane predicates (the vertex store goes to a spare row
      // when the lane emits nothing), so the wave runs it without branches.
      const int p0 = ci, p1 = next_local(p0), p2 = next_local(p1);
      const int32_t wa = r.w(p0), wb = r.w(p1), wc = r.w(p2);
      const int32_t base = t + t + t;
      bool live = act;
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int32_t wv = j == 0 ? wa : wb;
        const int32_t c = base + (j == 0 ? p0 : p1);
        const bool fr = live && wv < 0;
        const bool first = fr && s < 0;  // start found by turning about the seed's vertex 0
        const bool close = fr && !first && L > 0 && c == s;
        const bool over = fr && !close && L == walk_cap;
        const bool emit = fr && !close && !over;
        s = first ? c : s;
        const int32_t v = -1 - wv;
        buf[emit ? L : kWalkCap][threadIdx.x] = v;
        const uint64_t bit = 1ull << (v & 63);
        const uint64_t bit2 = 1ull << ((v ^ (v >> 5) ^ (v >> 11)) & 63);
        complex = complex || (emit && (sig & bit) != 0 && (sig2 & bit2) != 0);
        sig |= emit ? bit : 0ull;
        sig2 |= emit ? bit2 : 0ull;
        const bool lower = emit && v < minv;
        minv = lower ? v : minv;
        minhe = lower ? c : minhe;
        minpos = lower ? L : minpos;
        L += emit ? 1 : 0;
        done = done || close || over;
        result = over ? kLarge : result;
        live = emit;
      }
      // the first internal half-edge, crossed (none after two frontier ones
      // outside a seed triangle: not a triangulation)
      const int32_t wx = wa >= 0 ? wa : (wb >= 0 ? wb : wc);
      const bool stuck = act && !done && wx < 0;
      done = done || stuck;
      result = stuck ? kInvalid : result;
      const bool cr = act && !done && wx >= 0;
      steps += cr ? 1 : 0;
      const bool bad = cr && ((uint32_t)wx >= (uint32_t)nhe || steps > nhe);
      const bool go = cr && !bad;
      const int32_t tn = wx / 3;
      t = go ? tn : t;
      ci = go ? next_local(wx - (tn + tn + tn)) : ci;
      pending = pending || go;
      done = done || bad;
      result = bad ? kInvalid : result;
    }
    // one load site: the record of the triangle every lane that crossed an
    // edge (or took a new polygon) enters next, consumed next iteration
    if (pending) rn.load(t, wk);
    // ---- finished lanes: stage complete cycles (packed per wave, unrotated:
    // the emitter starts each at slot minpos, its smallest vertex), queue the others
    const bool fin = idx >= 0 && done;
    if (fin && result == kSimple && complex) result = kSmall;
    const bool fin_simple = fin && result == kSimple;
    if (fin && result == kSmall) ps.set(idx, L, 0, s, -1);  // the tip path walks it again from s
    if (fin && result == kLarge) ps.set(idx, 0, 0, s, -1);  // (and the long-cycle tip path)
    if (__ballot(fin_simple)) {
      const uint32_t need = fin_simple ? (uint32_t)L : 0u;
      const uint32_t incl = wave_incl_sum(need);
      const int32_t tot = __builtin_amdgcn_readlane((int32_t)incl, 63);
      if (tot > sleft) {  // new staging chunk for this wave
        const int32_t want_ints = max(tot, kStageChunk);
        int64_t nb = 0;
        if (lane == 0) nb = (int64_t)atomicAdd(&cnt->stage_top, (uint32_t)want_ints);
        sbase = __shfl(nb, 0, 64);
        sleft = want_ints;
      }
      const bool fits = sbase + tot <= stage_cap;
      if (fin_simple) {
        const int64_t off = sbase + incl - need;
        if (!fits) {
          set_error(cnt, POLYLLA_ENOMEM);
          ps.clear(idx);
        } else {
          ps.set_stream(idx, L, 1 | (minpos << kRotShift), minhe, (int32_t)off);
        }
      }
      // the staged words of all finished lanes, copied by the whole wave with
      // coalesced stores: word k belongs to the first lane whose inclusive
      // offset exceeds k (binary search over the 64 offsets by lane shuffles).
      // Staged words and records are not read again here: streaming stores,
      // so that they leave the L2 to the walk words first.
      if (fits) {
        const int col0 = threadIdx.x & ~63;
        for (int32_t k0 = 0; k0 < tot; k0 += 64) {
          const int32_t k = k0 + lane;
          int f = 0;
#pragma unroll
          for (int step = 32; step > 0; step >>= 1) {
            const uint32_t v = __shfl(incl, f + step - 1, 64);
            if (v <= (uint32_t)k) f += step;
          }
          const int32_t start = (int32_t)__shfl(incl - need, f, 64);
          if (k < tot) __builtin_nontemporal_store(buf[k - start][col0 + f], &stage[sbase + k]);
        }
      }
      sbase += tot;
      sleft -= tot;
    }
    // Queued polygons. Short ones with a repeated vertex collect in a
    // per-wave LDS queue that goes out 64 at a time with one counter update
    // (one update per polygon on a single counter queues the waves at its L2
    // channel); the rare long ones take one update per wave and event.
    const bool q_small = fin && result == kSmall, q_large = fin && result == kLarge;
    const uint64_t m_small = __ballot(q_small), m_large = __ballot(q_large);
    if (m_small) {
      const int n = __popcll(m_small);
      if (dq_n + n > 64) {
        flush_deferred();
      }
      if (q_small) dq[wv_id][dq_n + __popcll(m_small & ((1ull << lane) - 1ull))] = idx;
      dq_n += n;
    }
    if (m_large) {
      uint32_t b = 0;
      if (lane == 0) b = atomicAdd(&cnt->n_big, (uint32_t)__popcll(m_large));
      b = __shfl(b, 0, 64);
      if (q_large) deferred[deferred_cap - 1 - (b + __popcll(m_large & ((1ull << lane) - 1ull)))] = idx;
    }
    if (fin) {
      if (result == kInvalid) {
        set_error(cnt, steps > nhe ? POLYLLA_EDEGEN : POLYLLA_ETOPO);
        ps.clear(idx);
      }
      idx = -1;
      done = false;
    }
    if (!more && __ballot(idx >= 0) == 0ull) break;
  }
  flush_deferred();
}

// Reparation phase on the polygons of polylla_build (their vertices, start
// half-edges and count in the input CSR): a polygon without a barrier-edge tip
// (no cyclic v[k-1] == v[k+1]) is final as it is (already canonical) and its
// vertices are staged at its input offset; the others are queued, from their
// start half-edges, for the tip path or, longer than the walk cap, for the
// long-region path, so only they are walked again. Queue slots are reserved
// once per wave.
__global__ __launch_bounds__(256) void k_repair_prep(const int32_t* __restrict__ offsets,
                                                     const int32_t* __restrict__ verts,
                                                     const int32_t* __restrict__ start, int32_t* __restrict__ stage,
                                                     int64_t stage_cap, PolyState ps, int32_t* __restrict__ deferred,
                                                     int64_t deferred_cap, int walk_cap, Counters* cnt) {
  const uint32_t R = cnt->n_seeds;
  const int lane = threadIdx.x & 63;
  if (blockIdx.x == 0 && threadIdx.x == 0) cnt->stage_top = (uint32_t)offsets[R];  // the staged copies come first
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i0 = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63); i0 < R; i0 += stride) {
    const int64_t i = i0 + lane;
    const bool valid = i < R;
    int32_t o = 0, L = 0;
    bool tip = false;
    if (valid) {
      o = offsets[i];
      L = offsets[i + 1] - o;
      if (L >= 3)
        for (int32_t k = 0; k < L && !tip; ++k) tip = verts[o + (k == 0 ? L - 1 : k - 1)] == verts[o + (k + 1 == L ? 0 : k + 1)];
      if (!tip) {
        if ((int64_t)o + L > stage_cap) {
          set_error(cnt, POLYLLA_ENOMEM);
          ps.clear(i);
        } else {
          for (int32_t k = 0; k < L; ++k) stage[o + k] = verts[o + k];
          ps.set(i, L, 1, start[i], o);
        }
      } else {
        ps.set(i, L, 0, start[i], -1);
      }
    }
    const bool q_small = tip && L <= walk_cap, q_large = tip && L > walk_cap;
    const uint64_t m_small = __ballot(q_small), m_large = __ballot(q_large);
    uint32_t b_small = 0, b_large = 0;
    if (lane == 0) {
      if (m_small) b_small = atomicAdd(&cnt->n_deferred, (uint32_t)__popcll(m_small));
      if (m_large) b_large = atomicAdd(&cnt->n_big, (uint32_t)__popcll(m_large));
    }
    b_small = __shfl(b_small, 0, 64);
    b_large = __shfl(b_large, 0, 64);
    const uint64_t below = (1ull << lane) - 1ull;
    if (q_small) deferred[b_small + __popcll(m_small & below)] = (int32_t)i;
    if (q_large) deferred[deferred_cap - 1 - (b_large + __popcll(m_large & below))] = (int32_t)i;
  }
}

// ---------------------------------------------------------------------------
// general path

// Arrays of the per-lane general path: a plain pointer (global arena) or a
// column of an LDS array interleaved over the 64 lanes of a block.
struct GPtr {
  int32_t* p;
  __device__ __forceinline__ int32_t& operator[](int32_t k) const { return p[k]; }
};
struct LdsCol {
  int32_t* p;
  __device__ __forceinline__ int32_t& operator[](int32_t k) const { return p[k * 64]; }
};

template <typename A>
__device__ void heap_sort(A a, int32_t n) {
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
template <typename A>
__device__ __forceinline__ int32_t bsearch_idx(A a, int32_t n, int32_t x) {
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

// The whole general path for one polygon (index i in seed order, start
// half-edge s), by one thread with its data in the global arena. Used for
// short polygons with a tip or a repeated vertex, and for polygons too large
// for the cooperative kernel.
template <bool REPAIR, typename A>
__device__ void general_core(int32_t i, int32_t s, int32_t L, A cyc, A aux, int32_t nhe, int64_t nv,
                             const int32_t* __restrict__ twin, const int32_t* __restrict__ origin,
                             uint8_t* __restrict__ he, uint8_t* __restrict__ vtx, int32_t* __restrict__ stage,
                             int64_t stage_cap, int32_t* __restrict__ arena, int64_t arena_cap, PolyState ps,
                             Counters* cnt) {
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
      or_bits(he, e, kBarrier);
      if ((uint32_t)te < (uint32_t)nhe) or_bits(he, te, kBarrier);
    }
  }
  // tips: the next frontier half-edge is the twin of the current one
  int32_t ntip = 0;
  for (int32_t k = 0; k < L; ++k) {
    int32_t h = cyc[k], hn = cyc[k + 1 == L ? 0 : k + 1];
    if (twin[h] == hn) {
      int32_t v = origin[hn];
      if ((uint64_t)(uint32_t)v < (uint64_t)nv) or_bits(vtx, v, kTip);
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
      he[e] |= kFrontier | kRepaired;  // read back by the piece walk below
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
      return;
    }
    for (int32_t k = 0; k < L; ++k) stage[off + k] = origin[cyc[(best + k) % L]];
    ps.set(i, L, 1, cyc[best], (int32_t)off);
    return;
  }
  // pieces: walk from the opened half-edges, each piece once
  const int32_t nc = 2 * nsplit;
  A cand = cyc;  // the recorded cycle is no longer needed
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
    return;
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
    return;
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
    return;
  }
  int32_t w = (int32_t)off;
  for (int32_t q = 0; q < np; ++q) {
    int32_t h = rec[4 * q + 2];
    for (int32_t k = 0; k < rec[4 * q + 3] && h >= 0; ++k) {
      stage[w++] = origin[h];
      h = walk_next(h, nhe, twin, he, cnt);
    }
  }
  ps.set(i, total, np, -1, (int32_t)off);
  ps.prec[i] = (int32_t)r0;

}

template <bool REPAIR>
__device__ void general_one(int32_t i, int32_t s, int32_t nhe, int64_t nv, const int32_t* __restrict__ twin,
                            const int32_t* __restrict__ origin, uint8_t* __restrict__ he, uint8_t* __restrict__ vtx,
                            int32_t* __restrict__ stage, int64_t stage_cap, int32_t* __restrict__ arena,
                            int64_t arena_cap, PolyState ps, Counters* cnt) {
  ps.clear(i);
  if ((uint32_t)s >= (uint32_t)nhe) return;
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
      return;
    }
  }
  const uint32_t need = 2u * (uint32_t)L;
  const uint32_t a0 = atomicAdd(&cnt->arena_top, need);
  if ((int64_t)a0 + need > arena_cap) {
    set_error(cnt, POLYLLA_ENOMEM);
    return;
  }
  int32_t* cyc = arena + a0;
  int32_t* aux = cyc + L;
  general_core<REPAIR>(i, s, L, GPtr{cyc}, GPtr{aux}, nhe, nv, twin, origin, he, vtx, stage, stage_cap, arena,
                       arena_cap, ps, cnt);
}

// ---------------------------------------------------------------------------
// Per-lane region path for short polygons with a tip or a repeated vertex.
//
// Every step of the general path stays inside the polygon's region: turning
// about a vertex from one frontier half-edge to the next crosses internal
// edges only, and the whole fan of a barrier-edge tip lies in the region. So
// the lane first gathers the region's triangles (breadth-first over internal
// edges, all triangles of a level loaded together), keeping per triangle its
// id, its three vertex ids and one link per local edge:
//   internal edge : code of the twin in the region (slot * 4 + local index)
//   frontier edge : -2 - twin half-edge id, or -1 on the hull
// and then runs the cycle, barrier, tip, repair and piece steps on these LDS
// arrays. A region of a cycle with at most kWalkCap frontier half-edges has at
// most kWalkCap - 2 triangles (3k half-edges = L frontier + 2(k - 1) internal).

constexpr int kSmallK = kWalkCap - 2;
constexpr int32_t kUnset = INT32_MIN;
constexpr int kGather = 4;  // triangle records a lane loads per round

template <typename A>
struct Region {
  A tri, lnk, org;
  __device__ __forceinline__ int32_t gid(int c) const { return 3 * tri[c >> 2] + (c & 3); }
  __device__ __forceinline__ int32_t link(int c) const { return lnk[(c >> 2) * 3 + (c & 3)]; }
  __device__ __forceinline__ void set_link(int c, int32_t v) const { lnk[(c >> 2) * 3 + (c & 3)] = v; }
  __device__ __forceinline__ int32_t vert(int c) const { return org[(c >> 2) * 3 + (c & 3)]; }
  __device__ __forceinline__ int32_t twin_gid(int c) const {
    const int32_t l = link(c);
    return l >= 0 ? gid(l) : (l == -1 ? -1 : -2 - l);
  }
  // code of the edge after crossing internal code c: next local edge of its twin
  __device__ __forceinline__ int turn(int c) const {
    const int32_t l = link(c);
    return (l & ~3) | next_local(l & 3);
  }
  // next frontier code after frontier code c, turning about its end vertex; -1 if none within limit
  __device__ __forceinline__ int next_frontier(int c, int limit) const {
    int x = (c & ~3) | next_local(c & 3);
    for (int n = 0; n < limit; ++n) {
      if (link(x) < 0) return x;
      x = turn(x);
    }
    return -1;
  }
};

// Gather the region of triangle t0 into R. Returns its triangle count, or
// -1 if it has more than kcap triangles, -2 on an invalid mesh.
template <typename A>
__device__ int gather_region(const Region<A>& R, int32_t t0, int kcap, int32_t nhe, const int32_t* __restrict__ twin,
                             const int32_t* __restrict__ origin, const int32_t* __restrict__ wk) {
  R.tri[0] = t0;
  R.lnk[0] = R.lnk[1] = R.lnk[2] = kUnset;
  int head = 0, tail = 1, status = 0;
  while (head < tail && status == 0) {
    const int n = min(tail - head, kGather);
    TriRec rr[kGather];
#pragma unroll
    for (int u = 0; u < kGather; ++u)
      if (u < n) rr[u].load(R.tri[head + u], twin, origin, wk);
#pragma unroll
    for (int u = 0; u < kGather; ++u) {
      if (u >= n) continue;
      const int s = head + u;
#pragma unroll
      for (int e = 0; e < 3; ++e) {
        R.org[3 * s + e] = rr[u].org(e);
        if (R.lnk[3 * s + e] != kUnset) continue;  // the edge it was entered through
        const int32_t tw = rr[u].tw(e);
        if (rr[u].frontier(e)) {
          R.lnk[3 * s + e] = tw < 0 ? -1 : -2 - tw;
        } else if ((uint32_t)tw >= (uint32_t)nhe) {
          R.lnk[3 * s + e] = -1;
          status = -2;
        } else if (tail >= kcap) {
          R.lnk[3 * s + e] = -1;
          status = status ? status : -1;
        } else {
          const int ns = tail++;
          const int32_t t2 = tw / 3, e2 = tw - 3 * t2;
          R.tri[ns] = t2;
          R.lnk[3 * ns] = R.lnk[3 * ns + 1] = R.lnk[3 * ns + 2] = kUnset;
          R.lnk[3 * ns + e2] = 4 * s + e;
          R.lnk[3 * s + e] = 4 * ns + e2;
        }
      }
    }
    head += n;
  }
  return status ? status : tail;
}

// Lexicographic comparison of the vertex sequences of length len from
// frontier codes p and q of the same piece: -1, 0 or 1.
template <typename A>
__device__ int compare_rotations_lds(const Region<A>& R, int p, int q, int32_t len, int limit) {
  for (int32_t k = 0; k < len; ++k) {
    const int32_t a = R.vert(p), b = R.vert(q);
    if (a != b) return a < b ? -1 : 1;
    p = R.next_frontier(p, limit);
    q = R.next_frontier(q, limit);
    if (p < 0 || q < 0) return 0;
  }
  return 0;
}

// The general path for one polygon on its gathered region (k triangles);
// same steps and tie rules as general_core. cyc and aux hold kWalkCap ints.
template <bool REPAIR, typename A>
__device__ void region_core(int32_t i, const Region<A>& R, int k, int start, A cyc, A aux, int64_t nv,
                            uint8_t* __restrict__ he, uint8_t* __restrict__ vtx, int32_t* __restrict__ stage,
                            int64_t stage_cap, int32_t* __restrict__ arena, int64_t arena_cap, PolyState ps,
                            Counters* cnt) {
  const int limit = 3 * k + 3;
  // the cycle
  int32_t L = 0;
  {
    int c = start;
    do {
      if (L == kWalkCap) {
        set_error(cnt, POLYLLA_EINTERNAL);  // k <= kWalkCap - 2 bounds the cycle
        return;
      }
      cyc[L++] = c;
      c = R.next_frontier(c, limit);
    } while (c >= 0 && c != start);
    if (c != start) {
      set_error(cnt, POLYLLA_EDEGEN);
      return;
    }
  }
  // barrier edges: edge keys that occur twice on the cycle
  for (int32_t m = 0; m < L; ++m) {
    const int32_t h = R.gid(cyc[m]), tw = R.twin_gid(cyc[m]);
    aux[m] = tw < 0 ? -1 : (h < tw ? h : tw);
  }
  heap_sort(aux, L);
  for (int32_t m = 0; m < L; ++m) {
    const int32_t h = R.gid(cyc[m]), tw = R.twin_gid(cyc[m]);
    if (tw < 0) continue;
    const int32_t key = h < tw ? h : tw;
    const int32_t at = bsearch_idx(aux, L, key);
    if (at >= 0 && at + 1 < L && aux[at + 1] == key) or_bits(he, h, kBarrier);
  }
  // tips: the next frontier half-edge is the twin of the current one; the
  // pair keeps the tip vertex and the cycle position of that next half-edge
  int32_t ntip = 0;
  for (int32_t m = 0; m < L; ++m) {
    const int mn = m + 1 == L ? 0 : m + 1;
    if (R.twin_gid(cyc[m]) == R.gid(cyc[mn])) {
      const int32_t v = R.vert(cyc[mn]);
      if ((uint64_t)(uint32_t)v < (uint64_t)nv) or_bits(vtx, v, kTip);
      aux[2 * ntip] = v;
      aux[2 * ntip + 1] = mn;
      ++ntip;
    }
  }
  if (ntip) atomicAdd(&cnt->n_tips, (uint32_t)ntip);
  int32_t nsplit = 0;
  uint64_t opened[2] = {0ull, 0ull};  // codes of opened half-edges (code < 128)
  if (REPAIR && ntip) {
    // middle internal edge at every tip: c_{floor(d/2)} turning about the tip
    // vertex from its barrier half-edge c0 (whose twin is the previous cycle edge)
    for (int32_t q = 0; q < ntip; ++q) {
      const int32_t mn = aux[2 * q + 1];
      const int c0 = cyc[mn], tw0 = cyc[mn == 0 ? L - 1 : mn - 1];
      int32_t d = 0;
      int c = c0;
      do {
        const int tc = c == c0 ? tw0 : R.link(c);
        if (tc < 0) {
          d = -1;
          break;
        }
        c = (tc & ~3) | next_local(tc & 3);
        ++d;
      } while (c != c0 && d <= limit);
      if (d < 0 || c != c0) {
        set_error(cnt, POLYLLA_ETOPO);
        d = 0;
      }
      int e = c0;
      for (int32_t m = 0; m < d / 2; ++m) {
        const int tc = e == c0 ? tw0 : R.link(e);
        e = (tc & ~3) | next_local(tc & 3);
      }
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
        const int e = aux[2 * p + 1];
        dead = R.vert((e & ~3) | next_local(e & 3)) == v;
      }
      if (dead) aux[2 * q] = -1 - v;
    }
    // open the edges of the live tips; both half-edge codes go to cyc, which
    // is not needed any more once an edge is opened
    for (int32_t q = 0; q < ntip; ++q) {
      if (aux[2 * q] < 0) continue;
      const int e = aux[2 * q + 1];
      const int32_t te = R.link(e);
      if (te < 0) {  // only reachable on an invalid mesh
        set_error(cnt, POLYLLA_ETOPO);
        aux[2 * q] = -1 - aux[2 * q];
        continue;
      }
      const int32_t ge = R.gid(e), gt = R.gid(te);
      or_bits(he, ge, kFrontier | kRepaired);
      or_bits(he, gt, kFrontier | kRepaired);
      R.set_link(e, -2 - gt);
      R.set_link(te, -2 - ge);
      opened[e >> 6] |= 1ull << (e & 63);
      opened[te >> 6] |= 1ull << (te & 63);
      cyc[2 * nsplit] = e;
      cyc[2 * nsplit + 1] = te;
      ++nsplit;
    }
    if (nsplit) atomicAdd(&cnt->n_splits, (uint32_t)nsplit);
  }
  if (nsplit == 0) {
    // one piece: the cycle itself, rotated to its smallest vertex sequence
    int32_t best = 0, minv = R.vert(cyc[0]);
    for (int32_t m = 1; m < L; ++m) {
      const int32_t v = R.vert(cyc[m]);
      if (v < minv) {
        minv = v;
        best = m;
      }
    }
    for (int32_t m = best + 1; m < L; ++m) {
      if (R.vert(cyc[m]) != minv) continue;
      for (int32_t z = 1; z < L; ++z) {
        const int32_t a = R.vert(cyc[(m + z) % L]), b = R.vert(cyc[(best + z) % L]);
        if (a != b) {
          if (a < b) best = m;
          break;
        }
      }
    }
    const uint32_t off = atomicAdd(&cnt->stage_top, (uint32_t)L);
    if ((int64_t)off + L > stage_cap) {
      set_error(cnt, POLYLLA_ENOMEM);
      return;
    }
    for (int32_t m = 0; m < L; ++m) stage[off + m] = R.vert(cyc[(best + m) % L]);
    ps.set(i, L, 1, R.gid(cyc[best]), (int32_t)off);
    return;
  }
  // pieces: walk from the opened half-edges in increasing half-edge id, each
  // piece once
  const int32_t nc = 2 * nsplit;
  A cand = cyc;
  for (int32_t q = 1; q < nc; ++q) {
    const int32_t x = cand[q], gx = R.gid(x);
    int32_t p = q;
    while (p > 0 && R.gid(cand[p - 1]) > gx) {
      cand[p] = cand[p - 1];
      --p;
    }
    cand[p] = x;
  }
  const int32_t npieces = nsplit + 1;
  const uint32_t rneed = (uint32_t)(4 * npieces);
  const uint32_t r0 = atomicAdd(&cnt->arena_top, rneed);
  if ((int64_t)r0 + rneed > arena_cap) {
    set_error(cnt, POLYLLA_ENOMEM);
    return;
  }
  int32_t* rec = arena + r0;
  uint32_t seen = 0;
  int32_t np = 0, total = 0;
  bool bad = false;
  for (int32_t m = 0; m < nc && !bad; ++m) {
    if ((seen >> m) & 1u) continue;
    const int x = cand[m];
    int h = x;
    int32_t len = 0, minv = 0x7FFFFFFF, mincount = 0;
    int minh = -1;
    do {
      const int32_t v = R.vert(h);
      if (v < minv) {
        minv = v;
        minh = h;
        mincount = 1;
      } else if (v == minv) {
        ++mincount;
      }
      if ((opened[h >> 6] >> (h & 63)) & 1ull)
        for (int32_t z = 0; z < nc; ++z)
          if (cand[z] == h) seen |= 1u << z;
      ++len;
      h = R.next_frontier(h, limit);
    } while (h >= 0 && h != x && len <= limit);
    if (h != x || np >= npieces) {
      set_error(cnt, POLYLLA_EDEGEN);
      bad = true;
      break;
    }
    if (mincount > 1) {
      // pinched piece: lexicographically smallest rotation among the
      // occurrences of its smallest vertex
      int best = minh, q = R.next_frontier(minh, limit);
      for (int32_t z = 1; z < len && q >= 0; ++z) {
        if (R.vert(q) == minv && compare_rotations_lds(R, q, best, len, limit) < 0) best = q;
        q = R.next_frontier(q, limit);
      }
      minh = best;
    }
    const int nxt = R.next_frontier(minh, limit);
    rec[4 * np] = minv;
    rec[4 * np + 1] = nxt >= 0 ? R.vert(nxt) : 0;
    rec[4 * np + 2] = R.gid(minh);
    rec[4 * np + 3] = len;
    aux[np] = minh;  // start code of the piece, for staging its vertices
    ++np;
    total += len;
  }
  if (bad || np != npieces) {
    if (!bad) set_error(cnt, POLYLLA_EDEGEN);
    return;
  }
  // pieces by (first, second) vertex
  for (int32_t q = 1; q < np; ++q) {
    int32_t r[4] = {rec[4 * q], rec[4 * q + 1], rec[4 * q + 2], rec[4 * q + 3]};
    const int32_t sc = aux[q];
    int32_t p = q;
    while (p > 0 && (rec[4 * (p - 1)] > r[0] || (rec[4 * (p - 1)] == r[0] && rec[4 * (p - 1) + 1] > r[1]))) {
      for (int z = 0; z < 4; ++z) rec[4 * p + z] = rec[4 * (p - 1) + z];
      aux[p] = aux[p - 1];
      --p;
    }
    for (int z = 0; z < 4; ++z) rec[4 * p + z] = r[z];
    aux[p] = sc;
  }
  const uint32_t off = atomicAdd(&cnt->stage_top, (uint32_t)total);
  if ((int64_t)off + total > stage_cap) {
    set_error(cnt, POLYLLA_ENOMEM);
    return;
  }
  int32_t w = (int32_t)off;
  for (int32_t q = 0; q < np; ++q) {
    int h = aux[q];
    const int32_t len = rec[4 * q + 3];
    for (int32_t z = 0; z < len && h >= 0; ++z) {
      stage[w++] = R.vert(h);
      h = R.next_frontier(h, limit);
    }
  }
  ps.set(i, total, np, -1, (int32_t)off);
  ps.prec[i] = (int32_t)r0;
}

// ---------------------------------------------------------------------------
// Tip path: the common case of a short polygon with a repeated vertex, one
// barrier-edge tip, repaired from its cycle alone.
//
// The walk staged the cycle (vertices v and half-edges h, v[k] = origin of
// h[k]). A tip is a position m with v[m-1] = v[m+1] (the next frontier
// half-edge is the twin: the only edge joining two vertices). With exactly one
// tip, Algorithm 4 opens the middle internal edge e of its fan (found by
// turning about v[m] through the mesh, a few dependent loads), from v[m] to
// x. If x occurs once on the cycle, at q, the two pieces are the cycle from m
// to q closed by twin(e) and the cycle from q to m closed by e: their
// vertices are contiguous stretches of the staged cycle. Barrier edges are
// the pairs (a, b), (b, a) of consecutive vertices both on the cycle. Every
// other polygon (several tips, x repeated, a cycle not staged) is queued for
// the region path.
// vertex k of a piece: the stretch of `len` cycle positions from `a`
__device__ __forceinline__ int32_t piece_vertex(const LdsCol& v, int L, int a, int k) {
  const int p = a + k;
  return v[p >= L ? p - L : p];
}

// start (0..len-1) of the lexicographically smallest rotation of a piece
__device__ int piece_rotation(const LdsCol& v, int L, int a, int len) {
  int best = 0;
  int32_t mv = piece_vertex(v, L, a, 0);
  for (int k = 1; k < len; ++k) {
    const int32_t x = piece_vertex(v, L, a, k);
    if (x < mv) {
      mv = x;
      best = k;
    }
  }
  for (int k = best + 1; k < len; ++k) {
    if (piece_vertex(v, L, a, k) != mv) continue;
    for (int z = 1; z < len; ++z) {
      const int32_t p = piece_vertex(v, L, a, (k + z) % len), q = piece_vertex(v, L, a, (best + z) % len);
      if (p != q) {
        if (p < q) best = k;
        break;
      }
    }
  }
  return best;
}

// The rest of the tip path for one queued polygon whose cycle (vertices v,
// half-edges h) is in the lane's LDS columns; called by a whole wave (the
// space reservations are wave-wide).
template <bool REPAIR>
__device__ void tip_rest(bool ok, bool valid, int32_t i, int L, int32_t nhe, int64_t nv,
                         const int32_t* __restrict__ twin, const int32_t* __restrict__ origin,
                         uint8_t* __restrict__ he, uint8_t* __restrict__ vtx, int32_t* __restrict__ stage,
                         int64_t stage_cap, int32_t* __restrict__ arena, int64_t arena_cap, PolyState ps,
                         int32_t* __restrict__ rest, int64_t rest_cap, uint32_t* rest_count, const LdsCol& v,
                         const LdsCol& h, const LdsCol& f, uint32_t& n_rep, Counters* cnt) {
  const int lane = threadIdx.x & 63;
  int pairs = 0;
  if (ok)
    for (int a = 0; a < L; ++a)
      for (int b = a + 1; b < L; ++b) pairs += v[a] == v[b] ? 1 : 0;
  // no repeated vertex after all (the walk's filter flags a few such
  // cycles): a complete polygon, staged like the walk stages one
  const bool simple = ok && pairs == 0;
  bool fast = ok && !simple && REPAIR && L >= 4;
  int m = -1;
  if (fast) {
    int ntip = 0;
    for (int k = 0; k < L; ++k) {
      const int32_t vp = v[k == 0 ? L - 1 : k - 1], vn = v[k + 1 == L ? 0 : k + 1];
      if (vp == vn) {
        ++ntip;
        m = k;
      }
    }
    fast = ntip == 1;
    if (fast) {
      // The cycle may repeat vertices only along the slit ending at the tip
      // (v[m-k-1] == v[m+k+1], k < K): then the slit's K edges are all its
      // barrier edges. Any other repeated vertex (a lobe hanging off a
      // barrier edge, a region touching itself) goes to the region path.
      int K = 0;
      while (2 * K + 2 < L && v[(m - K - 1 + L) % L] == v[(m + K + 1) % L]) ++K;
      fast = pairs == K;
    }
  }
  int32_t e = -1, te = -1, x = -1;
  int q = -1;
  if (fast) {
    // middle internal edge c_{floor(d/2)} turning clockwise about v[m] from
    // c0 = h[m] (c_{j+1} = next(twin(c_j))): twin(c0) is h[m-1], so c1 is
    // next(h[m-1]), and the d - 1 internal edges of the fan are the ones the
    // walk crossed about v[m] (f[m])
    const int32_t d = f[m] + 1;
    fast = d >= 2;
    if (fast) {
      e = he_next(h[m == 0 ? L - 1 : m - 1]);
      for (int32_t k = 1; k < d / 2; ++k) {
        const int32_t tw = twin[e];
        if ((uint32_t)tw >= (uint32_t)nhe) {
          fast = false;
          break;
        }
        e = he_next(tw);
      }
    }
    if (fast) {
      te = twin[e];
      x = origin[he_next(e)];
      int occ = 0;
      for (int k = 0; k < L; ++k)
        if (v[k] == x) {
          ++occ;
          q = k;
        }
      fast = occ == 1 && q != m && (uint32_t)te < (uint32_t)nhe;
    }
  }
  // space for the whole wave: staging words, arena words, declined entries
  const bool declined = valid && !simple && !fast;
  const uint32_t ns = simple ? (uint32_t)L : (fast ? (uint32_t)(L + 2) : 0u);
  const uint32_t na = fast ? 8u : 0u;
  const uint32_t is = wave_incl_sum(ns), ia = wave_incl_sum(na);
  const uint64_t md = __ballot(declined);
  const uint32_t ts = (uint32_t)__builtin_amdgcn_readlane((int32_t)is, 63);
  const uint32_t ta = (uint32_t)__builtin_amdgcn_readlane((int32_t)ia, 63);
  uint32_t bs = 0, ba = 0, bd = 0;
  if (lane == 0) {
    if (ts) bs = atomicAdd(&cnt->stage_top, ts);
    if (ta) ba = atomicAdd(&cnt->arena_top, ta);
    if (md) bd = atomicAdd(rest_count, (uint32_t)__popcll(md));
  }
  bs = __shfl(bs, 0, 64);
  ba = __shfl(ba, 0, 64);
  bd = __shfl(bd, 0, 64);
  const int64_t off = (int64_t)bs + is - ns, r0 = (int64_t)ba + ia - na;
  if (declined) {
    const uint32_t r = bd + (uint32_t)__popcll(md & ((1ull << lane) - 1ull));
    if ((int64_t)r < rest_cap) rest[r] = i;
    else set_error(cnt, POLYLLA_EINTERNAL);
  }
  if ((simple || fast) && (off + ns > stage_cap || r0 + na > arena_cap)) {
    set_error(cnt, POLYLLA_ENOMEM);
    ps.clear(i);
    return;
  }
  if (simple) {
    int mp = 0;
    for (int k = 1; k < L; ++k)
      if (v[k] < v[mp]) mp = k;
    for (int k = 0; k < L; ++k) stage[off + k] = v[k];
    ps.set(i, L, 1 | (mp << kRotShift), h[mp], (int32_t)off);
  }
  if (!fast) return;
  // labels: barrier edges, the tip, the opened edge. The barrier edges of a
  // region form a forest inside it whose leaves are tips, so with one tip
  // they are the path v[m-k-1] = v[m+k+1] read outwards from the tip.
  for (int k = 0; 2 * k + 2 < L; ++k) {
    const int lo = (m - k - 1 + L) % L, hi = (m + k + 1) % L;
    if (v[lo] != v[hi]) break;
    or_bits(he, h[lo], kBarrier);             // v[lo] -> v[lo + 1]
    or_bits(he, h[(m + k) % L], kBarrier);    // v[m + k] -> v[hi]
  }
  const int32_t vt = v[m];
  if ((uint64_t)(uint32_t)vt < (uint64_t)nv) or_bits(vtx, vt, kTip);
  or_bits(he, e, kFrontier | kRepaired);
  or_bits(he, te, kFrontier | kRepaired);
  ++n_rep;
  // pieces: A = positions m..q (x last, leaving by te), B = q..m (v[m] last, leaving by e)
  const int lenA = (q - m + L) % L + 1, lenB = (m - q + L) % L + 1;
  const int ra = piece_rotation(v, L, m, lenA), rb = piece_rotation(v, L, q, lenB);
  const int32_t a0 = piece_vertex(v, L, m, ra), a1 = piece_vertex(v, L, m, (ra + 1) % lenA);
  const int32_t b0 = piece_vertex(v, L, q, rb), b1 = piece_vertex(v, L, q, (rb + 1) % lenB);
  const int32_t sa = ra == lenA - 1 ? te : h[(m + ra) % L];
  const int32_t sb = rb == lenB - 1 ? e : h[(q + rb) % L];
  const bool a_first = a0 < b0 || (a0 == b0 && a1 < b1);
  const int oa = a_first ? 0 : lenB, ob = a_first ? lenA : 0;
  for (int k = 0; k < lenA; ++k) stage[off + oa + k] = piece_vertex(v, L, m, (ra + k) % lenA);
  for (int k = 0; k < lenB; ++k) stage[off + ob + k] = piece_vertex(v, L, q, (rb + k) % lenB);
  const int pa = a_first ? 0 : 1, pb = 1 - pa;
  arena[r0 + 4 * pa] = a0;
  arena[r0 + 4 * pa + 1] = a1;
  arena[r0 + 4 * pa + 2] = sa;
  arena[r0 + 4 * pa + 3] = lenA;
  arena[r0 + 4 * pb] = b0;
  arena[r0 + 4 * pb + 1] = b1;
  arena[r0 + 4 * pb + 2] = sb;
  arena[r0 + 4 * pb + 3] = lenB;
  ps.set(i, L + 2, 2, -1, (int32_t)off);
  ps.prec[i] = (int32_t)r0;
}

template <bool REPAIR>
__global__ __launch_bounds__(128) void k_tip(int32_t nhe, int64_t nv, const int32_t* __restrict__ twin,
                                            const int32_t* __restrict__ origin, const int32_t* __restrict__ wk,
                                            uint8_t* __restrict__ he,
                                            uint8_t* __restrict__ vtx, int32_t* __restrict__ stage,
                                            int64_t stage_cap, int32_t* __restrict__ arena, int64_t arena_cap,
                                            PolyState ps, const int32_t* __restrict__ deferred,
                                            int32_t* __restrict__ rest, int64_t rest_cap, Counters* cnt) {
  __shared__ int32_t s_v[kWalkCap * 64];
  __shared__ int32_t s_h[kWalkCap * 64];
  __shared__ int32_t s_f[kWalkCap * 64];
  __shared__ uint8_t s_bok[64];
  // Two waves per 64 queued polygons: wave 0 walks each cycle forwards from
  // its start half-edge over its first half, wave 1 backwards from the start
  // over its second half (turning the other way about each vertex: the
  // previous frontier half-edge is the first frontier one met going to
  // prev(h) and across internal edges), so the chain of dependent loads is
  // half as long. Both count the internal edges crossed about each vertex
  // (f[k]: about v[k], between h[k-1] and h[k]). Wave 0 also takes the step
  // into the second half and checks that it meets wave 1 there, then does
  // the rest alone.
  const int lane = threadIdx.x & 63;
  const bool back = threadIdx.x >= 64;
  const LdsCol v{s_v + lane}, h{s_h + lane}, f{s_f + lane};
  const uint32_t nd = cnt->n_deferred;
  uint32_t n_rep = 0;  // tips repaired by this lane
  // the block takes 64 queued polygons at a time (the loop is block-uniform,
  // and wave 0 reserves the staging, arena and queue space of all 64 with one
  // counter update each)
  for (uint32_t j0 = blockIdx.x * 64; j0 < nd; j0 += gridDim.x * 64) {
    const uint32_t j = j0 + lane;
    const bool valid = j < nd;
    const int32_t i = valid ? deferred[j] : 0;
    const int4 rc = valid ? ps.rec[i] : make_int4(0, 0, -1, 0);
    const int L = rc.x;
    bool ok = valid && rc.y == 0 && L >= 3 && L <= kWalkCap && (uint32_t)rc.z < (uint32_t)nhe;
    const int half = (L + 1) >> 1;  // wave 0: positions [0, half); wave 1: [half, L)
    int32_t hm = -1;                 // wave 0: its half-edge at position half
    if (ok && !back) {
      // the first half again over the walk words (which the repair does not
      // change): frontier half-edges and their vertices
      const int32_t s0 = rc.z;
      int32_t c = s0, w = wk[s0];
      int k = 0;
      while (ok) {
        if (w >= 0) {
          ok = false;
          break;
        }
        if (k == half) {
          hm = c;
          break;
        }
        v[k] = -1 - w;
        h[k] = c;
        ++k;
        // next frontier half-edge: turn about the vertex across internal edges
        int32_t x = he_next(c), steps = 0;
        for (;;) {
          w = wk[x];
          if (w < 0) break;
          if ((uint32_t)w >= (uint32_t)nhe || ++steps > kWalkCap * 3) {
            ok = false;
            break;
          }
          x = he_next(w);
        }
        f[k] = steps;
        c = x;
        if (c == s0) ok = false;  // closed too early
      }
    }
    if (ok && back) {
      const int32_t s0 = rc.z;
      int32_t c = s0;
      for (int k = L - 1; ok && k >= half; --k) {
        // previous frontier half-edge: turn the other way about the origin of c
        int32_t x = he_next(he_next(c)), steps = 0, w;
        for (;;) {
          w = wk[x];
          if (w < 0) break;
          if ((uint32_t)w >= (uint32_t)nhe || ++steps > kWalkCap * 3) {
            ok = false;
            break;
          }
          x = he_next(he_next(w));
        }
        f[k + 1 == L ? 0 : k + 1] = steps;
        c = x;
        if (c == s0) ok = false;  // closed too early
        v[k] = -1 - w;
        h[k] = c;
      }
    }
    if (back) s_bok[lane] = ok ? 1 : 0;
    __syncthreads();
    if (!back) {
      // the halves meet
      ok = ok && s_bok[lane] != 0 && hm == h[half];
      tip_rest<REPAIR>(ok, valid, i, L, nhe, nv, twin, origin, he, vtx, stage, stage_cap, arena, arena_cap, ps,
                       rest, rest_cap, &cnt->n_gen, v, h, f, n_rep, cnt);
    }
    __syncthreads();  // (the columns are reused)
  }
  // repair counts: one update per wave
  const uint32_t tot = (uint32_t)__builtin_amdgcn_readlane((int32_t)wave_incl_sum(n_rep), 63);
  if (lane == 0 && tot) {
    atomicAdd(&cnt->n_tips, tot);
    atomicAdd(&cnt->n_splits, tot);
  }
}

// Long-cycle tip path: the cycles the walk gave up on (longer than its cap,
// listed from the back of `in`), one lane each, 64 per wave, walked again
// from their start half-edges up to kLongCap frontier half-edges. A cycle
// that closes within that is finished as the tip path finishes a short one
// (staged, or repaired at its one tip); the others (longer, several tips,
// other repeated vertices) are listed in `rest` for the region kernels. With
// at most few_max such cycles in all it does nothing: the 1024-thread region
// kernel then takes them all from the walk's list. With at most pass_max it
// only copies the list to `rest`: the one-wave region kernel then gives every
// cycle a wave of its own at once, which is sooner than this path's walk of
// up to kLongCap dependent steps; it pays when cycles queue for those waves.
constexpr int kLongCap = 32;
template <bool REPAIR>
__global__ __launch_bounds__(64) void k_tip_long(int32_t nhe, int64_t nv, const int32_t* __restrict__ twin,
                                                 const int32_t* __restrict__ origin, const int32_t* __restrict__ wk,
                                                 uint8_t* __restrict__ he, uint8_t* __restrict__ vtx,
                                                 int32_t* __restrict__ stage, int64_t stage_cap,
                                                 int32_t* __restrict__ arena, int64_t arena_cap, PolyState ps,
                                                 const int32_t* __restrict__ in, int64_t in_cap,
                                                 const uint32_t* in_count, uint32_t few_max, uint32_t pass_max,
                                                 int32_t* __restrict__ rest, int64_t rest_cap, uint32_t* rest_count,
                                                 Counters* cnt) {
  __shared__ int32_t s_v[kLongCap * 64];
  __shared__ int32_t s_h[kLongCap * 64];
  __shared__ int32_t s_f[kLongCap * 64];
  const int lane = threadIdx.x;
  const LdsCol v{s_v + lane}, h{s_h + lane}, f{s_f + lane};
  const uint32_t n = (uint32_t)min((int64_t)*in_count, in_cap);
  if (n <= few_max) return;
  if (n <= pass_max) {
    for (uint32_t j = blockIdx.x * 64 + lane; j < n && (int64_t)j < rest_cap; j += gridDim.x * 64)
      rest[j] = in[in_cap - 1 - j];
    if (blockIdx.x == 0 && lane == 0) {
      *rest_count = (uint32_t)min((int64_t)n, rest_cap);
      if ((int64_t)n > rest_cap) set_error(cnt, POLYLLA_EINTERNAL);
    }
    return;
  }
  uint32_t n_rep = 0;
  for (uint32_t j0 = blockIdx.x * 64; j0 < n; j0 += gridDim.x * 64) {
    const uint32_t j = j0 + lane;
    const bool valid = j < n;
    const int32_t i = valid ? in[in_cap - 1 - j] : 0;
    const int4 rc = valid ? ps.rec[i] : make_int4(0, 0, -1, 0);
    bool ok = valid && (uint32_t)rc.z < (uint32_t)nhe;
    int L = 0;
    if (ok) {
      // the cycle from its start half-edge over the walk words: frontier
      // half-edges, their vertices, and the internal edges crossed about
      // each vertex (f[k]: about v[k], between h[k-1] and h[k])
      const int32_t s0 = rc.z;
      int32_t c = s0, w = wk[s0];
      for (;;) {
        if (w >= 0) {
          ok = false;
          break;
        }
        v[L] = -1 - w;
        h[L] = c;
        ++L;
        int32_t x = he_next(c), steps = 0;
        for (;;) {
          w = wk[x];
          if (w < 0) break;
          if ((uint32_t)w >= (uint32_t)nhe || ++steps > kLongCap * 3) {
            ok = false;
            break;
          }
          x = he_next(w);
        }
        if (!ok) break;
        c = x;
        if (c == s0) {
          f[0] = steps;
          break;
        }
        if (L == kLongCap) {  // longer: the region kernels
          ok = false;
          break;
        }
        f[L] = steps;
      }
      ok = ok && L >= 3;
    }
    tip_rest<REPAIR>(ok, valid, i, L, nhe, nv, twin, origin, he, vtx, stage, stage_cap, arena, arena_cap, ps, rest,
                     rest_cap, rest_count, v, h, f, n_rep, cnt);
  }
  // repair counts: one update per wave
  const uint32_t tot = (uint32_t)__builtin_amdgcn_readlane((int32_t)wave_incl_sum(n_rep), 63);
  if (lane == 0 && tot) {
    atomicAdd(&cnt->n_tips, tot);
    atomicAdd(&cnt->n_splits, tot);
  }
}

// Short polygons with a tip or a repeated vertex: one lane each, the region
// in LDS columns interleaved over the 64 lanes of the block. Regions larger
// than kSmallK triangles (only on invalid input: the walk queues cycles of at
// most kWalkCap half-edges here) take general_one.
template <bool REPAIR>
__global__ __launch_bounds__(64) void k_general_small(const int32_t* __restrict__ list, bool from_seeds,
                                                      int32_t nhe, int64_t nv, const int32_t* __restrict__ twin,
                                                      const int32_t* __restrict__ origin,
                                                      const int32_t* __restrict__ wk, uint8_t* __restrict__ he,
                                                      uint8_t* __restrict__ vtx, int32_t* __restrict__ stage,
                                                      int64_t stage_cap, int32_t* __restrict__ arena,
                                                      int64_t arena_cap, PolyState ps,
                                                      const int32_t* __restrict__ deferred,
                                                      const uint32_t* n_in, uint32_t run_min, Counters* cnt) {
  __shared__ int32_t s_tri[kSmallK * 64];
  __shared__ int32_t s_lnk[3 * kSmallK * 64];
  __shared__ int32_t s_org[3 * kSmallK * 64];
  __shared__ int32_t s_cyc[kWalkCap * 64];
  __shared__ int32_t s_aux[kWalkCap * 64];
  const int lane = threadIdx.x;
  const Region<LdsCol> R{LdsCol{s_tri + lane}, LdsCol{s_lnk + lane}, LdsCol{s_org + lane}};
  const int32_t nt = nhe / 3;
  const uint32_t nd = *n_in;
  if (nd <= run_min) return;  // few of them: the one-wave region kernel takes them
  for (uint32_t j = blockIdx.x * 64 + threadIdx.x; j < nd; j += gridDim.x * 64) {
    const int32_t i = deferred[j];
    const int32_t item = list[i];
    ps.clear(i);
    const int32_t t0 = from_seeds ? item : (item >= 0 ? item / 3 : -1);
    if ((uint32_t)t0 >= (uint32_t)nt) {
      set_error(cnt, POLYLLA_ETOPO);
      continue;
    }
    const int k = gather_region(R, t0, kSmallK, nhe, twin, origin, wk);
    if (k == -2) {
      set_error(cnt, POLYLLA_ETOPO);
      continue;
    }
    if (k < 0) {
      const int32_t s = from_seeds ? seed_start(item, nhe, twin, he, cnt) : item;
      general_one<REPAIR>(i, s, nhe, nv, twin, origin, he, vtx, stage, stage_cap, arena, arena_cap, ps, cnt);
      continue;
    }
    // start: the seed's first frontier half-edge in local order, else the
    // first met turning about its vertex 0; or the given start half-edge
    int start;
    if (from_seeds) {
      start = R.link(0) < 0 ? 0 : (R.link(1) < 0 ? 1 : (R.link(2) < 0 ? 2 : -1));
      if (start < 0) {
        int c = 0;
        for (int n = 0; n <= 3 * k && R.link(c) >= 0; ++n) c = R.turn(c);
        start = R.link(c) < 0 ? c : -1;
      }
    } else {
      start = item - 3 * t0;
      if (R.link(start) >= 0) start = -1;
    }
    if (start < 0) {
      set_error(cnt, POLYLLA_EDEGEN);
      continue;
    }
    region_core<REPAIR>(i, R, k, start, LdsCol{s_cyc + lane}, LdsCol{s_aux + lane}, nv, he, vtx, stage, stage_cap,
                        arena, arena_cap, ps, cnt);
  }
}

// ---------------------------------------------------------------------------
// Cooperative path: one workgroup per long polygon, the region in LDS.
//
// 1. Breadth-first search of the region's dual tree from its seed triangle
//    through internal edges (depth = longest edge propagation path, short),
//    collecting the frontier half-edges and a hash map half-edge -> slot.
// 2. Successor of every frontier half-edge (turning about its end vertex),
//    in parallel; tips (successor == twin) and barrier edges (twin also in the
//    region) fall out of the same pass.
// 3. Repair: middle edge of every tip in parallel, tips ranked by vertex id,
//    the "a smaller live tip opened an edge at me" rule resolved in that
//    order, opened edges added to the frontier set, successors recomputed.
// 4. Pieces are the cycles of the successor map: piece id = smallest slot on
//    the cycle and ranks from the canonical start, both by pointer jumping;
//    pieces ordered by their first two vertices; vertices written to staging.
// Regions beyond the LDS capacity are queued for general_one on one lane.

// Capacities of one instance: KC triangles, LC frontier half-edges (opened
// ones included), HB hash bits (2^HB = 2 LC hash slots). The region is kept
// as links between local edges (code = 4 slot + local edge), so successors
// and the repair never go back to global memory. Several arrays change role
// between phases to fit the 1024-thread instance in 160 KB.
template <int KC, int LC, int HB>
struct BigLds {
  static constexpr int kKCap = KC, kLCap = LC, kHBits = HB, kHCap = 1 << HB;
  static constexpr bool kOrg = KC <= 256;  // small instances keep every local edge's origin
  static_assert(kHCap == 2 * LC, "the hash area is reused for two per-piece arrays");
  static_assert(3 * KC >= 2 * LC, "the link area holds the vertex ids of the frontier slots");
  int32_t q[KC];        // triangle of each region slot | (entry edge + 1) << 30; then distances
  int32_t fh[LC];       // frontier half-edges of the region
  int32_t hkey[kHCap];  // hash keys; then tips (vertex, frontier slot / middle edge code); then per-piece arrays
  int32_t hval[LC];     // hash values (int16 per hash slot); then per-piece start slot
  int16_t nx[LC];       // successor slot; then sorted piece order
  int16_t jp[LC];       // jump pointers; dead flags; piece list
  int32_t a[LC];        // twin of each frontier slot; then (int16) its frontier slot, far vertex of
                        // each tip's middle edge (upper half); tip order; piece id
  int32_t kc[LC / 2];   // repair: undecided smaller tips whose opened edge ends at this tip
  int16_t kf[LC / 2];   // repair: rank of the tip at the far end of this tip's opened edge, or -1
  int32_t sc[20];
  int16_t lnk[3 * KC];  // internal edge: code of its twin; frontier edge: -1 - its frontier slot;
                        // after the repair: vertex id of each frontier slot (int32)
  int16_t fcode[LC];    // code of each frontier slot
  int32_t org[kOrg ? 3 * KC : 1];  // origin of each local edge (small instances)
};

enum {
  SC_QLEN, SC_LO, SC_HI, SC_NFH, SC_NTIP, SC_OVER, SC_BAD, SC_NSPLIT, SC_NP, SC_ITEM, SC_SBASE, SC_RB,
  SC_PEND,  // two slots, used alternately
  SC_SNEXT = SC_PEND + 2, SC_SLEFT, SC_ANEXT, SC_ALEFT  // the workgroup's staging and arena chunks
};
constexpr uint32_t kSlotTri = 0x3FFFFFFFu;  // triangle bits of q[slot]

template <int HB>
__device__ __forceinline__ int hash_slot(int32_t key) {
  return (int)(((uint32_t)key * 2654435761u) >> (32 - HB));
}

// Open-addressing hash (linear probing) from half-edge id to slot; keys in
// hkey, values as int16 per hash slot in the hval area.
template <class LDS>
__device__ __forceinline__ void hash_insert(LDS& S, int16_t* hv, int32_t key, int32_t val) {
  constexpr int kHCap = LDS::kHCap;
  int s = hash_slot<LDS::kHBits>(key);
  for (int k = 0; k < kHCap; ++k) {
    int32_t old = atomicCAS(&S.hkey[s], -1, key);
    if (old == -1 || old == key) {
      hv[s] = (int16_t)val;
      return;
    }
    s = (s + 1) & (kHCap - 1);
  }
}

template <class LDS>
__device__ __forceinline__ int32_t hash_find(const LDS& S, const int16_t* hv, int32_t key) {
  constexpr int kHCap = LDS::kHCap;
  int s = hash_slot<LDS::kHBits>(key);
  for (int k = 0; k < kHCap; ++k) {
    const int32_t kk = S.hkey[s];
    if (kk == key) return hv[s];
    if (kk == -1) return -1;
    s = (s + 1) & (kHCap - 1);
  }
  return -1;
}

// Successor slot of every frontier slot from the region links (LDS only);
// flags an invalid region.
template <int NT, class LDS>
__device__ __forceinline__ void successors_links(LDS& S, int L) {
  constexpr int kBound = 3 * LDS::kKCap + 3;
  for (int k = threadIdx.x; k < L; k += NT) {
    int x = S.fcode[k];
    x = (x & ~3) | next_local(x & 3);
    int r = -1;
    for (int n = 0; n < kBound; ++n) {
      const int l = S.lnk[3 * (x >> 2) + (x & 3)];
      if (l < 0) {
        r = -1 - l;
        break;
      }
      x = (l & ~3) | next_local(l & 3);
    }
    if (r < 0) {
      S.sc[SC_BAD] = 1;
      r = k;
    }
    S.nx[k] = (int16_t)r;
  }
}

// One step of a turn about a vertex inside the region: cross the edge of code
// x to its twin and take the twin's next local edge; -1 if the twin is not in
// the region. ts: frontier slot of the twin of each frontier slot, or -1.
template <class LDS>
__device__ __forceinline__ int turn_links(const LDS& S, const int16_t* ts, int x) {
  int y = S.lnk[3 * (x >> 2) + (x & 3)];
  if (y < 0) {
    const int f2 = ts[-1 - y];
    if (f2 < 0) return -1;
    y = S.fcode[f2];
  }
  return (y & ~3) | next_local(y & 3);
}

// Global half-edge of a local edge code.
template <class LDS>
__device__ __forceinline__ int32_t code_gid(const LDS& S, int c) {
  return 3 * (int32_t)((uint32_t)S.q[c >> 2] & kSlotTri) + (c & 3);
}

// Origin of a local edge code: from LDS in small instances, else one load.
template <class LDS>
__device__ __forceinline__ int32_t code_origin(const LDS& S, const int32_t* __restrict__ origin, int c) {
  if constexpr (LDS::kOrg) return S.org[3 * (c >> 2) + (c & 3)];
  else return origin[code_gid(S, c)];
}

// Queue a polygon for the next, larger instance (bounded: the queues are sized
// from the smallest region that can exceed an instance's capacities).
__device__ __forceinline__ void push_over(int32_t* over, int64_t over_cap, uint32_t* over_count, int32_t i,
                                          Counters* cnt) {
  const uint32_t q = atomicAdd(over_count, 1u);
  if ((int64_t)q < over_cap) over[q] = i;
  else set_error(cnt, POLYLLA_EINTERNAL);
}

// One instance of the workgroup region path: NT threads per region, LDS
// capacities KC/LC/HB. Polygons come from `in` (in_rev: counted from the back
// of the array, in_cap its length), `in_count` of them, taken by `in_ticket`;
// regions beyond the capacities go to `over` (count `over_count`).
// With `few_count` given and at most `few_max` long polygons in all, the first
// instance (few_in null) leaves them all to the second, which then takes them
// from few_in (from the back, few_cap long) instead of `in`: a few long
// regions are then not gathered twice. An instance with more than `run_max`
// polygons to take does nothing (another kernel takes them).
template <bool REPAIR, int NT, int KC, int LC, int HB>
__global__ __launch_bounds__(NT) void k_general_big(
    const int32_t* __restrict__ list, bool from_seeds, int32_t nhe, int64_t nv, const int32_t* __restrict__ twin,
    const int32_t* __restrict__ origin, const int32_t* __restrict__ wk, uint8_t* __restrict__ he,
    uint8_t* __restrict__ vtx, int32_t* __restrict__ stage, int64_t stage_cap, int32_t* __restrict__ arena,
    int64_t arena_cap, PolyState ps, const int32_t* __restrict__ in, bool in_rev, int64_t in_cap,
    const uint32_t* in_count, uint32_t* in_ticket, int32_t* __restrict__ over, int64_t over_cap,
    uint32_t* over_count, const int32_t* __restrict__ few_in, int64_t few_cap, const uint32_t* few_count,
    uint32_t few_max, uint32_t run_max, int32_t cap_lim, Counters* cnt) {
  constexpr int kBigThreads = NT, kKCap = KC, kLCap = LC, kHCap = 1 << HB, kPer = LC / NT;
  const int kcap = min(kKCap, cap_lim), lcap = min(kLCap, cap_lim);  // limits in use
  static_assert(LC % NT == 0 && kPer >= 1, "slots per thread");
  static_assert(KC < (1 << 13) && LC < (1 << 14), "codes and slots are int16");
  __shared__ BigLds<KC, LC, HB> S;
  int16_t* hv = reinterpret_cast<int16_t*>(S.hval);  // hash values: int16 per hash slot (kHCap of them)
  int16_t* tslot = reinterpret_cast<int16_t*>(S.a);  // (after the successor pass)
  int32_t* bv = reinterpret_cast<int32_t*>(S.lnk);   // (after the repair)
  const int tid = threadIdx.x;
  // one-wave instances take polygons round-robin (no shared work counter);
  // staging and arena space is reserved in chunks per workgroup
  constexpr bool kStaticItems = NT == 64;
  constexpr int32_t kStageChunkWg = NT == 64 ? kBigStageChunk64 : kBigStageChunk1024;
  constexpr int32_t kArenaChunkWg = NT == 64 ? kBigArenaChunk64 : kBigArenaChunk1024;
  if (tid == 0) {
    S.sc[SC_SLEFT] = 0;
    S.sc[SC_ALEFT] = 0;
  }
  if (few_count && *few_count <= few_max) {
    if (!few_in) return;
    in = few_in;
    in_rev = true;
    in_cap = few_cap;
    in_count = few_count;
  }
  const uint32_t nbig = *in_count;
  if (nbig > run_max) return;
  const int32_t nt = nhe / 3;
  uint32_t next_item = blockIdx.x;
  for (;;) {
    uint32_t item;
    if constexpr (kStaticItems) {
      item = next_item;
      next_item += gridDim.x;
      __syncthreads();
    } else {
      if (tid == 0) S.sc[SC_ITEM] = (int32_t)atomicAdd(in_ticket, 1u);
      __syncthreads();
      item = (uint32_t)S.sc[SC_ITEM];
    }
    if (item >= nbig) break;
    const int32_t i = in_rev ? in[in_cap - 1 - item] : in[item];
    const int32_t li = list[i];
    const int32_t t0 = from_seeds ? li : li / 3;
    // ---- 1. breadth-first search of the region's dual tree: slots, links,
    // frontier slots (half-edge, twin, code) and the hash half-edge -> slot
    for (int k = tid; k < kHCap; k += kBigThreads) S.hkey[k] = -1;
    if (tid == 0) {
      S.q[0] = t0;  // entry edge: none
      S.sc[SC_QLEN] = 1;
      S.sc[SC_LO] = 0;
      S.sc[SC_HI] = 1;
      S.sc[SC_NFH] = 0;
      S.sc[SC_NTIP] = 0;
      S.sc[SC_OVER] = ((uint32_t)t0 >= (uint32_t)nt) ? 1 : 0;
      S.sc[SC_BAD] = 0;
      S.sc[SC_NSPLIT] = 0;
      S.sc[SC_NP] = 0;
    }
    __syncthreads();
    for (;;) {
      const int lo = S.sc[SC_LO], hi = S.sc[SC_HI];
      if (lo >= hi || S.sc[SC_OVER]) break;
      for (int j = lo + tid; j < hi; j += kBigThreads) {
        const uint32_t qj = (uint32_t)S.q[j];
        const int32_t t = (int32_t)(qj & kSlotTri);
        const int entry = (int)(qj >> 30) - 1;
        // walk, twin and origin triples of the triangle: one round trip
        const Int3 tw3 = *reinterpret_cast<const Int3*>(twin + 3 * t);
        const Int3 or3 = *reinterpret_cast<const Int3*>(origin + 3 * t);
        const Int3 wk3 = *reinterpret_cast<const Int3*>(wk + 3 * t);
#pragma unroll
        for (int e = 0; e < 3; ++e) {
          const int32_t h = 3 * t + e;
          if constexpr (BigLds<KC, LC, HB>::kOrg) S.org[3 * j + e] = sel3(or3.x, or3.y, or3.z, e);
          if (e == entry) continue;  // (its link was set by the parent)
          const int32_t tw = sel3(tw3.x, tw3.y, tw3.z, e);
          if (sel3(wk3.x, wk3.y, wk3.z, e) < 0) {  // frontier
            const int idx = atomicAdd(&S.sc[SC_NFH], 1);
            if (idx < lcap) {
              S.fh[idx] = h;
              S.a[idx] = tw;
              S.fcode[idx] = (int16_t)(4 * j + e);
              S.lnk[3 * j + e] = (int16_t)(-1 - idx);
              hash_insert(S, hv, h, idx);
            } else {
              S.sc[SC_OVER] = 1;
            }
          } else {
            if ((uint32_t)tw >= (uint32_t)nhe) {
              S.sc[SC_BAD] = 1;
              continue;
            }
            const int pos = atomicAdd(&S.sc[SC_QLEN], 1);
            if (pos < kcap) {
              const int32_t t2 = tw / 3;
              const int e2 = tw - 3 * t2;
              S.q[pos] = (int32_t)((uint32_t)t2 | ((uint32_t)(e2 + 1) << 30));
              S.lnk[3 * j + e] = (int16_t)(4 * pos + e2);
              S.lnk[3 * pos + e2] = (int16_t)(4 * j + e);
            } else {
              S.sc[SC_OVER] = 1;
            }
          }
        }
      }
      __syncthreads();
      if (tid == 0) {
        S.sc[SC_LO] = hi;
        S.sc[SC_HI] = min(S.sc[SC_QLEN], kcap);
      }
      __syncthreads();
    }
    if (S.sc[SC_BAD]) {
      if (tid == 0) {
        set_error(cnt, POLYLLA_ETOPO);
        ps.clear(i);
      }
      __syncthreads();
      continue;
    }
    if (S.sc[SC_OVER]) {
      if (tid == 0) push_over(over, over_cap, over_count, i, cnt);
      __syncthreads();
      continue;
    }
    int L = S.sc[SC_NFH];
    // ---- 2. successors, barrier edges (twin also a frontier slot), tips
    // (successor = twin)
    successors_links<NT>(S, L);
    __syncthreads();
    int16_t tsr[kPer];
    bool tip[kPer];
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int k = tid + u * kBigThreads;
      tsr[u] = -1;
      tip[u] = false;
      if (k >= L) continue;
      const int j = S.nx[k];
      const int32_t tw = S.a[k];
      const int32_t ts = (uint32_t)tw < (uint32_t)nhe ? hash_find(S, hv, tw) : -1;
      tsr[u] = (int16_t)ts;
      tip[u] = S.fh[j] == tw && j != k;
      if (ts >= 0) or_bits(he, S.fh[k], kBarrier);
    }
    __syncthreads();  // the hash and the twins are done with
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int k = tid + u * kBigThreads;
      if (k >= L) continue;
      tslot[k] = tsr[u];
      if (tip[u]) {  // tip list (vertex, frontier slot of the barrier half-edge leaving it)
        const int j = S.nx[k];
        const int p = atomicAdd(&S.sc[SC_NTIP], 1);
        S.hkey[2 * p] = code_origin(S, origin, S.fcode[j]);
        S.hkey[2 * p + 1] = j;
      }
    }
    __syncthreads();
    if (S.sc[SC_BAD]) {
      if (tid == 0) {
        set_error(cnt, POLYLLA_EDEGEN);
        ps.clear(i);
      }
      __syncthreads();
      continue;
    }
    const int ntip = S.sc[SC_NTIP];
    // ---- 3. repair
    if (REPAIR && ntip > 0) {
      // middle internal edge c_{floor(d/2)} of every tip's fan (which lies in
      // the region), turning from the barrier half-edge; its far vertex goes
      // to a[LC/2 + p]
      for (int p = tid; p < ntip; p += kBigThreads) {
        const int x0 = S.fcode[S.hkey[2 * p + 1]];
        int d = 0, x = x0;
        do {
          x = turn_links(S, tslot, x);
          ++d;
        } while (x >= 0 && x != x0 && d <= 3 * kKCap);
        if (x != x0) {
          S.sc[SC_BAD] = 1;
          d = 0;
        }
        int ec = x0;
        for (int k = 0; k < d / 2; ++k) ec = turn_links(S, tslot, ec);
        S.hkey[2 * p + 1] = ec;  // a code from here on
        S.a[kLCap / 2 + p] = code_origin(S, origin, (ec & ~3) | next_local(ec & 3));
      }
      __syncthreads();
      // tips ranked by vertex id (ids are distinct): a[rank] = tip
      for (int p = tid; p < ntip; p += kBigThreads) {
        const int32_t v = S.hkey[2 * p];
        int r = 0;
        for (int p2 = 0; p2 < ntip; ++p2) r += S.hkey[2 * p2] < v;
        S.a[r] = p;
      }
      __syncthreads();
      // Live tips in increasing vertex order; a live tip whose opened edge
      // ends at a larger tip's vertex removes that tip. kf[r] is that larger
      // tip's rank; the ranks form a forest with edges to larger ranks, decided
      // in rounds: a tip none of whose undecided smaller tips point at it is
      // live, and the tip it points at is dead.
      for (int r = tid; r < ntip; r += kBigThreads) {
        S.kc[r] = 0;
        S.jp[r] = 0;
      }
      if (tid == 0) {
        S.sc[SC_PEND] = 0;
        S.sc[SC_PEND + 1] = 0;
        S.sc[SC_NSPLIT] = 0;
      }
      __syncthreads();
      for (int r = tid; r < ntip; r += kBigThreads) {
        const int32_t x = S.a[kLCap / 2 + S.a[r]];
        int lo = r + 1, hi = ntip;
        while (lo < hi) {
          const int mid = (lo + hi) >> 1;
          if (S.hkey[2 * S.a[mid]] < x) lo = mid + 1;
          else hi = mid;
        }
        const int f = (lo < ntip && S.hkey[2 * S.a[lo]] == x) ? lo : -1;
        S.kf[r] = (int16_t)f;
        if (f >= 0) atomicAdd(&S.kc[f], 1);
      }
      __syncthreads();
      // jp: 0 undecided, 1 newly live, 2 live, 3 newly dead, 4 dead
      for (int round = 0;; ++round) {
        const int par = SC_PEND + (round & 1);
        for (int r = tid; r < ntip; r += kBigThreads) {
          if (S.jp[r] != 0) continue;
          if (S.kc[r] == 0) S.jp[r] = 1;
          else S.sc[par] = 1;
        }
        __syncthreads();
        if (tid == 0) S.sc[SC_PEND + ((round + 1) & 1)] = 0;
        for (int r = tid; r < ntip; r += kBigThreads) {
          if (S.jp[r] != 1) continue;
          S.jp[r] = 2;
          if (S.kf[r] >= 0) S.jp[S.kf[r]] = 3;
        }
        __syncthreads();
        for (int r = tid; r < ntip; r += kBigThreads) {
          if (S.jp[r] != 3) continue;
          S.jp[r] = 4;
          if (S.kf[r] >= 0) atomicSub(&S.kc[S.kf[r]], 1);
        }
        __syncthreads();
        if (!S.sc[par]) break;
      }
      // jp[r] = 1 marks a dead tip from here on; live tips count the splits
      for (int r = tid; r < ntip; r += kBigThreads) {
        const bool dead = S.jp[r] == 4;
        S.jp[r] = dead ? 1 : 0;
        if (!dead) atomicAdd(&S.sc[SC_NSPLIT], 1);
      }
      __syncthreads();
      if (tid == 0 && L + 2 * S.sc[SC_NSPLIT] > lcap) S.sc[SC_OVER] = 1;
      __syncthreads();
      if (S.sc[SC_BAD]) {
        if (tid == 0) {
          set_error(cnt, POLYLLA_ETOPO);
          ps.clear(i);
        }
        __syncthreads();
        continue;
      }
      if (S.sc[SC_OVER]) {
        if (tid == 0) push_over(over, over_cap, over_count, i, cnt);
        __syncthreads();
        continue;
      }
      // open the middle edges of the live tips: both half-edges become
      // frontier slots
      for (int r = tid; r < ntip; r += kBigThreads) {
        if (S.jp[r]) continue;
        const int ec = S.hkey[2 * S.a[r] + 1];
        const int tc = S.lnk[3 * (ec >> 2) + (ec & 3)];
        if (tc < 0) {  // the middle edge must be internal
          S.sc[SC_BAD] = 1;
          continue;
        }
        const int32_t ge = code_gid(S, ec), gt = code_gid(S, tc);
        or_bits(he, ge, kFrontier | kRepaired);
        or_bits(he, gt, kFrontier | kRepaired);
        const int idx = atomicAdd(&S.sc[SC_NFH], 2);
        S.fh[idx] = ge;
        S.fh[idx + 1] = gt;
        S.fcode[idx] = (int16_t)ec;
        S.fcode[idx + 1] = (int16_t)tc;
        S.lnk[3 * (ec >> 2) + (ec & 3)] = (int16_t)(-1 - idx);
        S.lnk[3 * (tc >> 2) + (tc & 3)] = (int16_t)(-2 - idx);
      }
      __syncthreads();
      if (tid == 0 && S.sc[SC_NSPLIT]) atomicAdd(&cnt->n_splits, (uint32_t)S.sc[SC_NSPLIT]);
      L = S.sc[SC_NFH];
      if (S.sc[SC_NSPLIT]) {
        successors_links<NT>(S, L);
        __syncthreads();
      }
      if (S.sc[SC_BAD]) {
        if (tid == 0) {
          set_error(cnt, POLYLLA_EDEGEN);
          ps.clear(i);
        }
        __syncthreads();
        continue;
      }
    }
    // tips (counted once the region stays in this instance)
    for (int p = tid; p < ntip; p += kBigThreads) {
      const int32_t v = S.hkey[2 * p];
      if ((uint64_t)(uint32_t)v < (uint64_t)nv) or_bits(vtx, v, kTip);
    }
    if (tid == 0 && ntip) atomicAdd(&cnt->n_tips, (uint32_t)ntip);
    // vertex id of every frontier slot, into the link area (the links are
    // done with)
    int32_t vreg[kPer];
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int k = tid + u * kBigThreads;
      vreg[u] = k < L ? code_origin(S, origin, S.fcode[k]) : 0;
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int k = tid + u * kBigThreads;
      if (k < L) bv[k] = vreg[u];
    }
    __syncthreads();
    // ---- 4. pieces = cycles of nx. One pointer-jumping pass gives every
    // slot the smallest (vertex, slot) pair on its cycle and its distance to
    // that slot, which starts the piece and names it: the window of slot k
    // grows to [k, k + 2 span) from its own and the one of the slot span
    // ahead; a = best vertex, q = best slot << 16 | distance (both < 2^13).
    for (int k = tid; k < L; k += kBigThreads) {
      S.a[k] = bv[k];
      S.q[k] = k << 16;
      S.jp[k] = S.nx[k];
    }
    __syncthreads();
    for (int span = 1; span < L; span <<= 1) {
      int32_t na[kPer], nq[kPer];
      int16_t nj[kPer];
#pragma unroll
      for (int u = 0; u < kPer; ++u) {
        const int k = tid + u * kBigThreads;
        if (k < L) {
          const int j = S.jp[k];
          const int32_t va = S.a[k], vq = S.q[k], ja = S.a[j], jq = S.q[j] + span;
          const bool take = ja < va || (ja == va && jq < vq);
          na[u] = take ? ja : va;
          nq[u] = take ? jq : vq;
          nj[u] = S.jp[j];
        }
      }
      __syncthreads();
#pragma unroll
      for (int u = 0; u < kPer; ++u) {
        const int k = tid + u * kBigThreads;
        if (k < L) {
          S.a[k] = na[u];
          S.q[k] = nq[u];
          S.jp[k] = nj[u];
        }
      }
      __syncthreads();
    }
    // piece id (its start slot) into a, distance to the start into q; per
    // piece: smallest vertex (hkey[p]), its multiplicity (hkey[kLCap + p]),
    // start slot (hval[p] as int32), length (fcode[p])
    int32_t* pmin = S.hkey;
    int32_t* pcnt = S.hkey + kLCap;
    int32_t* pstart = S.hval;
    int16_t* plen = S.fcode;
    for (int k = tid; k < L; k += kBigThreads) {
      const int32_t v = S.q[k];
      S.a[k] = v >> 16;
      S.q[k] = v & 0xFFFF;
    }
    __syncthreads();
    for (int k = tid; k < L; k += kBigThreads) {
      if (S.a[k] != k) continue;
      pmin[k] = bv[k];
      pcnt[k] = 0;
      pstart[k] = k;
      plen[k] = (int16_t)(S.q[S.nx[k]] + 1);
    }
    __syncthreads();
    for (int k = tid; k < L; k += kBigThreads) {
      const int p = S.a[k];
      if (bv[k] == pmin[p]) atomicAdd(&pcnt[p], 1);
    }
    __syncthreads();
    // a piece visiting its smallest vertex twice starts at the occurrence
    // with the lexicographically smallest continuation; its distances are
    // then taken again from that slot
    for (int p = tid; p < L; p += kBigThreads) {
      if (S.a[p] != p || pcnt[p] < 2) continue;
      const int len = plen[p];
      int best = p;
      for (int k = S.nx[p], m = 1; m < len; k = S.nx[k], ++m) {
        if (bv[k] != pmin[p]) continue;
        int x = k, y = best;
        for (int z = 0; z < len; ++z) {
          if (bv[x] != bv[y]) {
            if (bv[x] < bv[y]) best = k;
            break;
          }
          x = S.nx[x];
          y = S.nx[y];
        }
      }
      if (best != p) {
        for (int k = best, m = 0; m < len; k = S.nx[k], ++m) S.q[k] = m ? len - m : 0;
        pstart[p] = best;
      }
    }
    __syncthreads();
    // pieces: list (jp), second vertex (pcnt reused)
    for (int k = tid; k < L; k += kBigThreads) {
      if (S.a[k] != k) continue;
      const int idx = atomicAdd(&S.sc[SC_NP], 1);
      S.jp[idx] = (int16_t)k;
      pcnt[k] = bv[S.nx[pstart[k]]];
    }
    __syncthreads();
    const int np = S.sc[SC_NP];
    // order pieces by (first, second) vertex: nx[rank] = piece
    for (int u = tid; u < np; u += kBigThreads) {
      const int p = S.jp[u];
      const int32_t k0 = pmin[p], k1 = pcnt[p];
      int r = 0;
      for (int w = 0; w < np; ++w) {
        const int p2 = S.jp[w];
        r += (pmin[p2] < k0) || (pmin[p2] == k0 && pcnt[p2] < k1);
      }
      S.nx[r] = (int16_t)p;
    }
    __syncthreads();
    // piece lengths in output order and their offsets (block scan; np <= kLCap = kPer * kBigThreads)
    int32_t lens[kPer];
    uint32_t mine = 0;
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int r = kPer * tid + u;
      lens[u] = r < np ? plen[S.nx[r]] : 0;
      mine += (uint32_t)lens[u];
    }
    uint2 tot;
    const uint2 pre = block_exclusive_scan<NT>(mine, 0u, &tot);
    if (tid == 0) {
      const int32_t total = (int32_t)tot.x;
      bool ok = true;
      if (total > S.sc[SC_SLEFT]) {  // a new staging chunk for this workgroup
        const int32_t want = max(total, kStageChunkWg);
        const uint32_t nb = atomicAdd(&cnt->stage_top, (uint32_t)want);
        ok = (int64_t)nb + want <= stage_cap;
        S.sc[SC_SNEXT] = (int32_t)nb;
        S.sc[SC_SLEFT] = ok ? want : 0;
      }
      const int32_t sb = S.sc[SC_SNEXT];
      if (ok) {
        S.sc[SC_SNEXT] += total;
        S.sc[SC_SLEFT] -= total;
      }
      int32_t rb = -1;
      if (ok && np > 1) {
        const int32_t need = 4 * np;
        if (need > S.sc[SC_ALEFT]) {
          const int32_t want = max(need, kArenaChunkWg);
          const uint32_t nb = atomicAdd(&cnt->arena_top, (uint32_t)want);
          ok = (int64_t)nb + want <= arena_cap;
          S.sc[SC_ANEXT] = (int32_t)nb;
          S.sc[SC_ALEFT] = ok ? want : 0;
        }
        rb = S.sc[SC_ANEXT];
        if (ok) {
          S.sc[SC_ANEXT] += need;
          S.sc[SC_ALEFT] -= need;
        }
      }
      if (!ok) {
        set_error(cnt, POLYLLA_ENOMEM);
        S.sc[SC_OVER] = 1;
      } else {
        ps.set(i, total, np, np == 1 ? S.fh[pstart[S.nx[0]]] : -1, (int32_t)sb);
        ps.prec[i] = np > 1 ? rb : -1;
      }
      S.sc[SC_SBASE] = (int32_t)sb;
      S.sc[SC_RB] = rb;
    }
    __syncthreads();
    if (!S.sc[SC_OVER]) {
      // piece records for the emitter; pcnt[p] becomes the piece's output offset
      const int32_t rb = S.sc[SC_RB];
      int32_t run = (int32_t)pre.x;
#pragma unroll
      for (int u = 0; u < kPer; ++u) {
        const int r = kPer * tid + u;
        if (r >= np) continue;
        const int p = S.nx[r];
        if (np > 1) {
          arena[rb + 4 * r] = pmin[p];
          arena[rb + 4 * r + 1] = pcnt[p];
          arena[rb + 4 * r + 2] = S.fh[pstart[p]];
          arena[rb + 4 * r + 3] = lens[u];
        }
        pcnt[p] = run;
        run += lens[u];
      }
    }
    __syncthreads();
    if (!S.sc[SC_OVER]) {
      const int32_t sb = S.sc[SC_SBASE];
      for (int k = tid; k < L; k += kBigThreads) {
        const int p = S.a[k];
        const int32_t d = S.q[k];
        stage[sb + pcnt[p] + (d ? plen[p] - d : 0)] = bv[k];
      }
    } else if (tid == 0) {
      ps.clear(i);
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------

// Views of one workgroup's part of the global-memory region store (the same
// four steps as the LDS kernel, one array per role instead of shared areas,
// and ping-pong arrays instead of registers for the pointer jumping).
struct MemRegion {
  int32_t *q, *lnk;                                      // slots: km, links: 3 km
  int32_t *hkey, *hval;                                  // hash: mem_hcap(km) each
  int32_t *fh, *tw, *fcode, *nx, *ts, *bv;               // frontier slots: 2 km each
  int32_t *pid[2], *jp[2], *dd[2], *ds[2];               // pointer jumping: 2 km each
  int32_t *pmin, *pcnt, *pstart, *psec, *poff, *plist, *porder;  // pieces: 2 km each
  int32_t *tipv, *tipc, *tipfar, *torder, *kc, *kf, *tst;        // tips: km each
};

__device__ __forceinline__ MemRegion mem_region(int32_t* base, int64_t km) {
  MemRegion r;
  int32_t* p = base;
  auto take = [&](int64_t n) {
    int32_t* q = p;
    p += n;
    return q;
  };
  const int64_t lm = 2 * km, hc = mem_hcap(km);
  r.q = take(km);
  r.lnk = take(3 * km);
  r.hkey = take(hc);
  r.hval = take(hc);
  r.fh = take(lm);
  r.tw = take(lm);
  r.fcode = take(lm);
  r.nx = take(lm);
  r.ts = take(lm);
  r.bv = take(lm);
  for (int k = 0; k < 2; ++k) {
    r.pid[k] = take(lm);
    r.jp[k] = take(lm);
    r.dd[k] = take(lm);
    r.ds[k] = take(lm);
  }
  r.pmin = take(lm);
  r.pcnt = take(lm);
  r.pstart = take(lm);
  r.psec = take(lm);
  r.poff = take(lm);
  r.plist = take(lm);
  r.porder = take(lm);
  r.tipv = take(km);
  r.tipc = take(km);
  r.tipfar = take(km);
  r.torder = take(km);
  r.kc = take(km);
  r.kf = take(km);
  r.tst = take(km);
  return r;
}

__device__ __forceinline__ int32_t mem_code_gid(const MemRegion& R, int c) {
  return 3 * (int32_t)((uint32_t)R.q[c >> 2] & kSlotTri) + (c & 3);
}

__device__ __forceinline__ int mem_turn(const MemRegion& R, int x) {
  int y = R.lnk[3 * (x >> 2) + (x & 3)];
  if (y < 0) {
    const int f2 = R.ts[-1 - y];
    if (f2 < 0) return -1;
    y = R.fcode[f2];
  }
  return (y & ~3) | next_local(y & 3);
}

template <int NT>
__device__ __forceinline__ void mem_successors(const MemRegion& R, int L, int kcap, int32_t* sc) {
  const int bound = 3 * kcap + 3;
  for (int k = threadIdx.x; k < L; k += NT) {
    int x = R.fcode[k];
    x = (x & ~3) | next_local(x & 3);
    int r = -1;
    for (int n = 0; n < bound; ++n) {
      const int l = R.lnk[3 * (x >> 2) + (x & 3)];
      if (l < 0) {
        r = -1 - l;
        break;
      }
      x = (l & ~3) | next_local(l & 3);
    }
    if (r < 0) {
      sc[SC_BAD] = 1;
      r = k;
    }
    R.nx[k] = r;
  }
}

// Rank of key[p] among key[0..n) (keys distinct) for every p < n, into
// out[rank] = p; the keys are read back a workgroup-sized tile at a time
// through LDS. Two keys compare lexicographically when key2 is given.
template <int NT>
__device__ __forceinline__ void mem_rank(const int32_t* key, const int32_t* key2, const int32_t* ids, int n,
                                         int32_t* out, int32_t* s_k1, int32_t* s_k2) {
  const int tid = threadIdx.x;
  for (int pb = 0; pb < n; pb += NT) {
    const int u = pb + tid;
    const int p = u < n ? (ids ? ids[u] : u) : 0;
    const int32_t v1 = u < n ? key[p] : 0, v2 = (u < n && key2) ? key2[p] : 0;
    int r = 0;
    for (int tb = 0; tb < n; tb += NT) {
      __syncthreads();
      if (tb + tid < n) {
        const int q = ids ? ids[tb + tid] : tb + tid;
        s_k1[tid] = key[q];
        s_k2[tid] = key2 ? key2[q] : 0;
      }
      __syncthreads();
      const int m = min(NT, n - tb);
      for (int w = 0; w < m; ++w) r += (s_k1[w] < v1) || (s_k1[w] == v1 && s_k2[w] < v2);
    }
    if (u < n) out[r] = p;
  }
  __syncthreads();
}

// One region by one workgroup with its arrays in global memory (capacities
// kcap triangles, lcap frontier slots); beyond them it goes to the lane list.
template <bool REPAIR, int NT>
__device__ void region_mem(const MemRegion& R, int32_t i, int32_t t0, int32_t nhe, int64_t nv,
                           const int32_t* __restrict__ twin, const int32_t* __restrict__ origin,
                           const int32_t* __restrict__ wk, uint8_t* __restrict__ he, uint8_t* __restrict__ vtx,
                           int32_t* __restrict__ stage, int64_t stage_cap, int32_t* __restrict__ arena,
                           int64_t arena_cap, PolyState ps, int32_t* lane, int64_t lane_cap, int kcap, int lcap,
                           int32_t* sc, int32_t* s_k1, int32_t* s_k2, Counters* cnt) {
  const int tid = threadIdx.x;
  const int32_t nt = nhe / 3;
  // ---- 1. breadth-first search of the region's dual tree
  if (tid == 0) {
    R.q[0] = t0;
    sc[SC_QLEN] = 1;
    sc[SC_LO] = 0;
    sc[SC_HI] = 1;
    sc[SC_NFH] = 0;
    sc[SC_NTIP] = 0;
    sc[SC_OVER] = ((uint32_t)t0 >= (uint32_t)nt) ? 1 : 0;
    sc[SC_BAD] = 0;
    sc[SC_NSPLIT] = 0;
    sc[SC_NP] = 0;
  }
  __syncthreads();
  for (;;) {
    const int lo = sc[SC_LO], hi = sc[SC_HI];
    if (lo >= hi || sc[SC_OVER]) break;
    for (int j = lo + tid; j < hi; j += NT) {
      const uint32_t qj = (uint32_t)R.q[j];
      const int32_t t = (int32_t)(qj & kSlotTri);
      const int entry = (int)(qj >> 30) - 1;
      const Int3 tw3 = *reinterpret_cast<const Int3*>(twin + 3 * t);
      const Int3 wk3 = *reinterpret_cast<const Int3*>(wk + 3 * t);
#pragma unroll
      for (int e = 0; e < 3; ++e) {
        if (e == entry) continue;
        const int32_t h = 3 * t + e;
        const int32_t tw = sel3(tw3.x, tw3.y, tw3.z, e);
        if (sel3(wk3.x, wk3.y, wk3.z, e) < 0) {  // frontier
          const int idx = atomicAdd(&sc[SC_NFH], 1);
          if (idx < lcap) {
            R.fh[idx] = h;
            R.tw[idx] = tw;
            R.fcode[idx] = 4 * j + e;
            R.lnk[3 * j + e] = -1 - idx;
          } else {
            sc[SC_OVER] = 1;
          }
        } else {
          if ((uint32_t)tw >= (uint32_t)nhe) {
            sc[SC_BAD] = 1;
            continue;
          }
          const int pos = atomicAdd(&sc[SC_QLEN], 1);
          if (pos < kcap) {
            const int32_t t2 = tw / 3;
            const int e2 = tw - 3 * t2;
            R.q[pos] = (int32_t)((uint32_t)t2 | ((uint32_t)(e2 + 1) << 30));
            R.lnk[3 * j + e] = 4 * pos + e2;
            R.lnk[3 * pos + e2] = 4 * j + e;
          } else {
            sc[SC_OVER] = 1;
          }
        }
      }
    }
    __syncthreads();
    if (tid == 0) {
      sc[SC_LO] = hi;
      sc[SC_HI] = min(sc[SC_QLEN], kcap);
    }
    __syncthreads();
  }
  if (sc[SC_BAD]) {
    if (tid == 0) {
      set_error(cnt, POLYLLA_ETOPO);
      ps.clear(i);
    }
    return;
  }
  if (sc[SC_OVER]) {
    if (tid == 0) push_over(lane, lane_cap, &cnt->n_lane, i, cnt);
    return;
  }
  int L = sc[SC_NFH];
  // hash of the frontier half-edges (open addressing, 2 L <= capacity)
  int hb = 6;
  while ((1 << hb) < 2 * L) ++hb;
  const int hcap = 1 << hb;
  for (int k = tid; k < hcap; k += NT) R.hkey[k] = -1;
  __syncthreads();
  for (int k = tid; k < L; k += NT) {
    const int32_t key = R.fh[k];
    int s = (int)(((uint32_t)key * 2654435761u) >> (32 - hb));
    for (int n = 0; n < hcap; ++n) {
      const int32_t old = atomicCAS(&R.hkey[s], -1, key);
      if (old == -1 || old == key) {
        R.hval[s] = k;
        break;
      }
      s = (s + 1) & (hcap - 1);
    }
  }
  __syncthreads();
  // ---- 2. successors, barrier edges, tips
  mem_successors<NT>(R, L, kcap, sc);
  __syncthreads();
  const int tipcap = lcap / 2;
  for (int k = tid; k < L; k += NT) {
    const int j = R.nx[k];
    const int32_t tw = R.tw[k];
    int32_t f = -1;
    if ((uint32_t)tw < (uint32_t)nhe) {
      int s = (int)(((uint32_t)tw * 2654435761u) >> (32 - hb));
      for (int n = 0; n < hcap; ++n) {
        const int32_t kk = R.hkey[s];
        if (kk == tw) {
          f = R.hval[s];
          break;
        }
        if (kk == -1) break;
        s = (s + 1) & (hcap - 1);
      }
    }
    R.ts[k] = f;
    if (f >= 0) or_bits(he, R.fh[k], kBarrier);
    if (R.fh[j] == tw && j != k) {  // tip (vertex, frontier slot of the barrier half-edge leaving it)
      const int p = atomicAdd(&sc[SC_NTIP], 1);
      if (p < tipcap) {
        R.tipv[p] = origin[mem_code_gid(R, R.fcode[j])];
        R.tipc[p] = j;
      } else {
        sc[SC_OVER] = 1;
      }
    }
  }
  __syncthreads();
  if (sc[SC_BAD]) {
    if (tid == 0) {
      set_error(cnt, POLYLLA_EDEGEN);
      ps.clear(i);
    }
    return;
  }
  if (sc[SC_OVER]) {
    if (tid == 0) push_over(lane, lane_cap, &cnt->n_lane, i, cnt);
    return;
  }
  const int ntip = sc[SC_NTIP];
  // ---- 3. repair
  if (REPAIR && ntip > 0) {
    // middle internal edge of every tip's fan, turning from the barrier
    // half-edge, and the far vertex of that edge
    for (int p = tid; p < ntip; p += NT) {
      const int x0 = R.fcode[R.tipc[p]];
      int d = 0, x = x0;
      do {
        x = mem_turn(R, x);
        ++d;
      } while (x >= 0 && x != x0 && d <= 3 * kcap);
      if (x != x0) {
        sc[SC_BAD] = 1;
        d = 0;
      }
      int ec = x0;
      for (int k = 0; k < d / 2; ++k) ec = mem_turn(R, ec);
      R.tipc[p] = ec;
      R.tipfar[p] = origin[mem_code_gid(R, (ec & ~3) | next_local(ec & 3))];
    }
    __syncthreads();
    // tips in increasing vertex order: torder[rank] = tip
    mem_rank<NT>(R.tipv, nullptr, nullptr, ntip, R.torder, s_k1, s_k2);
    // the rule of the LDS kernel: the live tips, in vertex order, remove the
    // larger tips at the far ends of their opened edges; decided in rounds
    // over the forest of ranks (tst: 0 undecided, 1 newly live, 2 live,
    // 3 newly dead, 4 dead)
    for (int r = tid; r < ntip; r += NT) {
      R.kc[r] = 0;
      R.tst[r] = 0;
    }
    if (tid == 0) {
      sc[SC_PEND] = 0;
      sc[SC_PEND + 1] = 0;
      sc[SC_NSPLIT] = 0;
    }
    __syncthreads();
    for (int r = tid; r < ntip; r += NT) {
      const int32_t x = R.tipfar[R.torder[r]];
      int lo = r + 1, hi = ntip;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (R.tipv[R.torder[mid]] < x) lo = mid + 1;
        else hi = mid;
      }
      const int f = (lo < ntip && R.tipv[R.torder[lo]] == x) ? lo : -1;
      R.kf[r] = f;
      if (f >= 0) atomicAdd(&R.kc[f], 1);
    }
    __syncthreads();
    for (int round = 0;; ++round) {
      const int par = SC_PEND + (round & 1);
      for (int r = tid; r < ntip; r += NT) {
        if (R.tst[r] != 0) continue;
        if (R.kc[r] == 0) R.tst[r] = 1;
        else sc[par] = 1;
      }
      __syncthreads();
      if (tid == 0) sc[SC_PEND + ((round + 1) & 1)] = 0;
      for (int r = tid; r < ntip; r += NT) {
        if (R.tst[r] != 1) continue;
        R.tst[r] = 2;
        if (R.kf[r] >= 0) R.tst[R.kf[r]] = 3;
      }
      __syncthreads();
      for (int r = tid; r < ntip; r += NT) {
        if (R.tst[r] != 3) continue;
        R.tst[r] = 4;
        if (R.kf[r] >= 0) atomicSub(&R.kc[R.kf[r]], 1);
      }
      __syncthreads();
      if (!sc[par]) break;
    }
    // tst = 1 marks a dead tip from here on; live tips count the splits
    for (int r = tid; r < ntip; r += NT) {
      const bool dead = R.tst[r] == 4;
      R.tst[r] = dead ? 1 : 0;
      if (!dead) atomicAdd(&sc[SC_NSPLIT], 1);
    }
    __syncthreads();
    if (tid == 0 && L + 2 * sc[SC_NSPLIT] > lcap) sc[SC_OVER] = 1;
    __syncthreads();
    if (sc[SC_BAD]) {
      if (tid == 0) {
        set_error(cnt, POLYLLA_ETOPO);
        ps.clear(i);
      }
      return;
    }
    if (sc[SC_OVER]) {
      if (tid == 0) push_over(lane, lane_cap, &cnt->n_lane, i, cnt);
      return;
    }
    // open the middle edges of the live tips
    for (int r = tid; r < ntip; r += NT) {
      if (R.tst[r]) continue;
      const int ec = R.tipc[R.torder[r]];
      const int tc = R.lnk[3 * (ec >> 2) + (ec & 3)];
      if (tc < 0) {
        sc[SC_BAD] = 1;
        continue;
      }
      const int32_t ge = mem_code_gid(R, ec), gt = mem_code_gid(R, tc);
      or_bits(he, ge, kFrontier | kRepaired);
      or_bits(he, gt, kFrontier | kRepaired);
      const int idx = atomicAdd(&sc[SC_NFH], 2);
      R.fh[idx] = ge;
      R.fh[idx + 1] = gt;
      R.fcode[idx] = ec;
      R.fcode[idx + 1] = tc;
      R.lnk[3 * (ec >> 2) + (ec & 3)] = -1 - idx;
      R.lnk[3 * (tc >> 2) + (tc & 3)] = -2 - idx;
    }
    __syncthreads();
    if (tid == 0 && sc[SC_NSPLIT]) atomicAdd(&cnt->n_splits, (uint32_t)sc[SC_NSPLIT]);
    L = sc[SC_NFH];
    if (sc[SC_NSPLIT]) {
      mem_successors<NT>(R, L, kcap, sc);
      __syncthreads();
    }
    if (sc[SC_BAD]) {
      if (tid == 0) {
        set_error(cnt, POLYLLA_EDEGEN);
        ps.clear(i);
      }
      return;
    }
  }
  for (int p = tid; p < ntip; p += NT) {
    const int32_t v = R.tipv[p];
    if ((uint64_t)(uint32_t)v < (uint64_t)nv) or_bits(vtx, v, kTip);
  }
  if (tid == 0 && ntip) atomicAdd(&cnt->n_tips, (uint32_t)ntip);
  // ---- 4. pieces = cycles of nx: one pointer-jumping pass gives every slot
  // the smallest (vertex, slot) pair on its cycle (the piece's start and
  // name) and its distance to it (best vertex in pid, best slot in dd,
  // distance in ds; ping-pong buffers)
  for (int k = tid; k < L; k += NT) {
    const int32_t v = origin[mem_code_gid(R, R.fcode[k])];
    R.bv[k] = v;
    R.pid[0][k] = v;
    R.dd[0][k] = k;
    R.ds[0][k] = 0;
    R.jp[0][k] = R.nx[k];
  }
  __syncthreads();
  int c = 0;
  for (int span = 1; span < L; span <<= 1) {
    for (int k = tid; k < L; k += NT) {
      const int j = R.jp[c][k];
      const int32_t va = R.pid[c][k], vs = R.dd[c][k], vd = R.ds[c][k];
      const int32_t ja = R.pid[c][j], js = R.dd[c][j], jd = R.ds[c][j] + span;
      const bool take = ja < va || (ja == va && (js < vs || (js == vs && jd < vd)));
      R.pid[c ^ 1][k] = take ? ja : va;
      R.dd[c ^ 1][k] = take ? js : vs;
      R.ds[c ^ 1][k] = take ? jd : vd;
      R.jp[c ^ 1][k] = R.jp[c][j];
    }
    __syncthreads();
    c ^= 1;
  }
  const int32_t* pid = R.dd[c];  // piece id: its start slot
  int32_t* dist = R.ds[c];       // distance to the piece's start
  int32_t* plen = R.pid[c];      // (best vertices no longer needed) piece length, by piece id
  // per piece: smallest vertex, its multiplicity, start slot, length
  for (int k = tid; k < L; k += NT) {
    if (pid[k] != k) continue;
    R.pmin[k] = R.bv[k];
    R.pcnt[k] = 0;
    R.pstart[k] = k;
    plen[k] = dist[R.nx[k]] + 1;
  }
  __syncthreads();
  for (int k = tid; k < L; k += NT) {
    const int p = pid[k];
    if (R.bv[k] == R.pmin[p]) atomicAdd(&R.pcnt[p], 1);
  }
  __syncthreads();
  // a piece visiting its smallest vertex twice starts at the occurrence with
  // the lexicographically smallest continuation; its distances are then
  // taken again from that slot
  for (int p = tid; p < L; p += NT) {
    if (pid[p] != p || R.pcnt[p] < 2) continue;
    const int len = plen[p];
    int best = p;
    for (int k = R.nx[p], m = 1; m < len; k = R.nx[k], ++m) {
      if (R.bv[k] != R.pmin[p]) continue;
      int x = k, y = best;
      for (int z = 0; z < len; ++z) {
        if (R.bv[x] != R.bv[y]) {
          if (R.bv[x] < R.bv[y]) best = k;
          break;
        }
        x = R.nx[x];
        y = R.nx[y];
      }
    }
    if (best != p) {
      for (int k = best, m = 0; m < len; k = R.nx[k], ++m) dist[k] = m ? len - m : 0;
      R.pstart[p] = best;
    }
  }
  __syncthreads();
  // pieces: list and second vertex
  for (int k = tid; k < L; k += NT) {
    if (pid[k] != k) continue;
    const int idx = atomicAdd(&sc[SC_NP], 1);
    R.plist[idx] = k;
    R.psec[k] = R.bv[R.nx[R.pstart[k]]];
  }
  __syncthreads();
  const int np = sc[SC_NP];
  // order pieces by (first, second) vertex: porder[rank] = piece
  mem_rank<NT>(R.pmin, R.psec, R.plist, np, R.porder, s_k1, s_k2);
  // output offset of every piece within the polygon
  uint32_t run = 0;
  for (int base = 0; base < np; base += NT) {
    const int r = base + tid;
    const uint32_t len = r < np ? (uint32_t)plen[R.porder[r]] : 0u;
    uint2 tot;
    const uint2 pre = block_exclusive_scan<NT>(len, 0u, &tot);
    if (r < np) R.poff[R.porder[r]] = (int32_t)(run + pre.x);
    run += tot.x;
  }
  if (tid == 0) {
    const int32_t total = (int32_t)run;
    const uint32_t sb = atomicAdd(&cnt->stage_top, (uint32_t)total);
    bool ok = (int64_t)sb + total <= stage_cap;
    int32_t rb = -1;
    if (ok && np > 1) {
      const uint32_t ab = atomicAdd(&cnt->arena_top, (uint32_t)(4 * np));
      ok = (int64_t)ab + 4 * np <= arena_cap;
      rb = (int32_t)ab;
    }
    if (!ok) {
      set_error(cnt, POLYLLA_ENOMEM);
      sc[SC_OVER] = 1;
      ps.clear(i);
    } else {
      ps.set(i, total, np, np == 1 ? R.fh[R.pstart[R.porder[0]]] : -1, (int32_t)sb);
      ps.prec[i] = np > 1 ? rb : -1;
    }
    sc[SC_SBASE] = (int32_t)sb;
    sc[SC_RB] = rb;
  }
  __syncthreads();
  if (sc[SC_OVER]) return;
  const int32_t sb = sc[SC_SBASE], rb = sc[SC_RB];
  if (np > 1) {
    for (int r = tid; r < np; r += NT) {
      const int p = R.porder[r];
      arena[rb + 4 * r] = R.pmin[p];
      arena[rb + 4 * r + 1] = R.psec[p];
      arena[rb + 4 * r + 2] = R.fh[R.pstart[p]];
      arena[rb + 4 * r + 3] = plen[p];
    }
  }
  for (int k = tid; k < L; k += NT) {
    const int p = pid[k];
    const int32_t d = dist[k];
    stage[sb + R.poff[p] + (d ? plen[p] - d : 0)] = R.bv[k];
  }
}

// Regions beyond the LDS of the 1024-thread workgroup (listed in `in`,
// cnt->n_fallback of them, in_cap at most): one workgroup each, taken by ticket, with the
// region in the workgroup's part of `store` (km triangles of capacity; kcap,
// lcap the limits in use). Regions beyond those go to `lane`; the last
// workgroup to finish then builds them one lane each.
template <bool REPAIR>
__global__ __launch_bounds__(1024) void k_general_huge(
    const int32_t* __restrict__ list, bool from_seeds, int32_t nhe, int64_t nv, const int32_t* __restrict__ twin,
    const int32_t* __restrict__ origin, const int32_t* __restrict__ wk, uint8_t* __restrict__ he,
    uint8_t* __restrict__ vtx, int32_t* __restrict__ stage, int64_t stage_cap, int32_t* __restrict__ arena,
    int64_t arena_cap, PolyState ps, const int32_t* __restrict__ in, int64_t in_cap, int32_t* __restrict__ lane,
    int64_t lane_cap, int32_t* __restrict__ store, int64_t km, int32_t kcap, int32_t lcap, Counters* cnt) {
  constexpr int NT = 1024;
  __shared__ int32_t sc[24];
  __shared__ int32_t s_k1[NT], s_k2[NT];
  __shared__ int32_t s_last;
  const int tid = threadIdx.x;
  const uint32_t nin = (uint32_t)min((int64_t)cnt->n_fallback, in_cap);
  if (nin == 0) return;  // (the one-lane list is filled only by this path)
  {
    const MemRegion R = mem_region(store + (int64_t)blockIdx.x * mem_words(km), km);
    for (;;) {
      if (tid == 0) sc[SC_ITEM] = (int32_t)atomicAdd(&cnt->mem_ticket, 1u);
      __syncthreads();
      const uint32_t item = (uint32_t)sc[SC_ITEM];
      if (item >= nin) break;
      const int32_t i = in[item];
      const int32_t li = list[i];
      const int32_t t0 = from_seeds ? li : li / 3;
      region_mem<REPAIR, NT>(R, i, t0, nhe, nv, twin, origin, wk, he, vtx, stage, stage_cap, arena, arena_cap, ps,
                             lane, lane_cap, kcap, lcap, sc, s_k1, s_k2, cnt);
      __syncthreads();
    }
  }
  // the last workgroup to finish sees every region queued for one lane
  if (tid == 0) {
    __threadfence();
    s_last = atomicAdd(&cnt->mem_done, 1u) == gridDim.x - 1;
  }
  __syncthreads();
  if (!s_last) return;
  __threadfence();
  const uint32_t n = __hip_atomic_load(&cnt->n_lane, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  for (uint32_t j = tid; j < n && (int64_t)j < lane_cap; j += NT) {
    const int32_t i = lane[j];
    const int32_t s = from_seeds ? seed_start(list[i], nhe, twin, he, cnt) : list[i];
    general_one<REPAIR>(i, s, nhe, nv, twin, origin, he, vtx, stage, stage_cap, arena, arena_cap, ps, cnt);
  }
}

// Scan and emission in one pass. A tile of kScanTile polygons (in seed order)
// sums its (pieces, vertices), gets its exclusive prefix by decoupled
// look-back and writes its part of the CSR output: offsets and start
// half-edges per output polygon (staged in LDS, stored coalesced), then the
// vertex range of the whole tile with all threads, each output slot finding
// its polygon by binary search in LDS so that the stores are coalesced.
// Blocks beyond the tile count exit before taking a ticket.
// BATCH: the group of a batched call writes the caller's output directly
// (`be`): int64 offsets after the earlier groups' totals, vertex ids and
// start half-edges less the base of the polygon's mesh (the mesh of its seed
// triangle), and the first output polygon of every mesh that has one.
constexpr int kScanItems = 4;
constexpr int kScanTile = 256 * kScanItems;
constexpr int kScanLog = 10;            // log2(kScanTile)
constexpr int kScanOut = kScanTile + 512;  // output polygons of a tile staged in LDS (else direct stores)
static_assert((1 << kScanLog) == kScanTile, "binary search depth");

// Mesh of group triangle t among meshes [lo, hi] of a batch group: the last
// m with he_off[m] - he_off[0] <= 3t.
__device__ __forceinline__ int64_t mesh_of_tri(const int64_t* __restrict__ he_off, int64_t lo, int64_t hi,
                                               int64_t t) {
  const int64_t x = 3 * t + he_off[0];
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) >> 1;
    if (he_off[mid] <= x) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

template <bool BATCH>
__global__ __launch_bounds__(256) void k_scan_emit(PolyState ps, uint64_t* status, const int32_t* __restrict__ stage,
                                                   const int32_t* __restrict__ arena, int32_t* __restrict__ offsets,
                                                   int32_t* __restrict__ verts, int32_t* __restrict__ start,
                                                   int64_t* __restrict__ counts, int64_t cap_polys,
                                                   int64_t cap_verts, Counters* cnt, BatchEmit be,
                                                   int32_t out_lds_max) {
  __shared__ int32_t s_voff[kScanTile + 1];
  __shared__ int32_t s_src[kScanTile];
  __shared__ uint8_t s_rot[kScanTile];
  __shared__ int32_t s_po[kScanOut];  // offsets of the tile's output polygons
  __shared__ int32_t s_ps[kScanOut];  // their start half-edges
  __shared__ int32_t s_vb[BATCH ? kScanTile : 1];  // vertex base of each polygon's mesh
  __shared__ int64_t s_mesh[2];                    // meshes of the tile's first and last polygon
  __shared__ int32_t s_ok;
  const uint32_t R = cnt->n_seeds;
  const uint32_t ntiles = (R + kScanTile - 1) / kScanTile;
  if (BATCH && be.base[2]) return;  // an earlier group failed: nothing more is written
  if (ntiles == 0) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      if constexpr (BATCH) {
        be.counts_g[0] = 0;
        be.counts_g[1] = 0;
      } else {
        counts[0] = 0;
        counts[1] = 0;
        offsets[0] = 0;
      }
    }
    return;
  }
  if (blockIdx.x >= ntiles) return;
  const uint32_t tile = take_tile(&cnt->tile_ticket[1]);
  const int64_t i0 = (int64_t)tile * kScanTile + (int64_t)threadIdx.x * kScanItems;
  int4 rc[kScanItems];
  uint32_t a = 0, b = 0;
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    const int64_t i = i0 + j;
    rc[j] = i < R ? ps.rec[i] : make_int4(0, 0, -1, 0);
    a += (uint32_t)(rc[j].y & kPiecesMask);
    b += (uint32_t)rc[j].x;
  }

  uint2 total;
  if (BATCH && threadIdx.x == 0) {
    // meshes of the tile's first and last polygon (meshes are contiguous in
    // seed order); published by the scan's barriers
    const int64_t t0 = (int64_t)tile * kScanTile;
    const int64_t t1 = min((int64_t)R, t0 + kScanTile) - 1;
    s_mesh[0] = mesh_of_tri(be.he_off, 0, be.nm - 1, be.seeds[t0]);
    s_mesh[1] = mesh_of_tri(be.he_off, s_mesh[0], be.nm - 1, be.seeds[t1]);
  }
  const uint2 pre = block_exclusive_scan<256>(a, b, &total);
  tile_publish(status, tile, total);
  // BATCH: the mesh of polygon i, its half-edge base, and whether it is the
  // first polygon of its mesh
  const int64_t mlo = BATCH ? s_mesh[0] : 0, mhi = BATCH ? s_mesh[1] : 0;
  const int64_t bh0 = BATCH ? be.he_off[0] : 0, bv0 = BATCH ? be.vtx_off[0] : 0;
  auto mesh_at = [&](int64_t i) -> int64_t {
    return mlo == mhi ? mlo : mesh_of_tri(be.he_off, mlo, mhi, be.seeds[i]);
  };
  uint32_t first_mask = 0;  // items that start their mesh
  // Tile-local staging before the look-back (so that it overlaps the wait
  // for earlier tiles): per input polygon its first vertex slot, staging
  // offset and rotation; per output polygon its tile-local vertex offset and
  // start half-edge.
  const bool fit = total.x <= (uint32_t)min(kScanOut, max(out_lds_max, 0));
  {
    uint32_t ra = pre.x, rb = pre.y;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
      const int64_t i = i0 + j;
      const int k = threadIdx.x * kScanItems + j;
      const int32_t nl = rc[j].x, np = rc[j].y & kPiecesMask, rot = (int32_t)((uint32_t)rc[j].y >> kRotShift);
      s_voff[k] = (int32_t)rb;
      s_src[k] = nl > 0 ? rc[j].w : 0;
      s_rot[k] = rot;
      int32_t hbj = 0;
      if constexpr (BATCH) {
        int32_t vbj = 0;
        if (i < R) {
          const int64_t m = mesh_at(i);
          const int64_t hm = be.he_off[m] - bh0;
          hbj = (int32_t)hm;
          vbj = (int32_t)(be.vtx_off[m] - bv0);
          if (i == 0 || 3 * (int64_t)be.seeds[i - 1] < hm) first_mask |= 1u << j;
        }
        s_vb[k] = vbj;
      }
      if (fit && i < R && np > 0) {
        if (np == 1) {
          s_po[ra] = (int32_t)rb;
          s_ps[ra] = rc[j].z - hbj;
        } else {
          const int32_t* rec = arena + ps.prec[i];
          int32_t acc = 0;
          for (int32_t q = 0; q < np; ++q) {
            s_po[ra + q] = (int32_t)rb + acc;
            s_ps[ra + q] = rec[4 * q + 2] - hbj;
            acc += rec[4 * q + 3];
          }
        }
      }
      ra += (uint32_t)np;
      rb += (uint32_t)nl;
    }
    if (threadIdx.x == 255) s_voff[kScanTile] = (int32_t)rb;
  }
  const uint2 ex = tile_lookback(status, tile, total, cnt, true);  // (its barriers publish the staging)
  const int64_t tile_v0 = ex.y, tile_v1 = (int64_t)ex.y + total.y;
  const int64_t tile_p1 = (int64_t)ex.x + total.x;
  // BATCH: positions in the caller's output (after the earlier groups)
  const int64_t P0 = BATCH ? be.base[0] : 0, S0 = BATCH ? be.base[1] : 0;
  int64_t* const off64 = be.offsets;
  int32_t* const vout = BATCH ? be.verts : verts;
  int32_t* const sout = BATCH ? be.start : start;
  if (threadIdx.x == 0) {
    if constexpr (BATCH)
      s_ok = (P0 + tile_p1 <= be.cap_polys && S0 + tile_v1 <= be.cap_verts && !cnt->error) ? 1 : 0;
    else
      s_ok = (tile_p1 <= cap_polys && tile_v1 <= cap_verts) ? 1 : 0;
  }
  if (tile == ntiles - 1 && threadIdx.x == 0) {
    if constexpr (BATCH) {
      be.counts_g[0] = tile_p1;  // (the closing offset: the next group, or the end of the call)
      be.counts_g[1] = tile_v1;
    } else {
      counts[0] = tile_p1;
      counts[1] = tile_v1;
      if (tile_p1 <= cap_polys) offsets[tile_p1] = (int32_t)tile_v1;
    }
  }
  __syncthreads();
  const bool ok = s_ok != 0;
  if (!ok && threadIdx.x == 0 && (!BATCH || !cnt->error)) set_error(cnt, POLYLLA_ECAPACITY);
  if (!ok) return;
  if constexpr (BATCH) {
    // first output polygon of each mesh whose first polygon is in this tile
    uint32_t ra = ex.x + pre.x;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
      const int32_t np = rc[j].y & kPiecesMask;
      if ((first_mask >> j) & 1u) be.poly_off[mesh_at(i0 + j)] = P0 + ra;
      ra += (uint32_t)np;
    }
  }
  if (fit) {
    for (uint32_t k = threadIdx.x; k < total.x; k += 256) {
      if constexpr (BATCH) off64[P0 + ex.x + k] = S0 + tile_v0 + s_po[k];
      else offsets[ex.x + k] = (int32_t)(tile_v0 + s_po[k]);
      if (sout) sout[P0 + ex.x + k] = s_ps[k];
    }
  } else {
    // more output polygons than the LDS staging holds: direct stores
    uint32_t ra = ex.x + pre.x, rb = pre.y;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
      const int64_t i = i0 + j;
      const int32_t nl = rc[j].x, np = rc[j].y & kPiecesMask;
      const int32_t hbj = (BATCH && i < R) ? (int32_t)(be.he_off[mesh_at(i)] - bh0) : 0;
      if (i < R && np > 0) {
        const int64_t vg = tile_v0 + rb;
        if (np == 1) {
          if constexpr (BATCH) off64[P0 + ra] = S0 + vg;
          else offsets[ra] = (int32_t)vg;
          if (sout) sout[P0 + ra] = rc[j].z - hbj;
        } else {
          const int32_t* rec = arena + ps.prec[i];
          int32_t acc = 0;
          for (int32_t q = 0; q < np; ++q) {
            if constexpr (BATCH) off64[P0 + ra + q] = S0 + vg + acc;
            else offsets[ra + q] = (int32_t)(vg + acc);
            if (sout) sout[P0 + ra + q] = rec[4 * q + 2] - hbj;
            acc += rec[4 * q + 3];
          }
        }
      }
      ra += (uint32_t)np;
      rb += (uint32_t)nl;
    }
  }
  // the tile's vertex range, coalesced: every slot finds its polygon by
  // binary search in LDS, eight independent searches in lockstep per thread;
  // the searches of the next eight slots run while the staging words of the
  // current ones are being loaded
  const int32_t nv_tile = (int32_t)total.y;
  auto locate = [&](int32_t k0, int32_t (&src)[8], int32_t (&vbs)[8]) {
    int lo[8], hi[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      lo[u] = 0;
      hi[u] = kScanTile;
    }
#pragma unroll
    for (int step = 0; step < kScanLog; ++step) {  // last polygon with s_voff <= k
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int mid = (lo[u] + hi[u]) >> 1;
        if (s_voff[mid] <= k0 + 256 * u) lo[u] = mid;
        else hi[u] = mid;
      }
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int32_t k = k0 + 256 * u;
      const int32_t len = s_voff[lo[u] + 1] - s_voff[lo[u]];
      int32_t off = k - s_voff[lo[u]] + s_rot[lo[u]];
      off = off >= len ? off - len : off;
      src[u] = k < nv_tile ? s_src[lo[u]] + off : -1;
      vbs[u] = BATCH ? s_vb[lo[u]] : 0;
    }
  };
  int32_t src[8], vbs[8], v[8];
  int32_t k0 = threadIdx.x;
  if (k0 < nv_tile) locate(k0, src, vbs);
  while (k0 < nv_tile) {
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = src[u] >= 0 ? stage[src[u]] - vbs[u] : 0;
    const int32_t k1 = k0 + 8 * 256;
    if (k1 < nv_tile) locate(k1, src, vbs);
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (k0 + 256 * u < nv_tile) vout[S0 + tile_v0 + k0 + 256 * u] = v[u];
    k0 = k1;
  }
}

// ---------------------------------------------------------------------------
// Batches (CSR of meshes with mesh-local indices). A group of consecutive
// meshes runs through the single-mesh kernels with indices over the group:
// k_group_rebase writes the group's twin and origin into scratch, and the
// emitter writes the group's polygons into the caller's int64 CSR with the
// mesh-local ids restored.

// Mesh of position x: the last m in [0, n) with off[m] <= x (off[0] <= x).
__device__ __forceinline__ int64_t mesh_of(const int64_t* __restrict__ off, int64_t n, int64_t x) {
  int64_t lo = 0, hi = n;
  while (hi - lo > 1) {
    const int64_t mid = (lo + hi) >> 1;
    if (off[mid] <= x) lo = mid;
    else hi = mid;
  }
  return lo;
}

// Group indices of the meshes [0, nm) of he_off / vtx_off (pointers at the
// group's first mesh). Local indices out of their mesh's range become
// out-of-range group indices, which the label kernels report as ETOPO
// (instead of silently naming a half-edge or vertex of a neighbouring mesh).
__global__ __launch_bounds__(256) void k_group_rebase(const int32_t* __restrict__ twin,
                                                      const int32_t* __restrict__ origin,
                                                      int32_t* __restrict__ tw_g, int32_t* __restrict__ or_g,
                                                      int64_t nm, const int64_t* __restrict__ he_off,
                                                      const int64_t* __restrict__ vtx_off) {
  const int64_t h0 = he_off[0], v0 = vtx_off[0];
  const int64_t H = he_off[nm] - h0;
  // each block takes one contiguous chunk, so a thread's mesh only moves
  // forward over the few meshes the chunk spans; the mesh's bases stay in
  // registers, and four elements per thread are loaded together
  constexpr int kU = 4;
  const int64_t step = (int64_t)blockDim.x * kU;
  const int64_t chunk = ((H + gridDim.x - 1) / gridDim.x + step - 1) / step * step;
  const int64_t c0 = (int64_t)blockIdx.x * chunk, c1 = min(H, c0 + chunk);
  if (c0 + threadIdx.x >= c1) return;
  int64_t m = mesh_of(he_off, nm, h0 + c0 + threadIdx.x);
  int64_t hb = he_off[m] - h0, he = he_off[m + 1] - h0, vb = vtx_off[m] - v0, vn = vtx_off[m + 1] - vtx_off[m];
  for (int64_t g = c0 + threadIdx.x; g < c1; g += step) {
    int32_t tw[kU], og[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int64_t h = g + (int64_t)blockDim.x * u;
      tw[u] = h < c1 ? twin[h0 + h] : -1;
      og[u] = h < c1 ? origin[h0 + h] : 0;
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int64_t h = g + (int64_t)blockDim.x * u;
      if (h >= c1) break;
      while (h >= he) {  // the next mesh (rarely more than one step)
        ++m;
        hb = he;
        he = he_off[m + 1] - h0;
        vb = vtx_off[m] - v0;
        vn = vtx_off[m + 1] - vtx_off[m];
      }
      const int64_t hn = he - hb;
      tw_g[h] = tw[u] == -1 ? -1 : ((tw[u] >= 0 && tw[u] < hn) ? (int32_t)(tw[u] + hb) : INT32_MIN);
      or_g[h] = (og[u] >= 0 && og[u] < vn) ? (int32_t)(og[u] + vb) : -1;
    }
  }
}

// base: {polygons, vertices} written by earlier groups, then a capacity
// failure flag. Cleared by k_batch_begin at the start of a call.
__global__ void k_batch_begin(int64_t* __restrict__ base) {
  if (threadIdx.x < 4) base[threadIdx.x] = 0;
}

// After a group: running totals; after the last group, the closing offset,
// the counts and the end of poly_off.
__global__ void k_group_advance(const int64_t* __restrict__ counts_g, int64_t* __restrict__ base, bool last,
                                int64_t n_meshes, int64_t* __restrict__ offsets, int64_t* __restrict__ poly_off,
                                int64_t* __restrict__ counts, int64_t cap_polys, int64_t cap_verts,
                                const Counters* cnt) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int64_t F = counts_g[0], S = counts_g[1];
  if (!base[2]) {
    if (cnt->error || F < 0 || base[0] + F > cap_polys || base[1] + S > cap_verts) base[2] = 1;
    base[0] += F;
    base[1] += S;
  }
  if (last) {
    counts[0] = base[0];
    counts[1] = base[1];
    if (!base[2]) {
      offsets[base[0]] = base[1];
      poly_off[n_meshes] = base[0];
    }
  }
}

// After a failed call (capacity or a device error): every first-polygon offset is -1.
__global__ __launch_bounds__(256) void k_batch_close(const int64_t* __restrict__ base, int64_t n_meshes,
                                                     int64_t* __restrict__ poly_off) {
  if (!base[2]) return;
  for (int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; m <= n_meshes; m += (int64_t)gridDim.x * blockDim.x)
    poly_off[m] = -1;
}

// First output polygon of the meshes of a group without triangles (the
// emitter writes it for the others): that of the next mesh with triangles,
// or the end of the group's polygons.
__global__ __launch_bounds__(256) void k_batch_empty(int64_t n_meshes, const int64_t* __restrict__ he_off,
                                                     const int64_t* __restrict__ base,
                                                     const int64_t* __restrict__ counts_g,
                                                     int64_t* __restrict__ poly_off, const Counters* cnt) {
  if (base[2] || cnt->error) return;  // (the call's end marks every first-polygon offset -1)
  for (int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; m < n_meshes; m += (int64_t)gridDim.x * blockDim.x) {
    const int64_t h = he_off[m];
    if (he_off[m + 1] != h) continue;
    // the first j > m with he_off[j] > h: mesh j - 1 is the next with triangles
    int64_t lo = m + 1, hi = n_meshes + 1;
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if (he_off[mid] > h) hi = mid;
      else lo = mid + 1;
    }
    poly_off[m] = lo <= n_meshes ? poly_off[lo - 1] : base[0] + counts_g[0];
  }
}

template __global__ void k_scan_emit<false>(PolyState, uint64_t*, const int32_t*, const int32_t*, int32_t*, int32_t*,
                                            int32_t*, int64_t*, int64_t, int64_t, Counters*, BatchEmit, int32_t);
template __global__ void k_scan_emit<true>(PolyState, uint64_t*, const int32_t*, const int32_t*, int32_t*, int32_t*,
                                           int32_t*, int64_t*, int64_t, int64_t, Counters*, BatchEmit, int32_t);
template __global__ void k_walk<true>(const int32_t*, int32_t, const int32_t*,
                                      int32_t*, int64_t, PolyState, int32_t*, int64_t, int, Counters*);
template __global__ void k_general_small<true>(const int32_t*, bool, int32_t, int64_t, const int32_t*,
                                               const int32_t*, const int32_t*, uint8_t*, uint8_t*, int32_t*,
                                               int64_t, int32_t*, int64_t, PolyState, const int32_t*,
                                               const uint32_t*, uint32_t, Counters*);
template __global__ void k_general_small<false>(const int32_t*, bool, int32_t, int64_t, const int32_t*,
                                                const int32_t*, const int32_t*, uint8_t*, uint8_t*, int32_t*,
                                                int64_t, int32_t*, int64_t, PolyState, const int32_t*,
                                                const uint32_t*, uint32_t, Counters*);
template __global__ void k_tip<true>(int32_t, int64_t, const int32_t*, const int32_t*, const int32_t*, uint8_t*, uint8_t*, int32_t*,
                                     int64_t, int32_t*, int64_t, PolyState, const int32_t*, int32_t*, int64_t,
                                     Counters*);
template __global__ void k_tip<false>(int32_t, int64_t, const int32_t*, const int32_t*, const int32_t*, uint8_t*, uint8_t*, int32_t*,
                                      int64_t, int32_t*, int64_t, PolyState, const int32_t*, int32_t*, int64_t,
                                      Counters*);
template __global__ void k_tip_long<true>(int32_t, int64_t, const int32_t*, const int32_t*, const int32_t*, uint8_t*,
                                           uint8_t*, int32_t*, int64_t, int32_t*, int64_t, PolyState, const int32_t*,
                                           int64_t, const uint32_t*, uint32_t, uint32_t, int32_t*, int64_t, uint32_t*,
                                           Counters*);
template __global__ void k_tip_long<false>(int32_t, int64_t, const int32_t*, const int32_t*, const int32_t*, uint8_t*,
                                           uint8_t*, int32_t*, int64_t, int32_t*, int64_t, PolyState, const int32_t*,
                                           int64_t, const uint32_t*, uint32_t, uint32_t, int32_t*, int64_t, uint32_t*,
                                           Counters*);
template __global__ void k_general_big<true, 64, 128, 128, 8>(
    const int32_t*, bool, int32_t, int64_t, const int32_t*, const int32_t*, const int32_t*, uint8_t*, uint8_t*,
    int32_t*, int64_t, int32_t*, int64_t, PolyState, const int32_t*, bool, int64_t, const uint32_t*, uint32_t*,
    int32_t*, int64_t, uint32_t*, const int32_t*, int64_t, const uint32_t*, uint32_t, uint32_t, int32_t, Counters*);
template __global__ void k_general_big<true, 1024, 4096, 4096, 13>(
    const int32_t*, bool, int32_t, int64_t, const int32_t*, const int32_t*, const int32_t*, uint8_t*, uint8_t*,
    int32_t*, int64_t, int32_t*, int64_t, PolyState, const int32_t*, bool, int64_t, const uint32_t*, uint32_t*,
    int32_t*, int64_t, uint32_t*, const int32_t*, int64_t, const uint32_t*, uint32_t, uint32_t, int32_t, Counters*);
template __global__ void k_general_big<false, 64, 128, 128, 8>(
    const int32_t*, bool, int32_t, int64_t, const int32_t*, const int32_t*, const int32_t*, uint8_t*, uint8_t*,
    int32_t*, int64_t, int32_t*, int64_t, PolyState, const int32_t*, bool, int64_t, const uint32_t*, uint32_t*,
    int32_t*, int64_t, uint32_t*, const int32_t*, int64_t, const uint32_t*, uint32_t, uint32_t, int32_t, Counters*);
template __global__ void k_general_big<false, 1024, 4096, 4096, 13>(
    const int32_t*, bool, int32_t, int64_t, const int32_t*, const int32_t*, const int32_t*, uint8_t*, uint8_t*,
    int32_t*, int64_t, int32_t*, int64_t, PolyState, const int32_t*, bool, int64_t, const uint32_t*, uint32_t*,
    int32_t*, int64_t, uint32_t*, const int32_t*, int64_t, const uint32_t*, uint32_t, uint32_t, int32_t, Counters*);
template __global__ void k_general_huge<true>(const int32_t*, bool, int32_t, int64_t, const int32_t*,
                                              const int32_t*, const int32_t*, uint8_t*, uint8_t*, int32_t*, int64_t,
                                              int32_t*, int64_t, PolyState, const int32_t*, int64_t, int32_t*,
                                              int64_t, int32_t*, int64_t, int32_t, int32_t, Counters*);
template __global__ void k_general_huge<false>(const int32_t*, bool, int32_t, int64_t, const int32_t*,
                                               const int32_t*, const int32_t*, uint8_t*, uint8_t*, int32_t*, int64_t,
                                               int32_t*, int64_t, PolyState, const int32_t*, int64_t, int32_t*,
                                               int64_t, int32_t*, int64_t, int32_t, int32_t, Counters*);

}  // namespace polylla
