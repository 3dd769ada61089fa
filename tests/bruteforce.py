"""Definitional brute force for tiny triangulations (test-only).

Works from the triangle vertex triples and coordinates alone: edge adjacency
comes from matching vertex pairs (not from the twin/next arrays), regions from
union-find over internal edges, polygon boundaries from planar face tracing with
atan2-sorted edge directions, and the repair rule from angles about the tip
vertex. Nothing here is shared with the oracle or the GPU path.
"""
from __future__ import annotations

import math
from collections import defaultdict

import numpy as np

LONGEST, FRONTIER, TERMINAL, BORDER, BARRIER, REPAIRED, CONSTRAINED = 1, 2, 4, 8, 16, 32, 64


def _tris(mesh):
    return [tuple(int(x) for x in mesh.origin[3 * t:3 * t + 3]) for t in range(mesh.n_tri)]


def _sqlen(xy, a, b):
    dx = float(xy[b, 0]) - float(xy[a, 0])
    dy = float(xy[b, 1]) - float(xy[a, 1])
    return dx * dx + dy * dy


class Brute:
    def __init__(self, mesh):
        self.xy = np.asarray(mesh.xy, dtype=np.float64)
        self.tris = _tris(mesh)
        T = len(self.tris)
        self.T = T
        # directed edge (a, b) -> (triangle, local index)
        self.dedge = {}
        for t, (a, b, c) in enumerate(self.tris):
            for i, (u, v) in enumerate(((a, b), (b, c), (c, a))):
                self.dedge[(u, v)] = (t, i)
        # segments of the input PSLG, as undirected vertex pairs
        fx = getattr(mesh, "fixed", None)
        self.segments = set()
        if fx is not None:
            for t, tri in enumerate(self.tris):
                for i in range(3):
                    if fx[3 * t + i]:
                        self.segments.add(frozenset((tri[i], tri[(i + 1) % 3])))

    # ---- labels by definition -------------------------------------------------
    def mate(self, t, i):
        a = self.tris[t][i]
        b = self.tris[t][(i + 1) % 3]
        return self.dedge.get((b, a))

    def key(self, t, i):
        h = 3 * t + i
        m = self.mate(t, i)
        if m is None:
            return h
        return min(h, 3 * m[0] + m[1])

    def longest(self):
        out = []
        for t, tri in enumerate(self.tris):
            cand = []
            for i in range(3):
                L = _sqlen(self.xy, tri[i], tri[(i + 1) % 3])
                cand.append((-L, self.key(t, i), i))
            out.append(min(cand)[2])
        return out

    def labels(self):
        lg = self.longest()
        he = np.zeros(3 * self.T, np.uint8)
        seed = np.zeros(self.T, np.uint8)
        for t, tri in enumerate(self.tris):
            he[3 * t + lg[t]] |= LONGEST
            for i in range(3):
                m = self.mate(t, i)
                mine = lg[t] == i
                if m is None or frozenset((tri[i], tri[(i + 1) % 3])) in self.segments:
                    # a hull edge, or a side of a segment: bounds the domain
                    he[3 * t + i] |= (BORDER if m is None else CONSTRAINED) | FRONTIER
                    if mine:
                        he[3 * t + i] |= TERMINAL
                        seed[t] = 1
                    continue
                theirs = lg[m[0]] == m[1]
                if mine and theirs:
                    he[3 * t + i] |= TERMINAL
                    if t < m[0]:
                        seed[t] = 1
                if not mine and not theirs:
                    he[3 * t + i] |= FRONTIER
        return lg, he, seed

    def lepp(self):
        """Longest-edge propagation path of every triangle, by its definition:
        (terminal edge key, triangles on the path)."""
        lg = self.longest()
        out = []
        for t in range(self.T):
            cur, n = t, 1
            while True:
                i = lg[cur]
                a, b = self.tris[cur][i], self.tris[cur][(i + 1) % 3]
                m = self.mate(cur, i)
                if m is None or frozenset((a, b)) in self.segments:
                    out.append((3 * cur + i, n))
                    break
                n += 1
                if lg[m[0]] == m[1]:
                    out.append((min(3 * cur + i, 3 * m[0] + m[1]), n))
                    break
                cur = m[0]
        return out

    # ---- regions: union-find over internal edges ------------------------------
    def regions(self, frontier_of):
        parent = list(range(self.T))

        def find(x):
            while parent[x] != x:
                parent[x] = parent[parent[x]]
                x = parent[x]
            return x

        for t in range(self.T):
            for i in range(3):
                m = self.mate(t, i)
                if m is not None and not frontier_of(t, i):
                    ra, rb = find(t), find(m[0])
                    if ra != rb:
                        parent[ra] = rb
        return [find(t) for t in range(self.T)]

    # ---- face tracing ----------------------------------------------------------
    def _angle(self, a, b):
        return math.atan2(float(self.xy[b, 1] - self.xy[a, 1]), float(self.xy[b, 0] - self.xy[a, 0]))

    def faces(self, frontier_of):
        """Boundary cycles (vertex lists) of every region, region on the left."""
        comp = self.regions(frontier_of)
        out_edges = defaultdict(list)  # (region, vertex) -> [next vertex]
        edges = []
        for t, tri in enumerate(self.tris):
            for i in range(3):
                if frontier_of(t, i):
                    a, b = tri[i], tri[(i + 1) % 3]
                    out_edges[(comp[t], a)].append(b)
                    edges.append((comp[t], a, b))
        used = set()
        cycles = []
        for (r, a, b) in edges:
            if (r, a, b) in used:
                continue
            cyc = []
            cur = (a, b)
            while (r,) + cur not in used:
                used.add((r,) + cur)
                cyc.append(cur[0])
                u, v = cur
                back = self._angle(v, u)
                best, bd = None, None
                for x in out_edges[(r, v)]:
                    d = (back - self._angle(v, x)) % (2 * math.pi)
                    if d <= 1e-15:
                        d = 2 * math.pi
                    if bd is None or d < bd:
                        best, bd = x, d
                cur = (v, best)
            cycles.append((r, cyc))
        return comp, cycles

    # ---- the repair rule, simulated geometrically ------------------------------
    def spokes_clockwise(self, v, first):
        """Neighbours of v ordered clockwise starting at `first`."""
        nb = set()
        for (a, b) in self.dedge:
            if a == v:
                nb.add(b)
            if b == v:
                nb.add(a)
        a0 = self._angle(v, first)
        return sorted(nb, key=lambda x: ((a0 - self._angle(v, x)) % (2 * math.pi)))

    def mesh_pipeline(self):
        """Labels, pre-repair cycles and final cycles, by brute force."""
        lg, he, seed = self.labels()
        front = {(t, i) for t in range(self.T) for i in range(3) if he[3 * t + i] & FRONTIER}

        def fr(t, i):
            return (t, i) in front

        comp, pre = self.faces(fr)
        # barrier edges: both directions of one frontier edge on the same
        # boundary cycle before the repair; tips: v_b with v_a == v_c there
        barrier = np.zeros(3 * self.T, np.uint8)
        tipv = set()
        for _, c in pre:
            L = len(c)
            steps = {(c[k], c[(k + 1) % L]) for k in range(L)}
            for k in range(L):
                a, b = c[k], c[(k + 1) % L]
                if (b, a) in steps:
                    t, i = self.dedge[(a, b)]
                    barrier[3 * t + i] = BARRIER
                if L >= 3 and c[k] == c[(k + 2) % L]:
                    tipv.add(c[(k + 1) % L])
        extra = set()  # undirected frontier edges added by the repair

        def fr2(t, i):
            a, b = self.tris[t][i], self.tris[t][(i + 1) % 3]
            return (t, i) in front or frozenset((a, b)) in extra

        # pass loop: every polygon with a tip splits at its smallest tip
        while True:
            _, cyc = self.faces(fr2)
            changed = False
            for _, c in cyc:
                L = len(c)
                tips = [c[(k + 1) % L] for k in range(L) if L >= 3 and c[k] == c[(k + 2) % L]]
                if not tips:
                    continue
                v = min(tips)
                k = c.index(v)
                va = c[(k - 1) % L]
                order = self.spokes_clockwise(v, va)  # order[0] == va (barrier)
                d = len(order)
                e = order[d // 2]
                extra.add(frozenset((v, e)))
                changed = True
            if not changed:
                break
        _, final = self.faces(fr2)
        return {"longest": lg, "he": he, "seed": seed, "comp": comp, "barrier": barrier, "tips": tipv,
                "pre": [c for _, c in pre], "final": [c for _, c in final], "extra": extra}


def canonical(c):
    """Lexicographically smallest rotation of a cyclic vertex sequence."""
    L = len(c)
    return min(tuple(c[(r + k) % L] for k in range(L)) for r in range(L))


def csr_cycles(offsets, verts):
    return [tuple(int(x) for x in verts[offsets[i]:offsets[i + 1]]) for i in range(len(offsets) - 1)]
