"""Seeded point sets and their Delaunay triangulations as half-edge arrays.

Layout of a triangulation (shared by every consumer):
  xy      float64 [V, 2]   vertex coordinates
  origin  int32   [H]      origin vertex of half-edge h; triangle t owns h = 3t, 3t+1, 3t+2 (CCW)
  next    int32   [H]      next[3t+i] = 3t + (i+1) % 3
  twin    int32   [H]      opposite half-edge of the same edge, -1 on the hull

Point recipe common to every workload: draw FP64 points with numpy's PCG64
generator, snap them to the lattice of multiples of 2^-28 in [0, 1] (so the
triangulator's predicates are exact in integer arithmetic), drop exact
duplicates keeping the first occurrence, number the vertices in Morton order
of their lattice coordinates, triangulate, then rotate each triangle to start
at its smallest vertex id and sort triangles by their first two vertex ids.
The resulting arrays depend only on the point set (for points in general
position the Delaunay triangulation is unique).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
import threading
from dataclasses import dataclass, field

import numpy as np

LATTICE_BITS = 28
_SCALE = float(1 << LATTICE_BITS)

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "delaunay.cpp")
_LIB = os.path.join(_HERE, "libmeshgen.so")
_lib = None
_lib_lock = threading.Lock()


def build_native(force: bool = False) -> str:
    """Compile the native triangulator (g++, host only)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _native():
    global _lib
    with _lib_lock:
        if _lib is None:
            if not os.path.exists(_LIB):
                build_native()
            lib = ctypes.CDLL(_LIB)
            lib.mg_delaunay_run.restype = ctypes.c_void_p
            lib.mg_delaunay_run.argtypes = [ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                            ctypes.POINTER(ctypes.c_int64),
                                            ctypes.POINTER(ctypes.c_int32)]
            lib.mg_delaunay_fetch.restype = None
            lib.mg_delaunay_fetch.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
            lib.mg_delaunay_free.restype = None
            lib.mg_delaunay_free.argtypes = [ctypes.c_void_p]
            _lib = lib
    return _lib


@dataclass
class Mesh:
    xy: np.ndarray          # float64 [V, 2]
    origin: np.ndarray      # int32 [H]
    twin: np.ndarray        # int32 [H]
    next: np.ndarray        # int32 [H]
    lattice: np.ndarray | None = None   # int64 [V, 2] lattice coordinates (None for hand meshes)
    meta: dict = field(default_factory=dict)
    fixed: np.ndarray | None = None     # uint8 [H], nonzero on both half-edges of a PSLG segment

    @property
    def n_vertices(self) -> int:
        return int(self.xy.shape[0])

    @property
    def n_halfedges(self) -> int:
        return int(self.origin.shape[0])

    @property
    def n_tri(self) -> int:
        return self.n_halfedges // 3

    def nbytes(self) -> int:
        return self.xy.nbytes + self.origin.nbytes + self.twin.nbytes + self.next.nbytes


def _grouped_next(n_he: int) -> np.ndarray:
    h = np.arange(n_he, dtype=np.int64)
    return (h - h % 3 + (h + 1) % 3).astype(np.int32)


def _part1by1(x: np.ndarray) -> np.ndarray:
    x = x.astype(np.uint64) & np.uint64(0xFFFFFFFF)
    x = (x | (x << np.uint64(16))) & np.uint64(0x0000FFFF0000FFFF)
    x = (x | (x << np.uint64(8))) & np.uint64(0x00FF00FF00FF00FF)
    x = (x | (x << np.uint64(4))) & np.uint64(0x0F0F0F0F0F0F0F0F)
    x = (x | (x << np.uint64(2))) & np.uint64(0x3333333333333333)
    x = (x | (x << np.uint64(1))) & np.uint64(0x5555555555555555)
    return x


def snap(points: np.ndarray) -> np.ndarray:
    """FP64 points in [0,1]^2 -> int64 lattice coordinates in [0, 2^28]."""
    q = np.rint(np.asarray(points, dtype=np.float64) * _SCALE)
    return np.clip(q, 0, _SCALE).astype(np.int64)


def mesh_from_points(points: np.ndarray, meta: dict | None = None, vertex_of: list | None = None) -> Mesh:
    """Snap, deduplicate, Morton-number and Delaunay-triangulate a point set.
    If `vertex_of` is a list, the vertex id of every input point (after
    deduplication: the id of the kept copy) is appended to it as an array."""
    lat = snap(points)
    code = (_part1by1(lat[:, 0]) << np.uint64(1)) | _part1by1(lat[:, 1])
    order = np.argsort(code, kind="stable")
    code_s = code[order]
    keep = np.ones(order.shape[0], dtype=bool)
    keep[1:] = code_s[1:] != code_s[:-1]
    if vertex_of is not None:
        vid = np.empty(order.shape[0], np.int64)
        vid[order] = np.cumsum(keep) - 1
        vertex_of.append(vid)
    lat = np.ascontiguousarray(lat[order[keep]])
    n = lat.shape[0]
    X = np.ascontiguousarray(lat[:, 0])
    Y = np.ascontiguousarray(lat[:, 1])
    lib = _native()
    ntri = ctypes.c_int64(0)
    status = ctypes.c_int32(0)
    h = lib.mg_delaunay_run(n, X.ctypes.data, Y.ctypes.data, ctypes.byref(ntri), ctypes.byref(status))
    if status.value != 0 or not h:
        raise RuntimeError(f"triangulation failed (status {status.value}, {n} points)")
    T = ntri.value
    origin = np.empty(3 * T, dtype=np.int32)
    twin = np.empty(3 * T, dtype=np.int32)
    lib.mg_delaunay_fetch(h, origin.ctypes.data, twin.ctypes.data)
    lib.mg_delaunay_free(h)
    xy = lat.astype(np.float64) / _SCALE
    m = dict(meta or {})
    m.update(n_points_drawn=int(points.shape[0]), n_duplicates=int(points.shape[0] - n))
    return Mesh(xy=xy, origin=origin, twin=twin, next=_grouped_next(3 * T), lattice=lat, meta=m)


def mesh_from_triangles(xy, tris, check_ccw: bool = True) -> Mesh:
    """Hand-built mesh: triangles given as vertex triples, kept in the given
    order and rotation (so half-edge indices are exactly 3t+i)."""
    xy = np.asarray(xy, dtype=np.float64).reshape(-1, 2)
    tris = np.asarray(tris, dtype=np.int64).reshape(-1, 3)
    T = tris.shape[0]
    V = xy.shape[0]
    origin = tris.reshape(-1).astype(np.int32)
    nxt = _grouped_next(3 * T)
    a = origin.astype(np.int64)
    b = origin[nxt].astype(np.int64)
    key = a * V + b
    rkey = b * V + a
    if np.unique(key).shape[0] != key.shape[0]:
        raise ValueError("a directed edge occurs twice (non-manifold or inconsistent orientation)")
    srt = np.argsort(key)
    pos = np.searchsorted(key[srt], rkey)
    pos = np.minimum(pos, key.shape[0] - 1)
    hit = key[srt][pos] == rkey
    twin = np.where(hit, srt[pos], -1).astype(np.int32)
    mesh = Mesh(xy=xy, origin=origin, twin=twin, next=nxt, lattice=None, meta={})
    if check_ccw:
        p0, p1, p2 = xy[tris[:, 0]], xy[tris[:, 1]], xy[tris[:, 2]]
        o = (p1[:, 0] - p0[:, 0]) * (p2[:, 1] - p0[:, 1]) - (p1[:, 1] - p0[:, 1]) * (p2[:, 0] - p0[:, 0])
        if np.any(o <= 0):
            raise ValueError("triangles must be counter-clockwise")
    return mesh


# --------------------------------------------------------------------------
# Workload recipes (all seeded)
# --------------------------------------------------------------------------

def _uniform(rng, n):
    return rng.random((n, 2))


def _clusters(rng, n, k, sigma):
    centres = rng.random((k, 2))
    per = [n // k + (1 if i < n % k else 0) for i in range(k)]
    parts = [rng.normal(centres[i], sigma, size=(per[i], 2)) for i in range(k)]
    return np.clip(np.concatenate(parts, axis=0), 0.0, 1.0)


def config_points(name: str) -> np.ndarray:
    """Point sets of the single-mesh workloads.

    uniform10k : 10,000 points uniform in [0,1]^2 (seed 1)
    mixed1m    : 500,000 uniform + 8 Gaussian clusters of 62,500 (sigma 0.02),
                 clipped to the square (seed 2)
    grid10m    : 3163 x 3163 jittered grid, jitter uniform +-0.45 cell (seed 3)
    Small variants for tests: uniform<N> (seed 1), mixed<N> (seed 2, same recipe
    scaled), grid<g>x (g x g jittered grid, seed 3).
    """
    if name.startswith("uniform"):
        n = _parse_count(name[len("uniform"):])
        return _uniform(np.random.default_rng(1), n)
    if name.startswith("mixed"):
        n = _parse_count(name[len("mixed"):])
        rng = np.random.default_rng(2)
        u = _uniform(rng, n // 2)
        c = _clusters(rng, n - n // 2, 8, 0.02)
        return np.concatenate([u, c], axis=0)
    if name.startswith("pslg"):
        raise KeyError("pslg workloads are meshes with segments: use config_mesh")
    if name.startswith("grid"):
        spec = name[len("grid"):]
        g = 3163 if spec == "10m" else int(spec.rstrip("x"))
        rng = np.random.default_rng(3)
        jit = rng.uniform(-0.45, 0.45, size=(g * g, 2))
        j, i = np.divmod(np.arange(g * g, dtype=np.float64), g)
        x = (i + 0.5 + jit[:, 0]) / g
        y = (j + 0.5 + jit[:, 1]) / g
        return np.stack([x, y], axis=1)
    raise KeyError(name)


def _parse_count(s: str) -> int:
    s = s.lower()
    mult = 1
    if s.endswith("k"):
        mult, s = 1000, s[:-1]
    elif s.endswith("m"):
        mult, s = 1000000, s[:-1]
    return int(float(s) * mult)


def config_mesh(name: str) -> Mesh:
    if name.startswith("pslg"):
        # pslg<N>: N uniform points, 8 holes, 6 cracks (seed 6)
        n = _parse_count(name[len("pslg"):])
        return pslg_mesh(n, 8, 6, seed=6)
    pts = config_points(name)
    return mesh_from_points(pts, meta={"workload": name})


def batch_sizes(n_meshes: int = 2000, lo: float = 3.0, hi: float = 6.0, seed: int = 4) -> np.ndarray:
    """Point counts of the batched workload: round(10^U(lo, hi)) (seed 4)."""
    rng = np.random.default_rng(seed)
    return np.rint(10.0 ** rng.uniform(lo, hi, size=n_meshes)).astype(np.int64)


def batch_points(m: int, n: int) -> np.ndarray:
    """Points of mesh m of the batched workload (seed 40000 + m)."""
    return _uniform(np.random.default_rng(40_000 + m), int(n))


def serve_requests(n_requests: int, rate: float, seed: int = 5, lo: float = 3.0,
                   hi: float = math.log10(2e6)):
    """Request stream of the serving workload: Poisson arrivals at `rate` per
    second, sizes round(10^U(lo, hi)), each request uniform or 4-cluster
    Gaussian (sigma 0.05) with probability 1/2. Returns a list of
    (arrival_time_s, n_points, kind, seed)."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=n_requests)
    sizes = np.rint(10.0 ** rng.uniform(lo, hi, size=n_requests)).astype(np.int64)
    kinds = rng.integers(0, 2, size=n_requests)
    t = np.cumsum(gaps) - gaps[0]
    return [(float(t[j]), int(sizes[j]), "cluster" if kinds[j] else "uniform", 50_000 + j)
            for j in range(n_requests)]


def request_points(n: int, kind: str, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    if kind == "uniform":
        return _uniform(rng, n)
    return _clusters(rng, n, 4, 0.05)


def pslg_mesh(n: int, n_holes: int, n_cracks: int, seed: int) -> Mesh:
    """A triangulation of a planar straight-line graph in [0,1]^2: n points
    uniform in the square, n_holes circular holes (radius U(0.03, 0.08)) and
    n_cracks straight segments (length U(0.1, 0.3)) inside the domain, all
    seeded. The holes' rims and the cracks are sampled at the mean point
    spacing s = 1/sqrt(n), and uniform points within s of them (or inside a
    hole) are dropped, so that consecutive samples have an empty diametral
    disk and their edge is in the Delaunay triangulation (a conforming
    triangulation, no edge insertion needed). Triangles with their centroid
    in a hole are removed (the rim becomes boundary); the crack edges are
    marked as segments in `fixed` (both half-edges)."""
    rng = np.random.default_rng(seed)
    sp = 1.0 / math.sqrt(max(n, 1))
    holes = []
    tries = 0
    while len(holes) < n_holes and tries < 10000:
        tries += 1
        c = rng.uniform(0.12, 0.88, 2)
        r = rng.uniform(0.03, 0.08)
        if all(np.hypot(*(c - c2)) > r + r2 + 6 * sp for c2, r2 in holes):
            holes.append((c, r))
    cracks = []
    tries = 0

    def seg_dist(p, a, b):
        ab = b - a
        t = np.clip(((p - a) @ ab) / (ab @ ab), 0.0, 1.0)
        return np.hypot(*((a + np.outer(t, ab) if p.ndim > 1 else a + t * ab) - p).T)

    while len(cracks) < n_cracks and tries < 10000:
        tries += 1
        a = rng.uniform(0.08, 0.92, 2)
        ang = rng.uniform(0, 2 * math.pi)
        L = rng.uniform(0.1, 0.3)
        b = a + L * np.array([math.cos(ang), math.sin(ang)])
        if not (0.05 < b[0] < 0.95 and 0.05 < b[1] < 0.95):
            continue
        samples = a + np.outer(np.linspace(0, 1, 64), b - a)
        if any(np.min(np.abs(np.hypot(*(samples - c).T) - r)) < 6 * sp or np.min(np.hypot(*(samples - c).T)) < r
               for c, r in holes):
            continue
        if any(np.min(seg_dist(samples, a2, b2)) < 6 * sp for a2, b2 in cracks):
            continue
        cracks.append((a, b))
    P = rng.random((n, 2))
    keep = np.ones(n, bool)
    for c, r in holes:
        keep &= np.hypot(*(P - c).T) > r + sp
    for a, b in cracks:
        keep &= seg_dist(P, a, b) > sp
    feats, chains = [P[keep]], []
    base = int(keep.sum())
    for c, r in holes:
        k = max(8, int(math.ceil(2 * math.pi * r / sp)))
        ang = 2 * math.pi * np.arange(k) / k
        feats.append(c + r * np.stack([np.cos(ang), np.sin(ang)], 1))
        chains.append((base, k, True))
        base += k
    for a, b in cracks:
        k = int(math.ceil(np.hypot(*(b - a)) / sp)) + 1
        feats.append(a + np.outer(np.linspace(0, 1, k), b - a))
        chains.append((base, k, False))
        base += k
    pts = np.concatenate(feats)
    vid_l = []
    mesh = mesh_from_points(pts, meta={"workload": f"pslg n={n} holes={len(holes)} cracks={len(cracks)} seed={seed}"},
                            vertex_of=vid_l)
    vid = vid_l[0]
    T = mesh.n_tri
    o = mesh.origin.astype(np.int64)
    h = np.arange(3 * T)
    nx = o[h - h % 3 + (h + 1) % 3]
    V = mesh.n_vertices
    key = o * V + nx
    order = np.argsort(key)
    skey = key[order]

    def half_edge(u, v):
        i = np.searchsorted(skey, u * V + v)
        if i >= skey.size or skey[i] != u * V + v:
            raise RuntimeError(f"PSLG edge ({u}, {v}) is missing from the triangulation")
        return int(order[i])

    seg_he = []
    for b0, k, closed in chains:
        ids = vid[b0:b0 + k]
        for j in range(k if closed else k - 1):
            u, v = int(ids[j]), int(ids[(j + 1) % k])
            seg_he.append((half_edge(u, v), half_edge(v, u), closed))
    # remove the triangles inside the holes, keeping triangle order
    cen = (mesh.xy[o[0::3]] + mesh.xy[o[1::3]] + mesh.xy[o[2::3]]) / 3.0
    inside = np.zeros(T, bool)
    for c, r in holes:
        inside |= np.hypot(*(cen - c).T) < r
    newt = np.cumsum(~inside) - 1
    hmap = np.where(np.repeat(~inside, 3), 3 * np.repeat(newt, 3) + h % 3, -1)
    kept = np.repeat(~inside, 3)
    origin = mesh.origin[kept]
    tw_old = mesh.twin[kept]
    twin = np.where(tw_old >= 0, hmap[np.maximum(tw_old, 0)], -1).astype(np.int32)
    fixed = np.zeros(3 * T, np.uint8)
    for h1, h2, closed in seg_he:
        if not closed:
            fixed[h1] = fixed[h2] = 1
    fixed = fixed[kept]
    T2 = int((~inside).sum())
    meta = dict(mesh.meta)
    meta.update(holes=len(holes), cracks=len(cracks), triangles_removed=int(inside.sum()))
    return Mesh(xy=mesh.xy, origin=np.ascontiguousarray(origin), twin=twin, next=_grouped_next(3 * T2),
                lattice=mesh.lattice, meta=meta, fixed=fixed)


def pack_meshes(meshes, with_next: bool = True):
    """Concatenate meshes into one packed CSR of meshes with global indices:
    returns (mesh, vtx_off, he_off) where mesh m owns vertices
    vtx_off[m]:vtx_off[m+1] and half-edges he_off[m]:he_off[m+1]. Without
    `with_next` the implied grouped next array is left out (None)."""
    V = np.array([m.n_vertices for m in meshes], dtype=np.int64)
    H = np.array([m.n_halfedges for m in meshes], dtype=np.int64)
    vtx_off = np.zeros(len(meshes) + 1, np.int64)
    he_off = np.zeros(len(meshes) + 1, np.int64)
    np.cumsum(V, out=vtx_off[1:])
    np.cumsum(H, out=he_off[1:])
    if he_off[-1] >= 2 ** 31 or vtx_off[-1] >= 2 ** 31:
        raise ValueError("packed batch exceeds 2^31 half-edges or vertices")
    xy = np.empty((int(vtx_off[-1]), 2), np.float64)
    origin = np.empty(int(he_off[-1]), np.int32)
    twin = np.empty(int(he_off[-1]), np.int32)
    for k, m in enumerate(meshes):
        a, b = int(he_off[k]), int(he_off[k + 1])
        xy[vtx_off[k]:vtx_off[k + 1]] = m.xy
        origin[a:b] = m.origin + np.int32(vtx_off[k])
        twin[a:b] = np.where(m.twin >= 0, m.twin + np.int32(a), -1)
    nxt = _grouped_next(int(he_off[-1])) if with_next else None
    packed = Mesh(xy=xy, origin=origin, twin=twin, next=nxt, lattice=None, meta={"n_meshes": len(meshes)})
    return packed, vtx_off, he_off


# --------------------------------------------------------------------------
# Validation of the half-edge layout
# --------------------------------------------------------------------------

def validate(mesh: Mesh) -> dict:
    """Check the layout contract; raises ValueError on the first violation.
    Returns counts (T, h = hull edges, referenced vertices)."""
    H = mesh.n_halfedges
    V = mesh.n_vertices
    if H % 3:
        raise ValueError("n_halfedges % 3 != 0")
    T = H // 3
    if not np.array_equal(mesh.next, _grouped_next(H)):
        raise ValueError("next is not grouped per triangle")
    o = mesh.origin.astype(np.int64)
    if o.size and (o.min() < 0 or o.max() >= V):
        raise ValueError("origin out of range")
    tw = mesh.twin.astype(np.int64)
    if tw.size and (tw.min() < -1 or tw.max() >= H):
        raise ValueError("twin out of range")
    inner = np.nonzero(tw >= 0)[0]
    if not np.array_equal(tw[tw[inner]], inner):
        raise ValueError("twin is not an involution")
    if np.any(tw[inner] == inner):
        raise ValueError("twin maps a half-edge to itself")
    nx = mesh.next.astype(np.int64)
    if not np.array_equal(o[tw[inner]], o[nx[inner]]):
        raise ValueError("twin endpoints do not match")
    tri = o.reshape(T, 3)
    if mesh.lattice is not None:
        P = mesh.lattice
        a, b, c = P[tri[:, 0]], P[tri[:, 1]], P[tri[:, 2]]
        orient = (b[:, 0] - a[:, 0]) * (c[:, 1] - a[:, 1]) - (b[:, 1] - a[:, 1]) * (c[:, 0] - a[:, 0])
    else:
        P = mesh.xy
        a, b, c = P[tri[:, 0]], P[tri[:, 1]], P[tri[:, 2]]
        orient = (b[:, 0] - a[:, 0]) * (c[:, 1] - a[:, 1]) - (b[:, 1] - a[:, 1]) * (c[:, 0] - a[:, 0])
    if np.any(orient <= 0):
        raise ValueError("a triangle is not counter-clockwise")
    h = int(np.count_nonzero(tw < 0))
    nref = int(np.unique(o).shape[0])
    return {"T": T, "hull_edges": h, "referenced_vertices": nref}


# --------------------------------------------------------------------------
# The point grid that polylla_gen_grid draws on the device, drawn on the host
# from the same counter-based generator (SplitMix64, Steele, Lea and Flood
# 2014), for checking the on-device triangulation against mesh_from_points.
# --------------------------------------------------------------------------

_M64 = np.uint64(0xFFFFFFFFFFFFFFFF)


def splitmix64(seed: int, k: np.ndarray) -> np.ndarray:
    """Output k of the SplitMix64 stream that starts at state `seed`."""
    with np.errstate(over="ignore"):
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + (np.asarray(k, dtype=np.uint64) + np.uint64(1)) * np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def counter_grid_points(g: int, jitter: float, seed: int) -> np.ndarray:
    """[g*g, 2] points of cell c = j g + i: ((i + 0.5 + jitter (2u - 1)) / g,
    (j + 0.5 + jitter (2w - 1)) / g), u and w the top 53 bits of outputs 2c
    and 2c + 1 as fractions in [0, 1)."""
    c = np.arange(g * g, dtype=np.uint64)
    u = (splitmix64(seed, 2 * c) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    w = (splitmix64(seed, 2 * c + np.uint64(1)) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    j, i = np.divmod(np.arange(g * g, dtype=np.int64), g)
    x = (i.astype(np.float64) + 0.5 + jitter * (2.0 * u - 1.0)) / g
    y = (j.astype(np.float64) + 0.5 + jitter * (2.0 * w - 1.0)) / g
    return np.stack([x, y], axis=1)


def tiled_grid_id(i, j, g: int, tile: int = 32):
    """Vertex id of grid point (i, j) in polylla_gen_grid's numbering: tiles
    of tile x tile points in row order, points row by row inside a tile."""
    i = np.asarray(i, dtype=np.int64)
    j = np.asarray(j, dtype=np.int64)
    tj, ti = j // tile, i // tile
    hj = np.minimum(tile, g - tile * tj)
    wi = np.minimum(tile, g - tile * ti)
    return tile * g * tj + tile * hj * ti + (j - tile * tj) * wi + (i - tile * ti)
