"""Hand fixtures and small seeded meshes shared by the CPU and GPU tests."""
from __future__ import annotations

import glob
import json
import os

import numpy as np

from meshgen.gen import mesh_from_points, mesh_from_triangles

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def golden_names():
    return sorted(os.path.splitext(os.path.basename(p))[0] for p in glob.glob(os.path.join(GOLDEN, "*.json")))


def golden(name):
    with open(os.path.join(GOLDEN, name + ".json")) as f:
        g = json.load(f)
    mesh = mesh_from_triangles(np.array(g["xy"], dtype=np.float64), np.array(g["tris"]))
    if g.get("fixed"):
        mesh.fixed = fixed_from_pairs(mesh, g["fixed"])
    return mesh, g


def fixed_from_pairs(mesh, pairs):
    """Segment flags per half-edge (both half-edges of every listed vertex pair)."""
    want = {frozenset((int(a), int(b))) for a, b in pairs}
    o = mesh.origin
    h = np.arange(o.size)
    nxt = o[h - h % 3 + (h + 1) % 3]
    fixed = np.array([frozenset((int(a), int(b))) in want for a, b in zip(o, nxt)], dtype=np.uint8)
    return fixed


def random_mesh(seed: int, n: int, kind: str = "uniform"):
    """Tiny seeded Delaunay meshes of several point distributions."""
    rng = np.random.default_rng(seed)
    if kind == "uniform":
        P = rng.random((n, 2))
    elif kind == "cluster":
        c = rng.random((3, 2))
        P = np.clip(c[rng.integers(0, 3, n)] + rng.normal(0, 0.05, (n, 2)), 0, 1)
    elif kind == "grid":
        g = max(2, int(round(n ** 0.5)))
        j, i = np.divmod(np.arange(g * g), g)
        P = np.stack([(i + 0.5 + rng.uniform(-0.45, 0.45, g * g)) / g,
                      (j + 0.5 + rng.uniform(-0.45, 0.45, g * g)) / g], 1)
    elif kind == "lattice":
        # coarse integer lattice: many exactly equal edge lengths (ties)
        k = max(3, int(round(n ** 0.5)))
        pts = set()
        while len(pts) < min(n, k * k):
            pts.add((int(rng.integers(0, k)), int(rng.integers(0, k))))
        P = np.array(sorted(pts), dtype=np.float64) / k
    else:
        raise KeyError(kind)
    return mesh_from_points(P)


def empty_mesh():
    return mesh_from_triangles(np.zeros((0, 2)), np.zeros((0, 3), dtype=np.int64))


def permute_mesh(mesh, seed: int, block: int = 0, rotate: bool = True):
    """The same triangulation with its triangles renumbered and each triangle's
    half-edges rotated (a seeded relabelling, no geometry changes).

    block = 0 shuffles triangles uniformly (no index locality left); block > 0
    shuffles whole runs of `block` consecutive triangles, keeping locality
    inside each run. Returns (mesh, tri_map, rot): old triangle t becomes
    tri_map[t], and its half-edge 3t+i becomes 3*tri_map[t] + (i - rot[t]) % 3.
    """
    from meshgen.gen import Mesh
    T = mesh.n_tri
    rng = np.random.default_rng(seed)
    if block > 0:
        nb = (T + block - 1) // block
        order = np.concatenate([np.arange(b * block, min(T, (b + 1) * block)) for b in rng.permutation(nb)])
    else:
        order = rng.permutation(T)
    tri_map = np.empty(T, np.int64)
    tri_map[order] = np.arange(T)
    rot = rng.integers(0, 3, T) if rotate else np.zeros(T, np.int64)
    h = np.arange(3 * T, dtype=np.int64)
    t, i = np.divmod(h, 3)
    he_map = 3 * tri_map[t] + (i - rot[t]) % 3
    origin = np.empty(3 * T, np.int32)
    origin[he_map] = mesh.origin
    twin = np.full(3 * T, -1, np.int32)
    inner = mesh.twin >= 0
    twin[he_map[inner]] = he_map[mesh.twin[inner]]
    nxt = (h - h % 3 + (h + 1) % 3).astype(np.int32)
    out = Mesh(xy=mesh.xy, origin=origin, twin=twin, next=nxt, lattice=mesh.lattice, meta=dict(mesh.meta))
    return out, tri_map, rot


def spiral_fan(n):
    """n >= 7 triangles around vertex 0, spoke k (to vertex k+1) of length 1 +
    0.001 k, rims shorter than spokes: triangle i's longest edge is spoke i+1
    (spoke n-1 for the last),
    so Lepp(t_i) runs to spoke n-1: n - i triangles (2 for the last one),
    terminal key 3n - 4 (half-edge n -> 0 of triangle n-2)."""
    ang = 2 * np.pi * np.arange(n) / n
    r = 1.0 + 0.001 * np.arange(n)
    xy = np.concatenate([[[0.0, 0.0]], np.stack([r * np.cos(ang), r * np.sin(ang)], 1)])
    tris = [(0, i + 1, i + 2) for i in range(n - 1)] + [(0, n, 1)]
    return mesh_from_triangles(xy, tris)
