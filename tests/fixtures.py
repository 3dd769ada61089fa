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
    return mesh, g


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
