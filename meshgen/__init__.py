"""Seeded synthetic triangulations shared by the oracle tests and the GPU path.

This package only draws points and triangulates them (Delaunay, exact lattice
predicates). It holds none of the meshing method's arithmetic.
"""
from .gen import (  # noqa: F401
    LATTICE_BITS,
    Mesh,
    build_native,
    mesh_from_points,
    mesh_from_triangles,
    pack_meshes,
    config_points,
    config_mesh,
    batch_sizes,
    batch_points,
    request_points,
    snap,
    serve_requests,
    validate,
)
