"""ctypes front end of the C oracle (test infrastructure only)."""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None
_lock = threading.Lock()

# label bits (the documented output layout)
HE = {"LONGEST": 1, "FRONTIER": 2, "TERMINAL": 4, "BORDER": 8, "BARRIER": 16, "REPAIRED": 32, "CONSTRAINED": 64}
TRI = {"SEED": 1}
VTX = {"TIP": 1}
STATS = ["seeds", "tip_polygons", "tips", "splits", "passes", "nonsimple_final",
         "maxlen_pre", "maxlen_final", "barrier_edges"]


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (single thread, no FP contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
                               "-shared", "-fPIC", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB):
                build()
            lib = ctypes.CDLL(_LIB)
            P = ctypes.c_void_p
            I = ctypes.c_int64
            lib.oracle_lepp.restype = ctypes.c_int
            lib.oracle_lepp.argtypes = [I, I, P, P, P, P, P, P, P]
            lib.oracle_mesh.restype = ctypes.c_int
            lib.oracle_mesh.argtypes = [I, I, P, P, P, P, P, P, P, P, P, P, P, P, P, P, P, P, I, I, P]
            _lib = lib
    return _lib


def _ptr(a):
    return a.ctypes.data if a is not None and a.size else None


def oracle_mesh(xy, twin, next_, origin, check: bool = True, fixed=None):
    """Run label -> traversal -> repair on one triangulation.

    `fixed` (uint8 per half-edge, nonzero on both half-edges of a segment of
    the input PSLG) may be None. Returns a dict with he/tri/vtx labels
    (uint8), the polygons before repair (pre_offsets, pre_verts, pre_start)
    and after (offsets, verts, start) as CSR int32 arrays of canonical CCW
    cycles, and a stats dict. Raises RuntimeError with the oracle's code when
    `check` and the call fails.
    """
    lib = _load()
    xy = np.ascontiguousarray(xy, dtype=np.float64)
    twin = np.ascontiguousarray(twin, dtype=np.int32)
    next_ = np.ascontiguousarray(next_, dtype=np.int32)
    origin = np.ascontiguousarray(origin, dtype=np.int32)
    fixed = None if fixed is None else np.ascontiguousarray(fixed, dtype=np.uint8)
    if fixed is not None and fixed.shape[0] != origin.shape[0]:
        raise ValueError("fixed must hold one byte per half-edge")
    nv = xy.shape[0]
    nhe = origin.shape[0]
    nt = nhe // 3
    cap_p = max(nt, 1)
    cap_v = max(3 * nt, 1)
    he = np.zeros(max(nhe, 1), np.uint8)
    tri = np.zeros(max(nt, 1), np.uint8)
    vtx = np.zeros(max(nv, 1), np.uint8)
    pre_off = np.zeros(cap_p + 1, np.int32)
    pre_verts = np.zeros(cap_v, np.int32)
    pre_start = np.zeros(cap_p, np.int32)
    pre_counts = np.zeros(2, np.int64)
    off = np.zeros(cap_p + 1, np.int32)
    verts = np.zeros(cap_v, np.int32)
    start = np.zeros(cap_p, np.int32)
    counts = np.zeros(2, np.int64)
    stats = np.zeros(len(STATS), np.int64)
    rc = lib.oracle_mesh(nv, nhe, _ptr(xy), _ptr(twin), _ptr(next_), _ptr(origin), _ptr(fixed),
                         he.ctypes.data, tri.ctypes.data, vtx.ctypes.data,
                         pre_off.ctypes.data, pre_verts.ctypes.data, pre_start.ctypes.data,
                         pre_counts.ctypes.data, off.ctypes.data, verts.ctypes.data,
                         start.ctypes.data, counts.ctypes.data, cap_p, cap_v, stats.ctypes.data)
    if rc != 0 and check:
        raise RuntimeError(f"oracle failed with code {rc}")
    Fp, Sp = int(pre_counts[0]), int(pre_counts[1])
    F, S = int(counts[0]), int(counts[1])
    return {
        "rc": rc,
        "he": he[:nhe], "tri": tri[:nt], "vtx": vtx[:nv],
        "pre_offsets": pre_off[:Fp + 1], "pre_verts": pre_verts[:Sp], "pre_start": pre_start[:Fp],
        "offsets": off[:F + 1], "verts": verts[:S], "start": start[:F],
        "stats": dict(zip(STATS, (int(x) for x in stats))),
    }


def oracle_on(mesh, check: bool = True):
    return oracle_mesh(mesh.xy, mesh.twin, mesh.next, mesh.origin, check=check,
                       fixed=getattr(mesh, "fixed", None))


def oracle_lepp(mesh, check: bool = True):
    """Longest-edge propagation path of every triangle: (terminal edge key,
    number of triangles) per triangle, as int32 arrays."""
    lib = _load()
    xy = np.ascontiguousarray(mesh.xy, dtype=np.float64)
    twin = np.ascontiguousarray(mesh.twin, dtype=np.int32)
    next_ = np.ascontiguousarray(mesh.next, dtype=np.int32)
    origin = np.ascontiguousarray(mesh.origin, dtype=np.int32)
    fixed = getattr(mesh, "fixed", None)
    fixed = None if fixed is None else np.ascontiguousarray(fixed, dtype=np.uint8)
    nt = origin.shape[0] // 3
    terminal = np.zeros(max(nt, 1), np.int32)
    length = np.zeros(max(nt, 1), np.int32)
    rc = lib.oracle_lepp(xy.shape[0], origin.shape[0], _ptr(xy), _ptr(twin), _ptr(next_), _ptr(origin),
                         _ptr(fixed), terminal.ctypes.data, length.ctypes.data)
    if rc != 0 and check:
        raise RuntimeError(f"oracle_lepp failed with code {rc}")
    return terminal[:nt], length[:nt]
