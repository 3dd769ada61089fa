"""Python binding of libpolylla (ctypes). Argument marshalling only: every step
of the mesher runs in the HIP kernels of the shared library. PyTorch provides
device memory and the current HIP stream.

There is no CPU fallback: loading fails loudly when the library is missing.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpolylla.so")

OK, EINVAL, ELAYOUT, ETOPO, ECAPACITY, ENOMEM, EHIP, EDEGEN, EINTERNAL, ETOOBIG = 0, -1, -2, -3, -4, -5, -6, -7, -8, -9
LONGEST, FRONTIER, TERMINAL, BORDER, BARRIER, REPAIRED, CONSTRAINED = 1, 2, 4, 8, 16, 32, 64
SEED, TIP = 1, 1
PARAM_WALK_CAP = 1
PARAM_WALK_BLOCKS = 2
PARAM_GEN_WAVE_MAX = 3
PARAM_REGION_LDS_MAX = 4
PARAM_REGION_MEM_MAX = 5
PARAM_BATCH_GROUP_HE = 6
PARAM_LONGEST_ITEMS = 7
PARAM_LONG_TIP_MIN = 8
PARAM_EMIT_LDS_MAX = 9
PROFILE_OFF, PROFILE_ALL, PROFILE_WALK = 0, 1, 2


class PolyllaError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: {strerror(code)} ({code})")
        self.code = code


class _Tri(ctypes.Structure):
    _fields_ = [("n_vertices", ctypes.c_int64), ("n_halfedges", ctypes.c_int64),
                ("xy", ctypes.c_void_p), ("twin", ctypes.c_void_p),
                ("next", ctypes.c_void_p), ("origin", ctypes.c_void_p), ("fixed", ctypes.c_void_p)]


class _Labels(ctypes.Structure):
    _fields_ = [("he", ctypes.c_void_p), ("tri", ctypes.c_void_p), ("vtx", ctypes.c_void_p)]


class _Polys(ctypes.Structure):
    _fields_ = [("offsets", ctypes.c_void_p), ("verts", ctypes.c_void_p), ("start", ctypes.c_void_p),
                ("counts", ctypes.c_void_p), ("cap_polys", ctypes.c_int64), ("cap_verts", ctypes.c_int64)]


class _Batch(ctypes.Structure):
    _fields_ = [("n_meshes", ctypes.c_int64), ("vtx_off", ctypes.c_void_p), ("he_off", ctypes.c_void_p),
                ("vtx_off_host", ctypes.c_void_p), ("he_off_host", ctypes.c_void_p), ("xy", ctypes.c_void_p),
                ("twin", ctypes.c_void_p), ("origin", ctypes.c_void_p), ("fixed", ctypes.c_void_p)]


class _BatchOut(ctypes.Structure):
    _fields_ = [("offsets", ctypes.c_void_p), ("verts", ctypes.c_void_p), ("start", ctypes.c_void_p),
                ("poly_off", ctypes.c_void_p), ("counts", ctypes.c_void_p), ("cap_polys", ctypes.c_int64),
                ("cap_verts", ctypes.c_int64)]


_lib = None


def load() -> ctypes.CDLL:
    """Load libpolylla.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2204_05438_amd.build` (there is no fallback)")
        lib = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        lib.polylla_ctx_create.argtypes = [ctypes.POINTER(P), ctypes.c_int]
        lib.polylla_ctx_destroy.argtypes = [P]
        lib.polylla_ctx_destroy.restype = None
        lib.polylla_reserve.argtypes = [P, ctypes.c_int64, ctypes.c_int64]
        lib.polylla_reserve_batch.argtypes = [P, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64]
        lib.polylla_label.argtypes = [P, ctypes.POINTER(_Tri), ctypes.POINTER(_Labels), P]
        lib.polylla_build.argtypes = [P, ctypes.POINTER(_Tri), ctypes.POINTER(_Labels), ctypes.POINTER(_Polys), P]
        lib.polylla_repair.argtypes = [P, ctypes.POINTER(_Tri), ctypes.POINTER(_Labels), ctypes.POINTER(_Polys),
                                       ctypes.POINTER(_Polys), P]
        lib.polylla_mesh.argtypes = [P, ctypes.POINTER(_Tri), ctypes.POINTER(_Labels), ctypes.POINTER(_Polys), P]
        lib.polylla_lepp.argtypes = [P, ctypes.POINTER(_Tri), P, P, P]
        lib.polylla_mesh_mixed.argtypes = [P, ctypes.POINTER(_Tri), P, P, P, ctypes.POINTER(_Polys),
                                           ctypes.POINTER(ctypes.c_double), P]
        lib.polylla_mesh_noalloc.argtypes = [P, ctypes.POINTER(_Tri), ctypes.POINTER(_Labels),
                                             ctypes.POINTER(_Polys), P]
        lib.polylla_validate.argtypes = [P, ctypes.POINTER(_Tri), P]
        lib.polylla_gen_grid.argtypes = [P, ctypes.c_int64, ctypes.c_double, ctypes.c_uint64, P, P, P,
                                         ctypes.c_int64, ctypes.POINTER(ctypes.c_int64),
                                         ctypes.POINTER(ctypes.c_int32), P]
        lib.polylla_mesh_batched.argtypes = [P, ctypes.POINTER(_Batch), ctypes.POINTER(_Labels),
                                             ctypes.POINTER(_BatchOut), P]
        lib.polylla_status.argtypes = [P, P]
        lib.polylla_stats.argtypes = [P, ctypes.POINTER(ctypes.c_int64), ctypes.c_int]
        lib.polylla_set_param.argtypes = [P, ctypes.c_int, ctypes.c_int64]
        lib.polylla_profile.argtypes = [P, ctypes.c_int]
        lib.polylla_profile_read.argtypes = [P, ctypes.c_char_p, ctypes.POINTER(ctypes.c_double),
                                             ctypes.POINTER(ctypes.c_int64), ctypes.c_int]
        lib.polylla_strerror.argtypes = [ctypes.c_int]
        lib.polylla_strerror.restype = ctypes.c_char_p
        for f in ("polylla_ctx_create", "polylla_reserve", "polylla_reserve_batch", "polylla_label", "polylla_build", "polylla_repair",
                  "polylla_mesh", "polylla_lepp", "polylla_mesh_mixed", "polylla_mesh_noalloc", "polylla_mesh_batched", "polylla_validate", "polylla_gen_grid", "polylla_status",
                  "polylla_stats", "polylla_set_param", "polylla_profile", "polylla_profile_read"):
            getattr(lib, f).restype = ctypes.c_int
        _lib = lib
    return _lib


def strerror(code: int) -> str:
    return load().polylla_strerror(int(code)).decode()


def _check(code: int, what: str):
    if code != OK:
        raise PolyllaError(code, what)


def np_u8(a):
    import numpy as np
    return np.ascontiguousarray(a, dtype=np.uint8)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


@dataclass
class Tri:
    """A triangulation resident on the device (see polylla.h for the layout)."""
    xy: torch.Tensor       # float64 [V, 2]
    twin: torch.Tensor     # int32 [H]
    next: torch.Tensor | None  # int32 [H]; only polylla_validate reads it
    origin: torch.Tensor   # int32 [H]
    fixed: torch.Tensor | None = None  # uint8 [H]: segments of an input planar straight-line graph

    @property
    def n_vertices(self):
        return int(self.xy.shape[0])

    @property
    def n_halfedges(self):
        return int(self.origin.shape[0])

    @property
    def n_tri(self):
        return self.n_halfedges // 3

    def c(self) -> _Tri:
        names = ("xy", "twin", "origin") + (("next",) if self.next is not None else ())
        for name in names:
            if not getattr(self, name).is_contiguous():
                raise ValueError(f"{name} must be contiguous")
        if self.xy.dtype != torch.float64 or any(getattr(self, n).dtype != torch.int32 for n in names[1:]):
            raise TypeError("xy must be float64 and twin/next/origin int32")
        if self.fixed is not None and (self.fixed.dtype != torch.uint8 or not self.fixed.is_contiguous()
                                       or self.fixed.shape[0] != self.n_halfedges):
            raise TypeError("fixed must be a contiguous uint8 tensor with one entry per half-edge")
        return _Tri(self.n_vertices, self.n_halfedges, self.xy.data_ptr(), self.twin.data_ptr(),
                    None if self.next is None else self.next.data_ptr(), self.origin.data_ptr(),
                    None if self.fixed is None else self.fixed.data_ptr())

    @staticmethod
    def from_mesh(mesh, device="cuda", with_next: bool = True) -> "Tri":
        """Copy a meshgen.Mesh (numpy arrays) to the device."""
        fx = getattr(mesh, "fixed", None)
        return Tri(xy=torch.from_numpy(mesh.xy).to(device).contiguous(),
                   twin=torch.from_numpy(mesh.twin).to(device),
                   next=torch.from_numpy(mesh.next).to(device) if with_next else None,
                   origin=torch.from_numpy(mesh.origin).to(device),
                   fixed=None if fx is None else torch.from_numpy(np_u8(fx)).to(device))


@dataclass
class Labels:
    he: torch.Tensor    # uint8 [H]
    tri: torch.Tensor   # uint8 [T]
    vtx: torch.Tensor   # uint8 [V]

    @staticmethod
    def empty(tri: Tri) -> "Labels":
        dev = tri.origin.device
        return Labels(he=torch.empty(tri.n_halfedges, dtype=torch.uint8, device=dev),
                      tri=torch.empty(tri.n_tri, dtype=torch.uint8, device=dev),
                      vtx=torch.empty(tri.n_vertices, dtype=torch.uint8, device=dev))

    def c(self) -> _Labels:
        return _Labels(self.he.data_ptr(), self.tri.data_ptr(), self.vtx.data_ptr())


@dataclass
class Polys:
    offsets: torch.Tensor   # int32 [cap_polys + 1]
    verts: torch.Tensor     # int32 [cap_verts]
    start: torch.Tensor | None
    counts: torch.Tensor    # int64 [2]

    @staticmethod
    def empty(tri: Tri, cap_polys: int | None = None, cap_verts: int | None = None, with_start=True) -> "Polys":
        dev = tri.origin.device
        T = tri.n_tri
        cp = T if cap_polys is None else cap_polys
        cv = 3 * T if cap_verts is None else cap_verts
        return Polys(offsets=torch.empty(cp + 1, dtype=torch.int32, device=dev),
                     verts=torch.empty(max(cv, 1), dtype=torch.int32, device=dev),
                     start=torch.empty(max(cp, 1), dtype=torch.int32, device=dev) if with_start else None,
                     counts=torch.zeros(2, dtype=torch.int64, device=dev))

    def c(self) -> _Polys:
        return _Polys(self.offsets.data_ptr(), self.verts.data_ptr(),
                      None if self.start is None else self.start.data_ptr(),
                      self.counts.data_ptr(), self.offsets.shape[0] - 1, self.verts.shape[0])

    def trimmed(self):
        """(offsets, verts, start) cut to the produced sizes (synchronises)."""
        F, S = (int(x) for x in self.counts.tolist())
        return (self.offsets[:F + 1], self.verts[:S],
                None if self.start is None else self.start[:F])


@dataclass
class Batch:
    """A batch of triangulations on the device, one after another with
    mesh-local indices (see polylla_batch in polylla.h)."""
    xy: torch.Tensor       # float64 [sum V, 2]
    twin: torch.Tensor     # int32 [sum H], local to each mesh
    origin: torch.Tensor   # int32 [sum H], local to each mesh
    vtx_off: torch.Tensor  # int64 [M + 1] on the device
    he_off: torch.Tensor   # int64 [M + 1] on the device
    vtx_off_host: torch.Tensor  # the same offsets on the host (int64, contiguous)
    he_off_host: torch.Tensor
    fixed: torch.Tensor | None = None  # uint8 [sum H]: segments of input planar straight-line graphs

    @property
    def n_meshes(self):
        return int(self.he_off_host.shape[0]) - 1

    @property
    def n_halfedges(self):
        return int(self.he_off_host[-1])

    @property
    def n_vertices(self):
        return int(self.vtx_off_host[-1])

    @property
    def n_tri(self):
        return self.n_halfedges // 3

    def c(self) -> _Batch:
        for name in ("xy", "twin", "origin", "vtx_off", "he_off"):
            t = getattr(self, name)
            if not t.is_cuda or not t.is_contiguous():
                raise ValueError(f"{name} must be a contiguous device tensor")
        for name in ("vtx_off_host", "he_off_host"):
            t = getattr(self, name)
            if t.is_cuda or not t.is_contiguous() or t.dtype != torch.int64:
                raise ValueError(f"{name} must be a contiguous int64 host tensor")
        if self.vtx_off.dtype != torch.int64 or self.he_off.dtype != torch.int64:
            raise TypeError("vtx_off and he_off must be int64")
        if self.xy.dtype != torch.float64 or self.twin.dtype != torch.int32 or self.origin.dtype != torch.int32:
            raise TypeError("xy must be float64 and twin/origin int32")
        if self.fixed is not None and (self.fixed.dtype != torch.uint8 or not self.fixed.is_contiguous()
                                       or self.fixed.shape[0] != self.n_halfedges):
            raise TypeError("fixed must be a contiguous uint8 tensor with one entry per half-edge")
        return _Batch(self.n_meshes, self.vtx_off.data_ptr(), self.he_off.data_ptr(),
                      self.vtx_off_host.data_ptr(), self.he_off_host.data_ptr(), self.xy.data_ptr(),
                      self.twin.data_ptr(), self.origin.data_ptr(),
                      None if self.fixed is None else self.fixed.data_ptr())

    @staticmethod
    def from_meshes(meshes, device="cuda") -> "Batch":
        """Copy meshgen meshes (numpy, local indices) into one device batch."""
        import numpy as np
        V = np.array([m.n_vertices for m in meshes], np.int64)
        H = np.array([m.n_halfedges for m in meshes], np.int64)
        vo = np.zeros(len(meshes) + 1, np.int64)
        ho = np.zeros(len(meshes) + 1, np.int64)
        np.cumsum(V, out=vo[1:])
        np.cumsum(H, out=ho[1:])
        xy = np.concatenate([m.xy for m in meshes]) if meshes else np.zeros((0, 2))
        tw = np.concatenate([m.twin for m in meshes]) if meshes else np.zeros(0, np.int32)
        og = np.concatenate([m.origin for m in meshes]) if meshes else np.zeros(0, np.int32)
        vh, hh = torch.from_numpy(vo), torch.from_numpy(ho)
        fixed = None
        if any(getattr(m, "fixed", None) is not None for m in meshes):
            fixed = np.concatenate([np_u8(m.fixed) if getattr(m, "fixed", None) is not None
                                    else np.zeros(m.n_halfedges, np.uint8) for m in meshes])
        return Batch(xy=torch.from_numpy(np.ascontiguousarray(xy)).to(device),
                     twin=torch.from_numpy(tw).to(device), origin=torch.from_numpy(og).to(device),
                     vtx_off=vh.to(device), he_off=hh.to(device), vtx_off_host=vh, he_off_host=hh,
                     fixed=None if fixed is None else torch.from_numpy(fixed).to(device))


@dataclass
class BatchOut:
    offsets: torch.Tensor   # int64 [cap_polys + 1]
    verts: torch.Tensor     # int32 [cap_verts], mesh-local vertex ids
    start: torch.Tensor | None  # int32 [cap_polys], mesh-local half-edge ids
    poly_off: torch.Tensor  # int64 [M + 1]
    counts: torch.Tensor    # int64 [2]

    @staticmethod
    def empty(batch: Batch, cap_polys: int | None = None, cap_verts: int | None = None,
              with_start=True) -> "BatchOut":
        dev = batch.twin.device
        T = batch.n_tri
        cp = T if cap_polys is None else cap_polys
        cv = 3 * T if cap_verts is None else cap_verts
        return BatchOut(offsets=torch.empty(cp + 1, dtype=torch.int64, device=dev),
                        verts=torch.empty(max(cv, 1), dtype=torch.int32, device=dev),
                        start=torch.empty(max(cp, 1), dtype=torch.int32, device=dev) if with_start else None,
                        poly_off=torch.empty(batch.n_meshes + 1, dtype=torch.int64, device=dev),
                        counts=torch.zeros(2, dtype=torch.int64, device=dev))

    def c(self) -> _BatchOut:
        return _BatchOut(self.offsets.data_ptr(), self.verts.data_ptr(),
                         None if self.start is None else self.start.data_ptr(), self.poly_off.data_ptr(),
                         self.counts.data_ptr(), self.offsets.shape[0] - 1, self.verts.shape[0])

    def trimmed(self):
        """(offsets, verts, start, poly_off) cut to the produced sizes (synchronises)."""
        F, S = (int(x) for x in self.counts.tolist())
        return (self.offsets[:F + 1], self.verts[:S], None if self.start is None else self.start[:F],
                self.poly_off)


class Context:
    """A libpolylla context on one device; calls run on torch's current stream."""

    def __init__(self, device: int = 0):
        lib = load()
        h = ctypes.c_void_p()
        _check(lib.polylla_ctx_create(ctypes.byref(h), int(device)), "polylla_ctx_create")
        self._h = h
        self.device = device

    def close(self):
        if getattr(self, "_h", None):
            load().polylla_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def _stream():
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)

    def reserve(self, n_halfedges: int, n_vertices: int):
        _check(load().polylla_reserve(self._h, int(n_halfedges), int(n_vertices)), "polylla_reserve")

    def reserve_batch(self, n_halfedges: int, n_vertices: int, n_meshes: int):
        _check(load().polylla_reserve_batch(self._h, int(n_halfedges), int(n_vertices), int(n_meshes)),
               "polylla_reserve_batch")

    def label(self, tri: Tri, labels: Labels | None = None) -> Labels:
        labels = labels or Labels.empty(tri)
        t, l = tri.c(), labels.c()
        _check(load().polylla_label(self._h, ctypes.byref(t), ctypes.byref(l), self._stream()), "polylla_label")
        return labels

    def build(self, tri: Tri, labels: Labels, out: Polys | None = None) -> Polys:
        out = out or Polys.empty(tri)
        t, l, o = tri.c(), labels.c(), out.c()
        _check(load().polylla_build(self._h, ctypes.byref(t), ctypes.byref(l), ctypes.byref(o), self._stream()),
               "polylla_build")
        return out

    def repair(self, tri: Tri, labels: Labels, polys_in: Polys, out: Polys | None = None) -> Polys:
        out = out or Polys.empty(tri)
        t, l, i, o = tri.c(), labels.c(), polys_in.c(), out.c()
        _check(load().polylla_repair(self._h, ctypes.byref(t), ctypes.byref(l), ctypes.byref(i),
                                     ctypes.byref(o), self._stream()), "polylla_repair")
        return out

    def mesh(self, tri: Tri, labels: Labels | None = None, out: Polys | None = None) -> Polys:
        out = out or Polys.empty(tri)
        t, o = tri.c(), out.c()
        lp = ctypes.byref(labels.c()) if labels is not None else None
        _check(load().polylla_mesh(self._h, ctypes.byref(t), lp, ctypes.byref(o), self._stream()), "polylla_mesh")
        return out

    def lepp(self, tri: Tri):
        """polylla_lepp: (terminal edge key, triangles on the path) of every
        triangle's longest-edge propagation path, int32 device tensors."""
        T = tri.n_tri
        dev = tri.origin.device
        terminal = torch.empty(max(T, 1), dtype=torch.int32, device=dev)
        length = torch.empty(max(T, 1), dtype=torch.int32, device=dev)
        t = tri.c()
        _check(load().polylla_lepp(self._h, ctypes.byref(t), _ptr(terminal), _ptr(length), self._stream()),
               "polylla_lepp")
        return terminal[:T], length[:T]

    def mesh_mixed(self, tri: Tri, twin_host, origin_host):
        """polylla_mesh_mixed: label and traversal on the device, repair on the
        host. twin_host/origin_host: host int32 arrays (numpy) equal to the
        device ones. Returns (offsets, verts, start, he, seconds) as numpy
        arrays and a dict of the three phase times."""
        import numpy as np
        H, T = tri.n_halfedges, tri.n_tri
        tw = np.ascontiguousarray(twin_host, dtype=np.int32)
        og = np.ascontiguousarray(origin_host, dtype=np.int32)
        if tw.size != H or og.size != H:
            raise ValueError("host twin/origin must match the device triangulation")
        he = np.empty(max(H, 1), np.uint8)
        off = np.empty(T + 1, np.int32)
        verts = np.empty(max(3 * T, 1), np.int32)
        start = np.empty(max(T, 1), np.int32)
        counts = np.zeros(2, np.int64)
        secs = (ctypes.c_double * 3)()
        out = _Polys(off.ctypes.data, verts.ctypes.data, start.ctypes.data, counts.ctypes.data, T, 3 * T)
        t = tri.c()
        _check(load().polylla_mesh_mixed(self._h, ctypes.byref(t), ctypes.c_void_p(tw.ctypes.data),
                                         ctypes.c_void_p(og.ctypes.data), ctypes.c_void_p(he.ctypes.data),
                                         ctypes.byref(out), secs, self._stream()), "polylla_mesh_mixed")
        F, S = int(counts[0]), int(counts[1])
        return (off[:F + 1], verts[:S], start[:F], he[:H],
                {"device_s": secs[0], "copy_s": secs[1], "host_repair_s": secs[2]})

    def mesh_noalloc(self, tri: Tri, labels: Labels | None, out: Polys) -> Polys:
        """polylla_mesh_noalloc: scratch in the library's static array; `out`
        must be given (nothing is allocated)."""
        t, o = tri.c(), out.c()
        lp = ctypes.byref(labels.c()) if labels is not None else None
        _check(load().polylla_mesh_noalloc(self._h, ctypes.byref(t), lp, ctypes.byref(o), self._stream()),
               "polylla_mesh_noalloc")
        return out

    def mesh_batched(self, batch: Batch, labels: Labels | None = None, out: BatchOut | None = None) -> BatchOut:
        """polylla_mesh_batched over a Batch (mesh-local indices, int64 offsets)."""
        out = out or BatchOut.empty(batch)
        b, o = batch.c(), out.c()
        lp = ctypes.byref(labels.c()) if labels is not None else None
        _check(load().polylla_mesh_batched(self._h, ctypes.byref(b), lp, ctypes.byref(o), self._stream()),
               "polylla_mesh_batched")
        return out

    def gen_grid(self, g: int, jitter: float = 0.45, seed: int = 3, with_next: bool = False):
        """polylla_gen_grid: the Delaunay triangulation of a jittered g x g
        grid, generated on the device. Returns (Tri, flip rounds)."""
        dev = torch.device("cuda", self.device)
        n = g * g if 2 <= g <= 18000 else 1  # the library rejects other sizes
        xy = torch.empty((n, 2), dtype=torch.float64, device=dev)
        cap = 6 * n
        twin = torch.empty(cap, dtype=torch.int32, device=dev)
        origin = torch.empty(cap, dtype=torch.int32, device=dev)
        n_he = ctypes.c_int64(0)
        rounds = ctypes.c_int32(0)
        _check(load().polylla_gen_grid(self._h, int(g), float(jitter), int(seed) & (2 ** 64 - 1), _ptr(xy),
                                       _ptr(twin), _ptr(origin), cap, ctypes.byref(n_he), ctypes.byref(rounds),
                                       self._stream()), "polylla_gen_grid")
        H = n_he.value
        nxt = None
        if with_next:
            h = torch.arange(H, dtype=torch.int32, device=dev)
            nxt = h - h % 3 + (h + 1) % 3
        return Tri(xy=xy, twin=twin[:H], next=nxt, origin=origin[:H]), rounds.value

    def validate(self, tri: Tri) -> int:
        t = tri.c()
        return load().polylla_validate(self._h, ctypes.byref(t), self._stream())

    def status(self, raise_on_error: bool = True) -> int:
        code = load().polylla_status(self._h, self._stream())
        if raise_on_error:
            _check(code, "device")
        return code

    def stats(self) -> dict:
        buf = (ctypes.c_int64 * 7)()
        n = load().polylla_stats(self._h, buf, 7)
        keys = ["seeds", "general_small", "tips", "splits", "general_big", "fallback", "lane"]
        return {k: int(buf[i]) for i, k in enumerate(keys[:n])}

    def set_param(self, param: int, value: int):
        _check(load().polylla_set_param(self._h, int(param), int(value)), "polylla_set_param")

    def profile(self, enable, walk_only: bool = False):
        """Start (clearing earlier records) or stop per-kernel event timing;
        walk_only times the walk kernel alone."""
        mode = (PROFILE_WALK if walk_only else PROFILE_ALL) if enable else PROFILE_OFF
        _check(load().polylla_profile(self._h, mode), "polylla_profile")

    def profile_read(self) -> dict:
        """{kernel name: (summed ms, launches)} of the recorded launches."""
        n = 32
        names = ctypes.create_string_buffer(32 * n)
        ms = (ctypes.c_double * n)()
        cnt = (ctypes.c_int64 * n)()
        w = load().polylla_profile_read(self._h, names, ms, cnt, n)
        if w < 0:
            _check(w, "polylla_profile_read")
        raw = names.raw
        out = {}
        for i in range(w):
            nm = raw[32 * i:32 * i + 32].split(b"\0", 1)[0].decode()
            out[nm] = (float(ms[i]), int(cnt[i]))
        return out
