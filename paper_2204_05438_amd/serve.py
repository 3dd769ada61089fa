"""Serving loop: continuous batching of triangulation requests on one GPU.

Requests (a triangulation each, local indices, arrays in pinned host memory)
arrive over time. The loop
  * admits them in arrival order while their resident input bytes fit the
    device-memory budget: admission starts the host-to-device copy on an
    admission stream, and the meshes stay resident until their results are
    back on the host;
  * keeps `slots` independent contexts, each with its own stream and packed
    buffers; whenever a slot is idle it takes every admitted request not yet
    started (up to its triangle and mesh capacity), packs them on the device
    (device-to-device copies; indices stay local to each mesh) and runs ONE
    polylla_mesh_batched over the batch, so requests that arrive while other
    batches are on the GPU join the next free slot and their work overlaps
    with the running batches on the device;
  * checks the batch's device status once it is done: a batch with an error
    (a request that is not a valid triangulation) is served again one request
    at a time, so only the bad request fails (`error` set, no polygons);
  * copies each batch's polygons back (sizes first, then exactly the produced
    CSR) and splits them per request.
A request may also name its input instead of carrying it: a jittered g x g
grid (g, jitter, seed) is triangulated on the device after admission
(polylla_gen_grid, by a generator thread with its own context and stream, so
the loop keeps dispatching batches meanwhile), and nothing crosses PCIe on
the way in.
Latency of a request = results on the host - arrival, split into admission
wait, queueing after admission and service (pack + mesh + copy back).
"""
from __future__ import annotations

import collections
import dataclasses
import queue
import threading
import time

import numpy as np
import torch

from . import lib


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float        # seconds after the start of the run
    xy: torch.Tensor | None      # float64 [V, 2], pinned host memory (None: generated on the device)
    twin: torch.Tensor | None    # int32 [H], pinned, local indices
    origin: torch.Tensor | None  # int32 [H], pinned, local indices
    gen: tuple | None = None     # (g, jitter, seed): input generated on the device at admission
    admitted: float | None = None
    started: float | None = None
    done: float | None = None
    offsets: np.ndarray | None = None  # result: local CSR
    verts: np.ndarray | None = None
    error: int = 0                     # library error code of a request that could not be served
    alone: bool = False                # served in a batch of its own (after its batch failed)
    _dev: tuple | None = None
    _ready: torch.cuda.Event | None = None
    _charged: int = 0                  # bytes charged to the admission budget
    _size: tuple | None = None         # (vertices, half-edges) of a generated input

    @property
    def n_vertices(self) -> int:
        if self.xy is not None:
            return int(self.xy.shape[0])
        return self._size[0] if self._size else self.gen[0] * self.gen[0]

    @property
    def n_halfedges(self) -> int:
        if self.origin is not None:
            return int(self.origin.shape[0])
        # a grid not generated yet: its bound, 3 (2 g^2 - 5) < 6 g^2
        return self._size[1] if self._size else 6 * self.gen[0] * self.gen[0]

    @property
    def n_tri(self) -> int:
        return self.n_halfedges // 3

    def input_bytes(self) -> int:
        return 16 * self.n_vertices + 8 * self.n_halfedges

    @staticmethod
    def from_mesh(rid: int, arrival: float, mesh) -> "Request":
        return Request(rid, arrival, torch.from_numpy(mesh.xy).pin_memory(),
                       torch.from_numpy(mesh.twin).pin_memory(), torch.from_numpy(mesh.origin).pin_memory())

    @staticmethod
    def from_grid(rid: int, arrival: float, g: int, jitter: float = 0.45, seed: int = 0) -> "Request":
        """A request whose input is the Delaunay triangulation of a jittered
        g x g grid, generated on the device when it is admitted."""
        return Request(rid, arrival, None, None, None, gen=(int(g), float(jitter), int(seed)))


class _Slot:
    IDLE, COMPUTE, COPY = range(3)

    def __init__(self, device: int, max_tri: int, max_vert: int, max_meshes: int):
        dev = torch.device("cuda", device)
        self.ctx = lib.Context(device)
        self.stream = torch.cuda.Stream(dev)
        self.max_tri, self.max_vert, self.max_meshes = max_tri, max_vert, max_meshes
        self.xy = torch.empty((max_vert, 2), dtype=torch.float64, device=dev)
        self.twin = torch.empty(3 * max_tri, dtype=torch.int32, device=dev)
        self.origin = torch.empty(3 * max_tri, dtype=torch.int32, device=dev)
        self.offsets = torch.empty(max_tri + 1, dtype=torch.int64, device=dev)
        self.verts = torch.empty(3 * max_tri, dtype=torch.int32, device=dev)
        self.counts = torch.zeros(2, dtype=torch.int64, device=dev)
        self.poly_off = torch.empty(max_meshes + 1, dtype=torch.int64, device=dev)
        self.offs = torch.empty((2, max_meshes + 1), dtype=torch.int64, device=dev)  # he_off, vtx_off
        self.h_offs = torch.empty((2, max_meshes + 1), dtype=torch.int64).pin_memory()
        self.h_counts = torch.empty(2, dtype=torch.int64).pin_memory()
        self.h_poly_off = torch.empty(max_meshes + 1, dtype=torch.int64).pin_memory()
        self.h_offsets = torch.empty(max_tri + 1, dtype=torch.int64).pin_memory()
        self.h_verts = torch.empty(3 * max_tri, dtype=torch.int32).pin_memory()
        self.state = _Slot.IDLE
        self.batch: list[Request] = []
        self.event = None
        self.failed = 0
        # scratch for a full slot, so that batches allocate nothing
        self.ctx.reserve_batch(3 * max_tri, max_vert, max_meshes)

    def _run(self, n: int, Ht: int, Vt: int):
        offs = self.h_offs
        batch = lib.Batch(xy=self.xy[:Vt], twin=self.twin[:Ht], origin=self.origin[:Ht],
                          vtx_off=self.offs[1, :n + 1], he_off=self.offs[0, :n + 1],
                          vtx_off_host=offs[1, :n + 1], he_off_host=offs[0, :n + 1])
        out = lib.BatchOut(offsets=self.offsets[:Ht // 3 + 1], verts=self.verts[:Ht], start=None,
                           poly_off=self.poly_off[:n + 1], counts=self.counts)
        self.ctx.mesh_batched(batch, None, out)

    def launch(self, batch: list[Request]):
        n = len(batch)
        V = np.fromiter((r.n_vertices for r in batch), np.int64, n)
        H = np.fromiter((r.n_halfedges for r in batch), np.int64, n)
        offs = self.h_offs.numpy()
        offs[:, 0] = 0
        np.cumsum(H, out=offs[0, 1:n + 1])
        np.cumsum(V, out=offs[1, 1:n + 1])
        Ht, Vt = int(offs[0, n]), int(offs[1, n])
        with torch.cuda.stream(self.stream):
            for r in batch:
                self.stream.wait_event(r._ready)
            self.offs[:, :n + 1].copy_(self.h_offs[:, :n + 1], non_blocking=True)
            for k, r in enumerate(batch):
                dxy, dtw, dor = r._dev
                a, b, va, vb = int(offs[0, k]), int(offs[0, k + 1]), int(offs[1, k]), int(offs[1, k + 1])
                self.xy[va:vb].copy_(dxy)
                self.twin[a:b].copy_(dtw)
                self.origin[a:b].copy_(dor)
            self._run(n, Ht, Vt)
            self.h_counts.copy_(self.counts, non_blocking=True)
            self.h_poly_off[:n + 1].copy_(self.poly_off[:n + 1], non_blocking=True)
            self.event = torch.cuda.Event()
            self.event.record(self.stream)
        self.batch = batch
        self.state = _Slot.COMPUTE

    def copy_back(self):
        """The batch is done: read its device status, then copy exactly the
        produced polygons back. Returns False (nothing copied) when the
        batch failed; its requests are then in self.batch with the code in
        self.failed."""
        code = self.ctx.status(raise_on_error=False)
        n = len(self.batch)
        if code == lib.OK and int(self.h_poly_off[0]) < 0:
            code = lib.ECAPACITY  # every first-polygon offset is -1 after a capacity failure
        if code != lib.OK:
            self.failed = code
            return False
        F, S = (int(x) for x in self.h_counts.tolist())
        assert int(self.h_poly_off[n]) == F
        with torch.cuda.stream(self.stream):
            self.h_offsets[:F + 1].copy_(self.offsets[:F + 1], non_blocking=True)
            self.h_verts[:S].copy_(self.verts[:S], non_blocking=True)
            self.event = torch.cuda.Event()
            self.event.record(self.stream)
        self.state = _Slot.COPY
        return True

    def take_failed(self):
        batch, self.batch = self.batch, []
        self.state = _Slot.IDLE
        return batch

    def finish(self, now: float):
        n = len(self.batch)
        po = self.h_poly_off.numpy()[:n + 1]
        offs = self.h_offsets.numpy()
        verts = self.h_verts.numpy()
        for k, r in enumerate(self.batch):
            a, b = int(po[k]), int(po[k + 1])
            o = offs[a:b + 1]
            r.offsets = (o - o[0]).astype(np.int32)
            r.verts = verts[int(o[0]):int(o[-1])].copy()
            r.done = now
            r._dev = None
        batch, self.batch = self.batch, []
        self.state = _Slot.IDLE
        return batch

    def close(self):
        self.ctx.status(raise_on_error=False)
        self.ctx.close()


class Server:
    """Continuous-batching server on one GPU (see the module docstring)."""

    def __init__(self, device: int = 0, slots: int = 4, budget_bytes: int = 64 << 30,
                 max_batch_tri: int = 1 << 24, max_batch_meshes: int = 256, max_vert: int | None = None):
        self.device = device
        self.budget = int(budget_bytes)
        mv = max_vert or max_batch_tri + 2 * max_batch_meshes  # V <= T + 2 for a triangulation
        self.slots = [_Slot(device, max_batch_tri, mv, max_batch_meshes) for _ in range(slots)]
        self.max_tri, self.max_meshes, self.max_vert = max_batch_tri, max_batch_meshes, mv
        self.admit_stream = torch.cuda.Stream(torch.device("cuda", device))
        # generator thread for requests that name a grid (started on first use)
        self._gen_q: queue.Queue = queue.Queue()
        self._gen_done: collections.deque = collections.deque()
        self._gen_thread = None

    def close(self):
        for s in self.slots:
            s.close()
        if self._gen_thread is not None:
            self._gen_q.put(None)
            self._gen_thread.join()
            self._gen_thread = None

    def _generator(self):
        """Generator thread: triangulates the named grids in admission order on
        its own context and stream; the library call waits for the stream with
        the interpreter lock released."""
        ctx = lib.Context(self.device)
        stream = torch.cuda.Stream(torch.device("cuda", self.device))
        try:
            while True:
                r = self._gen_q.get()
                if r is None:
                    return
                try:
                    with torch.cuda.stream(stream):
                        tri, _ = ctx.gen_grid(*r.gen)
                        r._dev = (tri.xy, tri.twin, tri.origin)
                        r._size = (tri.n_vertices, tri.n_halfedges)
                        r._ready = torch.cuda.Event()
                        r._ready.record(stream)
                except lib.PolyllaError as e:
                    r.error = e.code
                self._gen_done.append(r)
        finally:
            ctx.close()

    def _admit(self, r: Request, dev, resident):
        if r.gen is not None:
            if self._gen_thread is None:
                self._gen_thread = threading.Thread(target=self._generator, daemon=True)
                self._gen_thread.start()
            self._gen_q.put(r)
            return
        with torch.cuda.stream(self.admit_stream):
            r._dev = (r.xy.to(dev, non_blocking=True), r.twin.to(dev, non_blocking=True),
                      r.origin.to(dev, non_blocking=True))
            r._ready = torch.cuda.Event()
            r._ready.record(self.admit_stream)
        resident.append(r)

    def run(self, requests: list[Request]) -> dict:
        """Serve `requests` (sorted by arrival) in real time; returns throughput
        and latency statistics. Every request must fit one slot."""
        for r in requests:
            if r.n_tri > self.max_tri or r.n_vertices > self.max_vert:
                raise ValueError(f"request {r.rid} exceeds a slot ({r.n_tri} triangles)")
            if r.input_bytes() > self.budget:
                raise ValueError(f"request {r.rid} alone exceeds the admission budget")
        dev = torch.device("cuda", self.device)
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        waiting: collections.deque[Request] = collections.deque()   # arrived, not admitted
        resident: collections.deque[Request] = collections.deque()  # admitted, not started
        used = 0
        finished = []
        t0 = time.perf_counter()
        n_total = len(requests)
        while len(finished) < n_total:
            now = time.perf_counter() - t0
            progressed = False
            while pending and pending[0].arrival <= now:
                waiting.append(pending.popleft())
            while waiting and used + waiting[0].input_bytes() <= self.budget:
                r = waiting.popleft()
                r._charged = r.input_bytes()
                used += r._charged
                r.admitted = now
                self._admit(r, dev, resident)
                progressed = True
            while self._gen_done:  # generated inputs join the resident requests
                r = self._gen_done.popleft()
                progressed = True
                if r.error:
                    r.done = time.perf_counter() - t0
                    r.started = r.done
                    used -= r._charged
                    finished.append(r)
                else:
                    resident.append(r)
            for slot in self.slots:
                if slot.state == _Slot.COMPUTE and slot.event.query():
                    if not slot.copy_back():
                        bad = slot.take_failed()
                        if len(bad) == 1 and bad[0].alone:
                            r = bad[0]  # fails on its own: answered with the error, no polygons
                            r.error, r.done, r._dev = slot.failed, time.perf_counter() - t0, None
                            used -= r._charged
                            finished.append(r)
                        else:
                            for r in reversed(bad):  # served again, one request per batch
                                r.alone = True
                                resident.appendleft(r)
                    progressed = True
                if slot.state == _Slot.COPY and slot.event.query():
                    done = slot.finish(time.perf_counter() - t0)
                    for r in done:
                        used -= r._charged
                    finished.extend(done)
                    progressed = True
                if slot.state == _Slot.IDLE and resident:
                    batch, tri, verts = [], 0, 0
                    while resident and len(batch) < self.max_meshes and \
                            tri + resident[0].n_tri <= self.max_tri and \
                            verts + resident[0].n_vertices <= self.max_vert and \
                            not (batch and (batch[0].alone or resident[0].alone)):
                        r = resident.popleft()
                        tri += r.n_tri
                        verts += r.n_vertices
                        r.started = time.perf_counter() - t0
                        batch.append(r)
                    slot.launch(batch)
                    progressed = True
            if not progressed:
                time.sleep(20e-6)
        return summarize(finished)


def summarize(done: list[Request]) -> dict:
    failed = sum(1 for r in done if r.error)
    lat = np.array([r.done - r.arrival for r in done])
    adm = np.array([r.admitted - r.arrival for r in done])
    que = np.array([r.started - r.admitted for r in done])
    svc = np.array([r.done - r.started for r in done])
    span = max(r.done for r in done) - min(r.arrival for r in done)
    tri = sum(r.n_tri for r in done)

    def q(x, p):
        return round(float(np.percentile(x, p)) * 1e3, 3)

    return {"requests": len(done), "failed": failed, "span_s": round(span, 4),
            "meshes_per_s": round(len(done) / span, 2), "triangles_per_s": round(tri / span, 1),
            "latency_ms": {"p50": q(lat, 50), "p99": q(lat, 99), "mean": round(float(lat.mean()) * 1e3, 3)},
            "breakdown_ms_p50": {"admission_wait": q(adm, 50), "queued": q(que, 50), "service": q(svc, 50)},
            "breakdown_ms_p99": {"admission_wait": q(adm, 99), "queued": q(que, 99), "service": q(svc, 99)}}
