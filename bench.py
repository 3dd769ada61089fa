"""Throughput benchmark of the terminal-edge-region mesher on one MI355X.

The default run measures the three workloads of the metric and prints ONE
JSON line on stdout (progress goes to stderr):

  grid10m  (headline) one step = label -> build -> repair (polylla_mesh) over
           the resident 10M-point jittered-grid Delaunay mesh: inputs in HBM
           before timing starts, outputs at worst-case capacity; one event
           pair per step (mean, median, p99), per-kernel table from separate
           steps, HBM roofline of the dominant kernel and of the whole step;
  batched2000  2,000 uniform meshes (points log-uniform in [1e3, 1e6]) in one
           polylla_mesh_batched call, eager and replayed from a HIP graph,
           against one polylla_mesh launch per mesh on the same GPU;
  serve2000    continuous-batching server: capacity, then Poisson arrivals at
           0.5x and 0.9x of it; meshes/s, triangles/s, p50/p99 latency.

Every batched and served result is compared with the CPU oracle (digests of
labels and polygons per mesh, the oracle run by a process pool over the host
cores while the meshes are generated). cpu_baseline: the oracle on one core,
median of 3 runs on a bounded sample of the grid workload, plus the pool
throughput of the batched and served oracle runs.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload all|grid10m|batched2000|serve2000]
                  [--no-cpu] [--calib-copy-mb M] [--retune]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "triangles/sec (label+build+repair) at 10M pts; batched vs per-mesh launch; p99"
HBM_PEAK_GBS = 8000.0
POOL_MAX = 16  # host processes (the GPU machine's CPU share)


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# ---------------------------------------------------------------------------
# byte models

def paper_bytes(n: dict) -> dict:
    """Compulsory HBM bytes of one step by the method's own data flow (each
    array element read or written once): label 16N (xy) + 12T (origin) + 12T
    (twin) + 1T (labels); build 4R (seed list) + 8T (twin of the internal
    edges, crossed twice) + 1T (labels) + 4S' (origin of the cycle vertices)
    + 4S (vertex ids written) + 4F (offsets), S' = T + 2R before the repair,
    S = T + 2F after. Split by kernel of the path."""
    V, T, R, F, S, Sp = n["V"], n["T"], n["R"], n["F"], n["S"], n["Sp"]
    return {
        "k_longest": 16 * V + 12 * T,          # xy, origin (LabelMax)
        "k_label": 12 * T + T,                 # twin, labels (LabelSeed, LabelFrontier)
        "k_seeds": 4 * R,                      # seed list
        "k_walk": 8 * T + T + 4 * Sp,          # twin crossings, labels, cycle origins
        "k_scan_emit": 4 * S + 4 * F,          # CSR written
        "step": 16 * V + 25 * T + 4 * R + 9 * T + 4 * Sp + 4 * S + 4 * F,
    }


def design_bytes(n: dict) -> dict:
    """Bytes each kernel of this design moves by its own data layout (every
    array element once, including its own intermediate arrays)."""
    V, T, R, F, S, Sp = n["V"], n["T"], n["R"], n["F"], n["S"], n["Sp"]
    return {
        "k_longest": 13 * T + 17 * V,          # origin 12T + xy 16V read, Max 1T + vtx clear 1V written
        "k_label": 41 * T,                     # twin 12T + origin 12T + Max 1T; labels 4T + walk words 12T
        "k_seeds": T + 4 * R,
        "k_walk": 12 * T + 24 * R + 4 * Sp,    # walk words, seeds; staged cycles + per-polygon records
        "k_scan_emit": 8 * S + 28 * R + 4 * F,
    }


def kernel_sources_digest() -> str:
    """sha256 over the HIP sources of the library (file names and contents)."""
    d = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2204_05438_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        if name.endswith((".hip", ".h")):
            d.update(name.encode())
            with open(os.path.join(csrc, name), "rb") as f:
                d.update(f.read())
    return d.hexdigest()


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch of `kernel` (or, with kernel None, per step) from
    the committed counter summary, or None when it is missing or was taken on
    other kernel sources."""
    path = os.path.join(ROOT, "profiles", f"hbm_traffic.{workload}.md")
    try:
        lines = open(path).read().splitlines()
    except OSError:
        return None
    if f"sources sha256: {kernel_sources_digest()}" not in lines:
        return None
    for ln in lines:
        if kernel is None and ln.startswith("per-step total MB:"):
            return int(float(ln.split(":", 1)[1]) * 1e6)
        cells = [c.strip() for c in ln.strip("|").split("|")]
        if kernel is not None and len(cells) == 6 and cells[0].split("<")[0] == kernel:
            return int(float(cells[5]) * 1e6)
    return None


def host_info() -> dict:
    model = platform.processor() or ""
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                model = ln.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    return {"cpu_model": model, "nproc": os.cpu_count(), "cpus_available": avail}


def percentile(xs, p):
    import numpy as np
    return float(np.percentile(np.asarray(xs, dtype=np.float64), p))


# ---------------------------------------------------------------------------
# host workers (forked before the first GPU call; they never touch the GPU)

def digest(offsets, verts, he) -> str:
    import numpy as np
    d = hashlib.sha256()
    for a, dt in ((offsets, np.int32), (verts, np.int32), (he, np.uint8)):
        d.update(np.ascontiguousarray(a, dtype=dt).tobytes())
    return d.hexdigest()


def _oracle_digest(mesh, with_labels=True):
    import numpy as np
    import oracle
    t0 = time.perf_counter()
    o = oracle.oracle_on(mesh)
    dt = time.perf_counter() - t0
    he = o["he"] if with_labels else np.zeros(0, np.uint8)
    return digest(o["offsets"], o["verts"], he), dt, int(o["offsets"].size - 1)


def _job_batch_mesh(job):
    """Triangulate mesh m of the batched workload and digest its oracle output."""
    m, n, with_oracle = job
    from meshgen.gen import batch_points, mesh_from_points
    mesh = mesh_from_points(batch_points(m, n))
    dg = _oracle_digest(mesh) if with_oracle else (None, 0.0, -1)
    return m, mesh.xy, mesh.origin, mesh.twin, dg


def _job_request(job):
    """Triangulate one request of the serving workload and digest its oracle output."""
    j, n, kind, seed, with_oracle = job
    from meshgen.gen import mesh_from_points, request_points
    mesh = mesh_from_points(request_points(n, kind, seed))
    dg = _oracle_digest(mesh, with_labels=False) if with_oracle else (None, 0.0, -1)
    return j, mesh.xy, mesh.origin, mesh.twin, dg


def _job_arrays_oracle(job):
    """The oracle's digest (polygons only) of a mesh given as arrays (a grid
    generated on the device and copied back)."""
    import numpy as np
    from meshgen.gen import Mesh
    k, xy, origin, twin = job
    h = np.arange(origin.shape[0])
    mesh = Mesh(xy=xy, origin=origin, twin=twin, next=(h - h % 3 + (h + 1) % 3).astype(np.int32))
    return k, _oracle_digest(mesh, with_labels=False)[0]


def _job_workload_oracle(name):
    """The oracle on a whole single-mesh workload (identity check of the
    timed GPU output)."""
    from meshgen.gen import config_mesh
    mesh = config_mesh(name)
    return _oracle_digest(mesh)


def generate(pool, fn, jobs, n):
    """Run generation jobs largest first; returns meshes, digests, oracle seconds."""
    from meshgen.gen import Mesh
    meshes, digests, secs = [None] * n, [None] * n, 0.0
    t0 = time.time()
    for done, (k, xy, origin, twin, (dg, dt, _)) in enumerate(pool.imap_unordered(fn, jobs), 1):
        meshes[k] = Mesh(xy=xy, origin=origin, twin=twin, next=None)
        digests[k] = dg
        secs += dt
        if done % 250 == 0:
            log(f"  {done}/{n} meshes generated ({time.time() - t0:.0f}s)")
    return meshes, digests, secs


# ---------------------------------------------------------------------------
# grid10m

def bench_single(args, pool, workload: str):
    import numpy as np
    import torch
    from meshgen.gen import config_mesh
    from paper_2204_05438_amd import lib

    ident = None if args.no_cpu else pool.apply_async(_job_workload_oracle, (workload,))
    t0 = time.time()
    mesh = config_mesh(workload)
    log(f"generated {workload}: {mesh.n_vertices} vertices, {mesh.n_tri} triangles in {time.time() - t0:.1f}s")
    dev = torch.device("cuda:0")
    ctx = lib.Context(0)
    tri = lib.Tri.from_mesh(mesh, device=dev)
    labels = lib.Labels.empty(tri)
    out = lib.Polys.empty(tri, with_start=True)
    ctx.reserve(tri.n_halfedges, tri.n_vertices)
    for kv in args.param:
        name, val = kv.split("=")
        ctx.set_param({"walk_cap": lib.PARAM_WALK_CAP, "walk_blocks": lib.PARAM_WALK_BLOCKS}[name], int(val))
    torch.cuda.synchronize()
    log("inputs resident on the device")
    if args.calib_copy_mb:
        nb = args.calib_copy_mb << 20
        src = torch.empty(nb // 4, dtype=torch.int32, device=dev).fill_(1)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"calibration copy of {args.calib_copy_mb} MiB done")
    for _ in range(args.warmup):
        ctx.mesh(tri, labels, out)
    ctx.status()
    stats = ctx.stats()
    F, S = (int(x) for x in out.counts.tolist())
    log(f"warmup done: {stats}, F={F}, S={S}")

    # Timed steps, one event pair per step on the launching stream; the
    # library records events around the walk kernel only (its live duration
    # feeds the roofline; events around every kernel would add gaps).
    stream = torch.cuda.current_stream()
    ctx.profile(True, walk_only=True)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    for a, b in evs:
        a.record(stream)
        ctx.mesh(tri, labels, out)
        b.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ctx.status()
    walk_live = ctx.profile_read()
    ctx.profile(False)
    step_ms = [a.elapsed_time(b) for a, b in evs]
    ms_total = evs[0][0].elapsed_time(evs[-1][1])
    ms_step = ms_total / args.steps
    T = mesh.n_tri
    value = T / (ms_step / 1e3)
    log(f"{args.steps} steps: {ms_step:.3f} ms/step (median {percentile(step_ms, 50):.3f}, "
        f"p99 {percentile(step_ms, 99):.3f}), {value:.4g} triangles/s")
    ctx.profile(True)
    for _ in range(min(args.steps, 5)):
        ctx.mesh(tri, labels, out)
    torch.cuda.synchronize()
    prof = ctx.profile_read()
    ctx.profile(False)
    ctx.status()
    prof.update(walk_live)
    for k, (ms, nlaunch) in sorted(prof.items(), key=lambda kv: -kv[1][0] / max(kv[1][1], 1)):
        log(f"  {k:16s} {ms / max(nlaunch, 1) * 1e3:10.1f} us/launch  ({nlaunch} launches)")

    n = {"V": mesh.n_vertices, "T": T, "R": stats["seeds"], "F": F, "S": S, "Sp": T + 2 * stats["seeds"]}
    pb, db = paper_bytes(n), design_bytes(n)
    us = {k: ms / max(nl, 1) * 1e3 for k, (ms, nl) in prof.items()}
    dominant = max(us, key=us.get)
    dom_us = us[dominant]
    achieved = pb.get(dominant, 0) / (dom_us / 1e6) / 1e9
    step_gbs = pb["step"] / (ms_step / 1e3) / 1e9
    step_traffic = measured_traffic(None, workload)  # calibrated counter bytes of a whole step
    roofline = {"bound": "hbm", "kernel": dominant, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": measured_traffic(dominant, workload),
                "avg_launch_us": round(dom_us, 1), "algorithmic_bytes": pb.get(dominant, 0),
                "whole_step": {"algorithmic_bytes": pb["step"], "achieved": round(step_gbs, 1),
                               "frac": round(step_gbs / HBM_PEAK_GBS, 4), "traffic_bytes": step_traffic,
                               "traffic_GBps": None if step_traffic is None else round(step_traffic / (ms_step / 1e3) / 1e9, 1),
                               "traffic_frac": None if step_traffic is None else
                               round(step_traffic / (ms_step / 1e3) / 1e9 / HBM_PEAK_GBS, 4)},
                "design_bytes": {"bytes": db.get(dominant, 0),
                                 "achieved": round(db.get(dominant, 0) / (dom_us / 1e6) / 1e9, 1)}}
    kernels = {k: {"us_per_launch": round(v, 1),
                   "paper_GBps": round(pb.get(k, 0) / (v / 1e6) / 1e9, 1),
                   "design_GBps": round(db.get(k, 0) / (v / 1e6) / 1e9, 1)} for k, v in us.items()}

    # longest-edge propagation paths of every triangle (LabelMax + path kernels)
    ctx.lepp(tri)
    torch.cuda.synchronize()
    le0, le1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    le0.record(stream)
    for _ in range(5):
        ctx.lepp(tri)
    le1.record(stream)
    torch.cuda.synchronize()
    ctx.status()
    lepp_ms = le0.elapsed_time(le1) / 5
    lepp = {"ms_per_call": round(lepp_ms, 4), "triangles_per_s": round(T / (lepp_ms / 1e3), 1), "calls": 5}
    log(f"lepp: {lepp}")

    # the paper's mixed configuration on the same mesh: label and traversal
    # on the GPU, the reparation phase sequentially on one host core
    off_g, verts_g, _ = (x.cpu().numpy() for x in out.trimmed())
    he_g = labels.he.cpu().numpy()
    mixed_runs = []
    for _ in range(3):
        w0 = time.perf_counter()
        m_off, m_verts, _, m_he, secs = ctx.mesh_mixed(tri, mesh.twin, mesh.origin)
        mixed_runs.append((time.perf_counter() - w0, secs))
    mixed_runs.sort(key=lambda r: r[0])
    wall_m, secs_m = mixed_runs[1]
    mixed = {"wall_ms_median": round(wall_m * 1e3, 3), "triangles_per_s": round(T / wall_m, 1),
             "phases_ms": {k[:-2] + "_ms": round(v * 1e3, 3) for k, v in secs_m.items()},
             "runs": 3, "vs_all_gpu": round(wall_m * 1e3 / ms_step, 2),
             "identical_to_all_gpu": bool(np.array_equal(m_off, off_g) and np.array_equal(m_verts, verts_g)
                                          and np.array_equal(m_he, he_g))}
    log(f"mixed (GPU label + build, host repair): {mixed}")

    cpu, identical = None, None
    if not args.no_cpu:
        import oracle
        gpu_dg = digest(off_g, verts_g, he_g)
        # the CPU baseline: the oracle alone on one core, median of 3, on a
        # bounded sample of the same recipe (a 1000 x 1000 jittered grid)
        sample = config_mesh("grid1000x")
        secs = []
        for _ in range(3):
            c0 = time.perf_counter()
            oracle.oracle_on(sample)
            secs.append(time.perf_counter() - c0)
        med = sorted(secs)[1]
        dg, full_s, _ = ident.get()
        identical = dg == gpu_dg
        cpu = {"value": round(sample.n_tri / med, 1), "unit": "triangles/s", "cores": 1, "kind": "oracle",
               "sample": f"grid1000x ({sample.n_tri} triangles, the grid recipe at 1M points), label+build+repair, "
                         f"median of 3 runs on one host core",
               "seconds_runs": [round(x, 3) for x in secs],
               "full_mesh": {"seconds": round(full_s, 2), "triangles_per_s": round(T / full_s, 1),
                             "note": "one run on the whole grid10m mesh, in a pool process beside the GPU steps"},
               **host_info()}
        log(f"oracle: sample median {med:.2f}s ({cpu['value']:.4g} triangles/s); full mesh {full_s:.1f}s, "
            f"GPU output identical: {identical}")
    ctx.close()
    del tri, labels, out
    torch.cuda.empty_cache()
    return {
        "ms_per_step": round(ms_step, 4), "value": round(value, 1),
        "steps_ms": {"mean": round(ms_step, 4), "median": round(percentile(step_ms, 50), 4),
                     "p99": round(percentile(step_ms, 99), 4), "min": round(min(step_ms), 4),
                     "wall_mean": round(wall / args.steps * 1e3, 4)},
        "config": {"workload": f"{workload}: jittered 3163x3163 grid in [0,1]^2 (seed 3), Delaunay, "
                               f"{mesh.n_vertices} vertices, {T} triangles, one mesh per step",
                   "polygons": F, "seeds": stats["seeds"], "tips": stats["tips"], "splits": stats["splits"],
                   "general_small": stats["general_small"], "general_big": stats["general_big"]},
        "roofline": roofline, "kernels": kernels, "cpu_baseline": cpu, "oracle_identical": identical,
        "mixed": mixed, "lepp": lepp,
    }


# ---------------------------------------------------------------------------
# batched

def batch_digests(meshes, out, labels, he_off):
    """Per mesh: digest of its labels and polygons in the oracle's form."""
    import numpy as np
    off, verts, _, po = (x.cpu().numpy() if x is not None else None for x in out.trimmed())
    he = labels.he.cpu().numpy()
    res = []
    for k in range(len(meshes)):
        a, b = int(po[k]), int(po[k + 1])
        o = off[a:b + 1]
        res.append(digest((o - o[0]).astype(np.int32), verts[o[0]:o[-1]], he[he_off[k]:he_off[k + 1]]))
    return res


def bench_batched(args, pool, n_meshes: int):
    import numpy as np
    from meshgen.gen import batch_sizes
    t0 = time.time()
    sizes = batch_sizes(n_meshes)
    order = sorted(range(n_meshes), key=lambda m: -int(sizes[m]))
    meshes, ref, oracle_s = generate(pool, _job_batch_mesh, [(m, int(sizes[m]), not args.no_cpu) for m in order],
                                     n_meshes)
    T_all = sum(m.n_tri for m in meshes)
    log(f"batched: generated {n_meshes} meshes ({T_all} triangles) with {pool._processes} processes "
        f"in {time.time() - t0:.1f}s (oracle {oracle_s:.1f} process-s)")
    import torch
    from paper_2204_05438_amd import autotune, lib
    dev = torch.device("cuda:0")
    ctx = lib.Context(0)
    batch = lib.Batch.from_meshes(meshes, device=dev)
    labels = lib.Labels.empty(batch)
    out = lib.BatchOut.empty(batch, with_start=True)
    ctx.reserve_batch(batch.n_halfedges, batch.n_vertices, n_meshes)
    tris = [lib.Tri.from_mesh(m, device=dev, with_next=False) for m in meshes]
    labs = [lib.Labels.empty(t) for t in tris]
    outs = [lib.Polys.empty(t, with_start=True) for t in tris]
    ctx.reserve(max(t.n_halfedges for t in tris), max(t.n_vertices for t in tris))
    torch.cuda.synchronize()
    log("batched: inputs resident on the device (batch and per mesh)")

    def packed_call():
        ctx.mesh_batched(batch, labels, out)

    def per_mesh_loop():
        for t_, l_, o_ in zip(tris, labs, outs):
            ctx.mesh(t_, l_, o_)

    tuned = autotune.tune(ctx, packed_call, batch.n_halfedges, batched=True, reps=2,
                          cache=args.tune_cache or autotune.DEFAULT_CACHE, force=args.retune)
    log(f"batched: tuned {tuned}")
    stream = torch.cuda.current_stream()

    def timed(fn, reps):
        fn()
        ctx.status()
        ms = []
        torch.cuda.synchronize()
        for _ in range(reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            fn()
            e1.record(stream)
            torch.cuda.synchronize()
            ms.append(e0.elapsed_time(e1))
        ctx.status()
        return {"ms_mean": round(sum(ms) / len(ms), 3), "ms_median": round(percentile(ms, 50), 3),
                "ms_p99": round(percentile(ms, 99), 3)}

    steps = max(2, args.batch_steps)
    loop = timed(per_mesh_loop, steps)
    log(f"batched: one launch per mesh {loop}")
    eager = timed(packed_call, steps)
    log(f"batched: one call, eager {eager}")
    ctx.profile(True)
    packed_call()
    ctx.status()
    prof = ctx.profile_read()
    ctx.profile(False)
    stats = ctx.stats()
    side = torch.cuda.Stream()
    side.wait_stream(stream)
    with torch.cuda.stream(side):
        packed_call()
    stream.wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        packed_call()
    torch.cuda.synchronize()
    replay = timed(graph.replay, steps)
    log(f"batched: graph replay {replay}")
    # every mesh against the oracle, and the per-mesh launches against the batch
    identical, per_mesh_same = None, None
    got = batch_digests(meshes, out, labels, batch.he_off_host.numpy())
    if not args.no_cpu:
        identical = sum(1 for a, b in zip(got, ref) if a == b)
    per = []
    for t_, l_, o_ in zip(tris, labs, outs):
        off, verts, _ = (x.cpu().numpy() for x in o_.trimmed())
        per.append(digest(off, verts, l_.he.cpu().numpy()))
    per_mesh_same = sum(1 for a, b in zip(got, per) if a == b)
    log(f"batched: oracle-identical meshes {identical}/{n_meshes}, per-mesh launches identical {per_mesh_same}")
    g_ms = replay["ms_mean"]
    res = {
        "workload": f"batched{n_meshes}: {n_meshes} uniform meshes, points round(10^U(3,6)) (seed 4), mesh m seeded "
                    f"40000+m; {T_all} triangles, {batch.n_vertices} vertices, {batch.n_halfedges} half-edges",
        "meshes": n_meshes, "triangles": T_all,
        "one_launch_per_mesh": {**loop, "triangles_per_s": round(T_all / (loop["ms_mean"] / 1e3), 1),
                                "meshes_per_s": round(n_meshes / (loop["ms_mean"] / 1e3), 1)},
        "one_call_eager": {**eager, "triangles_per_s": round(T_all / (eager["ms_mean"] / 1e3), 1)},
        "one_call_graph": {**replay, "triangles_per_s": round(T_all / (g_ms / 1e3), 1),
                           "meshes_per_s": round(n_meshes / (g_ms / 1e3), 1)},
        "speedup_vs_one_launch_per_mesh": round(loop["ms_mean"] / g_ms, 3),
        "tuned": tuned, "paths": stats,
        "kernels_us": {k: round(ms / max(nl, 1) * 1e3, 1) for k, (ms, nl) in prof.items()},
        "oracle_identical_meshes": identical, "per_mesh_launch_identical_meshes": per_mesh_same,
    }
    if not args.no_cpu and oracle_s > 0:
        res["cpu_pool"] = {"value": round(T_all / (oracle_s / pool._processes), 1), "unit": "triangles/s",
                           "cores": pool._processes, "kind": "oracle",
                           "sample": f"every mesh of batched{n_meshes}, one oracle per mesh, "
                                     f"{pool._processes} processes; value = triangles / (summed oracle seconds "
                                     f"/ processes)", "oracle_process_seconds": round(oracle_s, 1)}
    del graph
    ctx.close()
    del batch, labels, out, tris, labs, outs
    torch.cuda.empty_cache()
    return res


# ---------------------------------------------------------------------------
# serving

def bench_serve(args, pool, n_requests: int):
    import numpy as np
    from meshgen.gen import serve_requests
    t0 = time.time()
    base = serve_requests(n_requests, rate=1.0)   # arrival times for rate 1/s; scaled below
    order = sorted(range(n_requests), key=lambda j: -base[j][1])
    meshes, ref, oracle_s = generate(
        pool, _job_request, [(j, base[j][1], base[j][2], base[j][3], not args.no_cpu) for j in order], n_requests)
    T_all = sum(m.n_tri for m in meshes)
    log(f"serve: generated {n_requests} requests ({T_all} triangles) in {time.time() - t0:.1f}s "
        f"(oracle {oracle_s:.1f} process-s)")
    from paper_2204_05438_amd import serve
    server = serve.Server(0, slots=args.slots, budget_bytes=64 << 30, max_batch_tri=1 << 24)
    log(f"serve: {args.slots} slots, 64 GB admission budget, batches of up to 2^24 triangles")
    pinned = [serve.Request.from_mesh(j, 0.0, meshes[j]) for j in range(n_requests)]
    del meshes

    def requests(scale):
        return [serve.Request(j, base[j][0] * scale, p.xy, p.twin, p.origin) for j, p in enumerate(pinned)]

    server.run(requests(0.0)[: min(32, n_requests)])  # warm-up
    runs = {}
    cap_reqs = requests(0.0)
    runs["saturated"] = server.run(cap_reqs)
    cap = runs["saturated"]["meshes_per_s"]
    log(f"serve: capacity (all at t=0) {cap} meshes/s, {runs['saturated']['triangles_per_s']:.4g} triangles/s")
    checked = None
    if not args.no_cpu:
        checked = 0
        for r in cap_reqs:
            if r.error == 0 and digest(r.offsets, r.verts, np.zeros(0, np.uint8)) == ref[r.rid]:
                checked += 1
    for f in (0.5, 0.9):
        rate = f * cap
        res = server.run(requests(1.0 / rate))
        res["rate_meshes_per_s"] = round(rate, 2)
        runs[f"{f}x"] = res
        log(f"serve: {f}x capacity ({rate:.1f}/s): p50 {res['latency_ms']['p50']} ms, "
            f"p99 {res['latency_ms']['p99']} ms, {res['meshes_per_s']} meshes/s")
    gen = bench_serve_generated(args, pool, server, base, n_requests)
    server.close()
    out = {"workload": f"serve{n_requests}: Poisson arrivals (seed 5), points round(10^U(3, log10 2e6)), uniform "
                       f"or 4-cluster (sigma 0.05) with probability 1/2, request j seeded 50000+j; {T_all} "
                       f"triangles; 64 GB admission budget; {args.slots} slots",
           "requests": n_requests, "triangles": T_all, "runs": runs,
           "oracle_identical_requests": checked, "generated_on_device": gen}
    if not args.no_cpu and oracle_s > 0:
        out["cpu_pool"] = {"value": round(T_all / (oracle_s / pool._processes), 1), "unit": "triangles/s",
                           "cores": pool._processes, "kind": "oracle",
                           "sample": f"every request of serve{n_requests}, one oracle per request, "
                                     f"{pool._processes} processes", "oracle_process_seconds": round(oracle_s, 1)}
    return out


def bench_serve_generated(args, pool, server, base, n_requests: int):
    """The same request stream with inputs named instead of sent: request j
    is the jittered g x g grid with g = round(sqrt(points of request j)),
    triangulated on the device at admission (no host-to-device copy).
    Capacity and 0.9x of it; every 64th request checked against the oracle
    on its generated mesh (copied back after the runs)."""
    import numpy as np
    from paper_2204_05438_amd import lib, serve
    grids = [(max(4, int(round(float(np.sqrt(base[j][1]))))), 0.45, 70_000 + j) for j in range(n_requests)]

    def requests(scale):
        return [serve.Request.from_grid(j, base[j][0] * scale, *grids[j]) for j in range(n_requests)]

    server.run(requests(0.0)[: min(32, n_requests)])  # warm-up (and the generation context)
    runs = {}
    cap_reqs = requests(0.0)
    runs["saturated"] = server.run(cap_reqs)
    cap = runs["saturated"]["meshes_per_s"]
    T_all = sum(r.n_tri for r in cap_reqs)
    log(f"serve (on-device input): capacity {cap} meshes/s, {runs['saturated']['triangles_per_s']:.4g} triangles/s")
    rate = 0.9 * cap
    res = server.run(requests(1.0 / rate))
    res["rate_meshes_per_s"] = round(rate, 2)
    runs["0.9x"] = res
    log(f"serve (on-device input): 0.9x capacity ({rate:.1f}/s): p50 {res['latency_ms']['p50']} ms, "
        f"p99 {res['latency_ms']['p99']} ms")
    checked = None
    if not args.no_cpu:
        ctx = lib.Context(0)
        jobs = []
        for j in range(0, n_requests, 64):
            tri, _ = ctx.gen_grid(*grids[j])
            jobs.append((j, tri.xy.cpu().numpy(), tri.origin.cpu().numpy(), tri.twin.cpu().numpy()))
            del tri
        ctx.close()
        got = {r.rid: digest(r.offsets, r.verts, np.zeros(0, np.uint8)) for r in cap_reqs if r.error == 0}
        checked = sum(1 for k, dg in pool.imap_unordered(_job_arrays_oracle, jobs) if got.get(k) == dg)
        checked = f"{checked}/{len(jobs)}"
        log(f"serve (on-device input): oracle-identical sampled requests {checked}")
    return {"workload": f"the same {n_requests} arrivals, request j = jittered g x g grid (jitter 0.45, SplitMix64 "
                        f"seed 70000+j), g = round(sqrt(points of request j)), generated on the device at admission; "
                        f"{T_all} triangles",
            "triangles": T_all, "runs": runs, "oracle_identical_sampled_requests": checked}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="all", help="all | grid10m (or another single mesh) | batchedN | serveN")
    ap.add_argument("--batched", type=int, default=2000, help="meshes of the batched workload (with --workload all)")
    ap.add_argument("--serve", type=int, default=2000, help="requests of the serving workload (with --workload all)")
    ap.add_argument("--batch-steps", type=int, default=3, help="timed repetitions of each batched variant")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle (baseline and identity checks)")
    ap.add_argument("--param", action="append", default=[],
                    help="context parameter NAME=VALUE (walk_cap, walk_blocks)")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="also run a plain device copy of this many MiB (counter calibration)")
    ap.add_argument("--tune-cache", default=None, help="autotuner cache file (batched workloads)")
    ap.add_argument("--retune", action="store_true", help="ignore the autotuner cache")
    ap.add_argument("--slots", type=int, default=4, help="serving: concurrent batches (contexts and streams)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); there is no multi-GPU path: "
              "batched and served meshes would shard across GPUs without communication", file=sys.stderr)
        sys.exit(2)

    # the host pool is forked before anything touches the GPU
    from multiprocessing import get_context
    try:
        ncpu = len(os.sched_getaffinity(0))
    except AttributeError:
        ncpu = os.cpu_count() or 1
    pool = get_context("fork").Pool(max(1, min(POOL_MAX, ncpu)))
    t_start = time.time()
    wl = args.workload
    line = {"metric": METRIC, "unit": "triangles/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64+i32",
            "data": "synthetic"}
    try:
        if wl == "all" or not (wl.startswith("batched") or wl.startswith("serve")):
            single = bench_single(args, pool, "grid10m" if wl == "all" else wl)
            line.update(value=single["value"], ms_per_step=single["ms_per_step"], config=single["config"],
                        steps_ms=single["steps_ms"], roofline=single["roofline"], kernels=single["kernels"],
                        cpu_baseline=single["cpu_baseline"], oracle_identical=single["oracle_identical"],
                        mixed=single["mixed"], lepp=single["lepp"])
        if wl == "all" or wl.startswith("batched"):
            nb = args.batched if wl == "all" else int(wl[len("batched"):] or 2000)
            b = bench_batched(args, pool, nb)
            line["batched"] = b
            if wl != "all":
                line.update(metric="triangles/sec (label+build+repair), batched meshes in one graph-replayed call",
                            value=b["one_call_graph"]["triangles_per_s"], ms_per_step=b["one_call_graph"]["ms_mean"],
                            config={"workload": b["workload"]}, steps=args.batch_steps, warmup=1)
        if wl == "all" or wl.startswith("serve"):
            ns = args.serve if wl == "all" else int(wl[len("serve"):] or 2000)
            sv = bench_serve(args, pool, ns)
            line["serving"] = sv
            if wl != "all":
                line.update(metric="served meshes: triangles/sec and p50/p99 latency at 0.9x capacity",
                            value=sv["runs"]["0.9x"]["triangles_per_s"], ms_per_step=None,
                            config={"workload": sv["workload"]}, steps=ns, warmup=32)
    finally:
        pool.terminate()
    line["bench_wall_s"] = round(time.time() - t_start, 1)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
