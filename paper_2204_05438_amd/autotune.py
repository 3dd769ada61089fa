"""Autotuner for the walk's launch parameters.

Three context parameters shape the hot path: the persistent grid of the walk
kernel (POLYLLA_PARAM_WALK_BLOCKS: workgroups of 256 threads, i.e. how many
polygons are in flight per XCD against the L2 they share), the walk cap
(POLYLLA_PARAM_WALK_CAP: the longest cycle a lane walks before the polygon is
queued for the workgroup kernel, i.e. the depth of that queue) and the
triangles per thread of the longest-edge kernel (POLYLLA_PARAM_LONGEST_ITEMS:
the loads a thread has in flight). `tune` times them one after the other on the
caller's own input with HIP events (walk grid, then walk cap at the best grid,
then the items at both), keeps
the fastest, leaves it set on the context and caches it in a JSON file keyed
by device and input size class, so later calls on inputs of the same class
skip the sweep.
"""
from __future__ import annotations

import json
import math
import os

import torch

from . import lib

BLOCKS = (512, 768, 1024, 1280, 1536)
CAPS = (12, 16, 20, 24)
ITEMS = (1, 2, 4)
DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "polylla", "tune.json")


def size_class(n_halfedges: int) -> str:
    """Inputs within a factor of 2 of each other share tuned parameters."""
    return "H2^%d" % max(0, int(math.log2(max(n_halfedges, 1))))


def _key(device: int, n_halfedges: int, batched: bool) -> str:
    name = torch.cuda.get_device_name(device).replace(" ", "_")
    return f"{name}|{size_class(n_halfedges)}|{'batched' if batched else 'single'}"


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(path, table):
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp%d" % os.getpid()
    with open(tmp, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def tune(ctx: lib.Context, run, n_halfedges: int, *, batched: bool = False, blocks=BLOCKS, caps=CAPS,
         items=ITEMS, reps: int = 3, cache: str | None = DEFAULT_CACHE, force: bool = False) -> dict:
    """Pick walk_blocks, walk_cap and longest_items for `run()` (one enqueue
    of the caller's polylla_mesh / polylla_mesh_batched on ctx). Returns
    {"walk_blocks", "walk_cap", "longest_items", "ms", "source": "cache" |
    "sweep", "table"}."""
    key = _key(ctx.device, n_halfedges, batched)
    table = _load(cache) if cache else {}
    if not force and key in table and "longest_items" in table[key]:
        best = table[key]
        ctx.set_param(lib.PARAM_WALK_BLOCKS, best["walk_blocks"])
        ctx.set_param(lib.PARAM_WALK_CAP, best["walk_cap"])
        ctx.set_param(lib.PARAM_LONGEST_ITEMS, best["longest_items"])
        return dict(best, source="cache", table=None)
    stream = torch.cuda.current_stream()

    def median_ms():
        run()
        ctx.status()
        times = []
        for _ in range(reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            run()
            e1.record(stream)
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1))
        ctx.status()
        times.sort()
        return times[len(times) // 2]

    # walk grid at the default cap, then the cap at the best grid, then the
    # longest-edge items at both
    results = []
    ctx.set_param(lib.PARAM_LONGEST_ITEMS, 2)
    ctx.set_param(lib.PARAM_WALK_CAP, 24)
    for wb in blocks:
        ctx.set_param(lib.PARAM_WALK_BLOCKS, wb)
        results.append((median_ms(), wb, 24, 2))
    ms, wb, cap, it = min(results)
    ctx.set_param(lib.PARAM_WALK_BLOCKS, wb)
    for cap in caps:
        if cap != 24:
            ctx.set_param(lib.PARAM_WALK_CAP, cap)
            results.append((median_ms(), wb, cap, 2))
    ms, wb, cap, it = min(results)
    ctx.set_param(lib.PARAM_WALK_BLOCKS, wb)
    ctx.set_param(lib.PARAM_WALK_CAP, cap)
    for k in items:
        if k != 2:
            ctx.set_param(lib.PARAM_LONGEST_ITEMS, k)
            results.append((median_ms(), wb, cap, k))
    ms, wb, cap, it = min(results)
    ctx.set_param(lib.PARAM_WALK_BLOCKS, wb)
    ctx.set_param(lib.PARAM_WALK_CAP, cap)
    ctx.set_param(lib.PARAM_LONGEST_ITEMS, it)
    best = {"walk_blocks": wb, "walk_cap": cap, "longest_items": it, "ms": round(ms, 4)}
    if cache:
        table[key] = best
        _store(cache, table)
    return dict(best, source="sweep", table=[{"walk_blocks": b, "walk_cap": c, "longest_items": k, "ms": round(t, 4)}
                                             for t, b, c, k in results])
