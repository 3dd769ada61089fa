"""Serving loop: requests served in a mix (continuous batching over several
slots, arrivals while other batches run) give exactly the polygons of the
oracle for each request alone; a request that is not a valid triangulation
fails alone and leaves the others' results unchanged."""
import numpy as np
import pytest

import oracle
from fixtures import random_mesh

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _requests(seed, n):
    rng = np.random.default_rng(seed)
    kinds = ["uniform", "cluster", "grid", "lattice"]
    meshes = [random_mesh(800 + j, int(k), kinds[j % 4]) for j, k in enumerate(np.rint(10 ** rng.uniform(1.2, 3.9, n)))]
    arrivals = np.cumsum(rng.exponential(0.002, size=n))
    return meshes, arrivals


def test_served_equals_oracle():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    print("[gpu-case] serve 40 requests, 2 slots", flush=True)
    from paper_2204_05438_amd import serve
    meshes, arrivals = _requests(31, 40)
    server = serve.Server(0, slots=2, budget_bytes=8 << 20, max_batch_tri=1 << 16, max_batch_meshes=8)
    reqs = [serve.Request.from_mesh(j, float(arrivals[j]), m) for j, m in enumerate(meshes)]
    stats = server.run(reqs)
    server.close()
    assert stats["requests"] == len(meshes) and stats["failed"] == 0
    for r, m in zip(reqs, meshes):
        o = oracle.oracle_on(m)
        assert r.error == 0
        assert np.array_equal(r.offsets, o["offsets"]), r.rid
        assert np.array_equal(r.verts, o["verts"]), r.rid


def test_bad_request_fails_alone():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    print("[gpu-case] serve 16 requests, one invalid", flush=True)
    from paper_2204_05438_amd import lib, serve
    meshes, arrivals = _requests(41, 16)
    server = serve.Server(0, slots=2, budget_bytes=8 << 20, max_batch_tri=1 << 16, max_batch_meshes=8)
    reqs = [serve.Request.from_mesh(j, 0.0, m) for j, m in enumerate(meshes)]
    bad = 5
    tw = reqs[bad].twin.clone()
    tw[3] = meshes[bad].n_halfedges + 7   # a twin outside its own mesh
    reqs[bad].twin = tw.pin_memory()
    stats = server.run(reqs)
    server.close()
    assert stats["requests"] == len(meshes) and stats["failed"] == 1
    for r, m in zip(reqs, meshes):
        if r.rid == bad:
            assert r.error == lib.ETOPO and r.offsets is None
            continue
        o = oracle.oracle_on(m)
        assert r.error == 0
        assert np.array_equal(r.offsets, o["offsets"]), r.rid
        assert np.array_equal(r.verts, o["verts"]), r.rid
