"""Serving loop: requests served in a mix (continuous batching over several
slots, arrivals while other batches run) give exactly the polygons each
request gets alone."""
import numpy as np
import pytest

from fixtures import random_mesh

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def test_served_equals_alone():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    print("[gpu-case] serve 40 requests, 2 slots", flush=True)
    from paper_2204_05438_amd import lib, serve
    rng = np.random.default_rng(31)
    kinds = ["uniform", "cluster", "grid", "lattice"]
    meshes = [random_mesh(800 + j, int(n), kinds[j % 4]) for j, n in enumerate(np.rint(10 ** rng.uniform(1.2, 3.9, 40)))]
    arrivals = np.cumsum(rng.exponential(0.002, size=len(meshes)))
    server = serve.Server(0, slots=2, budget_bytes=8 << 20, max_batch_tri=1 << 16, max_batch_meshes=8)
    reqs = [serve.Request.from_mesh(j, float(arrivals[j]), m) for j, m in enumerate(meshes)]
    stats = server.run(reqs)
    server.close()
    assert stats["requests"] == len(meshes)
    ctx = lib.Context(0)
    try:
        for r, m in zip(reqs, meshes):
            tri = lib.Tri.from_mesh(m)
            out = ctx.mesh(tri)
            ctx.status()
            off, verts, _ = (x.cpu().numpy() for x in out.trimmed())
            assert np.array_equal(r.offsets, off), r.rid
            assert np.array_equal(r.verts, verts), r.rid
    finally:
        ctx.close()
