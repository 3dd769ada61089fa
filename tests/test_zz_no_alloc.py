"""polylla_mesh_noalloc (scratch in the library's static device array)
against polylla_mesh (context scratch) through the C ABI: identical labels and
polygons on two calls in a row, the second on a smaller mesh (the static
array keeps the first call's contents), also with the labels left to the
library; a mesh beyond the static array's limits is refused."""
import numpy as np
import pytest

from fixtures import random_mesh
from meshgen.gen import config_mesh

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

FULL = ["he", "tri", "vtx", "offsets", "verts", "start"]


def _outputs(labels, out):
    off, verts, start = (x.cpu().numpy() for x in out.trimmed())
    r = {"offsets": off, "verts": verts, "start": start}
    if labels is not None:
        r.update(he=labels.he.cpu().numpy(), tri=labels.tri.cpu().numpy(), vtx=labels.vtx.cpu().numpy())
    return r


def _compare(ctx, mesh, with_labels=True):
    from paper_2204_05438_amd import lib
    tri = lib.Tri.from_mesh(mesh)
    la, oa = lib.Labels.empty(tri), lib.Polys.empty(tri)
    ctx.mesh(tri, la, oa)
    ctx.status()
    ref = _outputs(la, oa)
    lb = lib.Labels.empty(tri) if with_labels else None
    ob = lib.Polys.empty(tri)
    ob.verts.fill_(-7)
    ob.offsets.fill_(-7)
    if lb is not None:
        lb.he.fill_(0xEE)
    ctx.mesh_noalloc(tri, lb, ob)
    ctx.status()
    got = _outputs(lb, ob)
    for k in got:
        assert got[k].shape == ref[k].shape and np.array_equal(got[k], ref[k]), k
    return int(ob.counts[0])


def test_noalloc_equals_mesh():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2204_05438_amd import lib
    print("[gpu-case] no-alloc entry point: uniform120k then a 3000-point cluster mesh", flush=True)
    ctx = lib.Context(0)
    try:
        big = config_mesh("uniform120k")      # ~240k triangles, near the limit
        small = random_mesh(77, 3000, "cluster")
        assert big.n_tri <= 262144
        F1 = _compare(ctx, big)
        F2 = _compare(ctx, small)
        assert F2 < F1
        _compare(ctx, random_mesh(78, 2000, "lattice"), with_labels=False)
        # beyond the static array's limit: refused before any work
        too_big = config_mesh("uniform140k")
        assert too_big.n_tri > 262144
        tri = lib.Tri.from_mesh(too_big)
        with pytest.raises(lib.PolyllaError) as err:
            ctx.mesh_noalloc(tri, None, lib.Polys.empty(tri))
        assert err.value.code == lib.ETOOBIG
        # the context's own path still works afterwards
        _compare(ctx, small)
    finally:
        ctx.close()
