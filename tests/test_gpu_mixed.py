"""The paper's "mixed" configuration (label and traversal on the GPU, the
reparation phase sequentially on the host) through the C ABI: identical to
the oracle and to the all-GPU call."""
import numpy as np
import pytest

import oracle
from fixtures import golden, golden_names, random_mesh
from meshgen.gen import config_mesh

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2204_05438_amd import lib
    c = lib.Context(0)
    yield c
    c.close()


def _check(ctx, mesh):
    from paper_2204_05438_amd import lib
    tri = lib.Tri.from_mesh(mesh)
    off, verts, start, he, secs = ctx.mesh_mixed(tri, mesh.twin, mesh.origin)
    o = oracle.oracle_on(mesh)
    for name, a, b in (("offsets", off, o["offsets"]), ("verts", verts, o["verts"]), ("start", start, o["start"]),
                       ("he", he, o["he"])):
        assert a.shape == b.shape and np.array_equal(a, b), name
    return secs


@pytest.mark.parametrize("name", golden_names())
def test_mixed_golden(ctx, name):
    print(f"[gpu-case] mixed golden {name}", flush=True)
    _check(ctx, golden(name)[0])


@pytest.mark.parametrize("kind", ["uniform", "cluster", "grid", "lattice"])
def test_mixed_random(ctx, kind):
    print(f"[gpu-case] mixed random {kind}", flush=True)
    for seed in range(4):
        _check(ctx, random_mesh(2100 + seed, [50, 400, 3000, 20000][seed], kind))


@pytest.mark.parametrize("name", ["uniform10k", "mixed200k", "pslg20k"])
def test_mixed_workloads(ctx, name):
    print(f"[gpu-case] mixed workload {name}", flush=True)
    secs = _check(ctx, config_mesh(name))
    assert all(v >= 0 for v in secs.values())


def test_mixed_lobe(ctx):
    """The batched workload's mesh 32: a single-tip polygon with a lobe."""
    print("[gpu-case] mixed batched mesh 32", flush=True)
    from meshgen.gen import batch_points, batch_sizes, mesh_from_points
    _check(ctx, mesh_from_points(batch_points(32, int(batch_sizes(2000)[32]))))
