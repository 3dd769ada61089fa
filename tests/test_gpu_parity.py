"""GPU parity: the HIP library (through its C ABI) against the CPU oracle,
element by element, on hand fixtures, seeded tiny meshes and the workloads."""
import numpy as np
import pytest

import oracle
from bruteforce import csr_cycles
from fixtures import empty_mesh, golden, golden_names, permute_mesh, random_mesh, spiral_fan
from meshgen.gen import config_mesh as _config_mesh

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


_MESHES = {}


def config_mesh(name):
    """Workload meshes, generated once per test session."""
    if name not in _MESHES:
        _MESHES[name] = _config_mesh(name)
    return _MESHES[name]


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2204_05438_amd import lib
    c = lib.Context(0)
    yield c
    c.close()


def gpu_mesh(ctx, mesh, walk_cap=24):
    from paper_2204_05438_amd import lib
    ctx.set_param(lib.PARAM_WALK_CAP, walk_cap)
    tri = lib.Tri.from_mesh(mesh)
    labels = lib.Labels.empty(tri)
    out = ctx.mesh(tri, labels)
    ctx.status()
    ctx.set_param(lib.PARAM_WALK_CAP, 24)
    off, verts, start = out.trimmed()
    return {"he": labels.he.cpu().numpy(), "tri": labels.tri.cpu().numpy(), "vtx": labels.vtx.cpu().numpy(),
            "offsets": off.cpu().numpy(), "verts": verts.cpu().numpy(), "start": start.cpu().numpy(),
            "stats": ctx.stats()}


def gpu_three_calls(ctx, mesh, walk_cap=24):
    from paper_2204_05438_amd import lib
    ctx.set_param(lib.PARAM_WALK_CAP, walk_cap)
    tri = lib.Tri.from_mesh(mesh)
    labels = ctx.label(tri)
    pre = ctx.build(tri, labels)
    out = ctx.repair(tri, labels, pre)
    ctx.status()
    ctx.set_param(lib.PARAM_WALK_CAP, 24)
    po, pv, ps = pre.trimmed()
    fo, fv, fs = out.trimmed()
    return {"he": labels.he.cpu().numpy(), "tri": labels.tri.cpu().numpy(), "vtx": labels.vtx.cpu().numpy(),
            "pre_offsets": po.cpu().numpy(), "pre_verts": pv.cpu().numpy(), "pre_start": ps.cpu().numpy(),
            "offsets": fo.cpu().numpy(), "verts": fv.cpu().numpy(), "start": fs.cpu().numpy()}


def assert_same(g, o, keys):
    for k in keys:
        a, b = np.asarray(g[k]), np.asarray(o[k])
        assert a.shape == b.shape, (k, a.shape, b.shape)
        if not np.array_equal(a, b):
            bad = np.nonzero(a != b)[0]
            raise AssertionError(f"{k}: {bad.size} mismatches, first at {bad[:5]}: gpu {a[bad[:5]]} oracle {b[bad[:5]]}")


FULL = ["he", "tri", "vtx", "offsets", "verts", "start"]


@pytest.mark.parametrize("name", golden_names())
def test_golden(ctx, name):
    _say(f"golden {name}")
    mesh, g = golden(name)
    r = gpu_mesh(ctx, mesh)
    assert r["he"].tolist() == g["he"]
    assert r["tri"].tolist() == g["tri"]
    assert r["vtx"].tolist() == g["vtx"]
    assert csr_cycles(r["offsets"], r["verts"]) == [tuple(c) for c in g["final"]]
    assert_same(r, oracle.oracle_on(mesh), FULL)


@pytest.mark.parametrize("kind", ["uniform", "cluster", "grid", "lattice"])
@pytest.mark.parametrize("seed", range(10))
def test_random_small(ctx, kind, seed):
    n = [5, 10, 30, 60, 100, 200, 300, 500, 800, 1500][seed]
    _say(f"random {kind} seed {seed} n {n}")
    mesh = random_mesh(7000 + 13 * seed, n, kind)
    assert_same(gpu_mesh(ctx, mesh), oracle.oracle_on(mesh), FULL)


@pytest.mark.parametrize("walk_cap", [3, 10, 24])
@pytest.mark.parametrize("kind", ["uniform", "cluster", "lattice"])
def test_three_calls_match_oracle(ctx, kind, walk_cap):
    _say(f"label/build/repair {kind} walk_cap {walk_cap}")
    mesh = random_mesh(4242, 3000, kind)
    o = oracle.oracle_on(mesh)
    r = gpu_three_calls(ctx, mesh, walk_cap)
    assert_same(r, o, FULL + ["pre_offsets", "pre_verts", "pre_start"])


@pytest.mark.parametrize("walk_cap", [1, 3, 6, 12])
@pytest.mark.parametrize("kind", ["uniform", "cluster", "grid", "lattice"])
def test_cooperative_path(ctx, kind, walk_cap):
    """Small walk caps send most polygons through the workgroup kernel."""
    _say(f"cooperative {kind} walk_cap {walk_cap}")
    for seed in range(3):
        mesh = random_mesh(900 + seed, 2000, kind)
        r = gpu_mesh(ctx, mesh, walk_cap)
        assert_same(r, oracle.oracle_on(mesh), FULL)
        if walk_cap <= 3:
            assert r["stats"]["general_big"] > 0


@pytest.mark.parametrize("walk_cap", [3, 8, 16, 24])
@pytest.mark.parametrize("kind", ["uniform", "cluster", "grid", "lattice"])
def test_long_cycle_tip_path(ctx, kind, walk_cap):
    """With the long-cycle threshold at 0, every cycle longer than the walk cap
    (more than 128 of them) is walked again by the long-cycle tip path, which
    stages or repairs those of up to 32 frontier half-edges and passes the
    rest to the region kernels; the result is the oracle's."""
    from paper_2204_05438_amd import lib
    _say(f"long-cycle tip path {kind} walk_cap {walk_cap}")
    ctx.set_param(lib.PARAM_LONG_TIP_MIN, 0)
    try:
        for seed in range(2):
            n = {3: 3000, 8: 3000, 16: 8000, 24: 100000}[walk_cap]
            mesh = random_mesh(1300 + seed, n, kind)
            r = gpu_mesh(ctx, mesh, walk_cap)
            assert_same(r, oracle.oracle_on(mesh), FULL)
    finally:
        ctx.set_param(lib.PARAM_LONG_TIP_MIN, 4096)


@pytest.mark.parametrize("wave_max", [0, 1 << 20])
@pytest.mark.parametrize("kind", ["uniform", "cluster"])
def test_declined_short_polygon_paths(ctx, kind, wave_max):
    """The short polygons the single-tip path declines go one lane each (count
    above the threshold) or one wave each (count at most the threshold)."""
    from paper_2204_05438_amd import lib
    _say(f"declined short polygons {kind} wave_max {wave_max}")
    ctx.set_param(lib.PARAM_GEN_WAVE_MAX, wave_max)
    try:
        for seed in range(3):
            mesh = random_mesh(1300 + seed, 20000, kind)
            for walk_cap in (24, 12):
                assert_same(gpu_mesh(ctx, mesh, walk_cap), oracle.oracle_on(mesh), FULL)
    finally:
        ctx.set_param(lib.PARAM_GEN_WAVE_MAX, 8192)


@pytest.mark.parametrize("walk_cap,many", [(24, False), (4, True)])
def test_long_region_routes(ctx, walk_cap, many):
    """At most 128 long polygons go straight to the 1024-thread region kernel;
    more go through the one-wave kernel first (its overflow to the former)."""
    _say(f"long-region route walk_cap {walk_cap}")
    mesh = random_mesh(1400, 20000, "uniform")
    r = gpu_mesh(ctx, mesh, walk_cap)
    assert (r["stats"]["general_big"] > 128) == many, r["stats"]
    assert_same(r, oracle.oracle_on(mesh), FULL)


@pytest.mark.parametrize("lds_max,mem_max", [(32, 65536), (32, 32), (4096, 65536)])
@pytest.mark.parametrize("kind", ["uniform", "cluster"])
def test_region_memory_paths(ctx, kind, lds_max, mem_max):
    """Regions beyond the LDS limit of the 1024-thread kernel are built by the
    global-memory workgroup path, and beyond its own limit one lane each
    (limits lowered so that many regions take each route). The uniform mesh
    has at most 128 long polygons at walk cap 24 (all go to the 1024-thread
    kernel) and long regions past the one-wave kernel at walk cap 4."""
    from paper_2204_05438_amd import lib
    _say(f"region memory paths {kind} lds_max {lds_max} mem_max {mem_max}")
    ctx.set_param(lib.PARAM_REGION_LDS_MAX, lds_max)
    ctx.set_param(lib.PARAM_REGION_MEM_MAX, mem_max)
    try:
        mesh = random_mesh(1500, 20000, kind)
        o = oracle.oracle_on(mesh)
        for walk_cap in (24, 4):
            r = gpu_mesh(ctx, mesh, walk_cap)
            st = r["stats"]
            assert_same(r, o, FULL)
            if kind == "uniform":
                assert (st["fallback"] > 0) == (lds_max < 4096), st
                assert (st["lane"] > 0) == (lds_max < 4096 and mem_max < 65536), st
            assert st["splits"] == o["stats"]["splits"]
        r3 = gpu_three_calls(ctx, mesh, 24)
        assert_same(r3, o, FULL + ["pre_offsets", "pre_verts", "pre_start"])
    finally:
        ctx.set_param(lib.PARAM_REGION_LDS_MAX, 4096)
        ctx.set_param(lib.PARAM_REGION_MEM_MAX, 65536)


def test_empty(ctx):
    _say("empty mesh")
    r = gpu_mesh(ctx, empty_mesh())
    assert r["offsets"].tolist() == [0] and r["verts"].size == 0


@pytest.mark.parametrize("name", ["uniform10k", "mixed200k", "grid300x"])
def test_workloads_small(ctx, name):
    _say(f"workload {name}")
    mesh = config_mesh(name)
    o = oracle.oracle_on(mesh)
    r = gpu_mesh(ctx, mesh)
    assert_same(r, o, FULL)
    assert r["stats"]["seeds"] == o["stats"]["seeds"]
    assert r["stats"]["splits"] == o["stats"]["splits"]


def test_workload_mixed1m(ctx):
    _say("workload mixed1m")
    mesh = config_mesh("mixed1m")
    o = oracle.oracle_on(mesh)
    r = gpu_mesh(ctx, mesh)
    assert_same(r, o, FULL)
    _say("workload mixed1m, walk cap 4")
    r = gpu_mesh(ctx, mesh, 4)
    assert_same(r, o, FULL)


@pytest.mark.parametrize("block", [0, 3000])
def test_permuted_layout_mixed1m(ctx, block):
    """The 1M-point mixed workload with its triangles renumbered (uniformly at
    random, or as shuffled runs of 3000 triangles that straddle the label
    kernel's tiles) and every triangle's half-edges rotated. Without the
    space-filling order most neighbour lookups miss the label kernel's LDS
    window and the walk's per-XCD seed ranges hold scattered triangles; the
    output must still equal the oracle's on the same input, and its polygons
    those of the unpermuted mesh."""
    _say(f"permuted mixed1m block {block}")
    mesh = config_mesh("mixed1m")
    p, _, _ = permute_mesh(mesh, 17 + block, block=block)
    r = gpu_mesh(ctx, p)
    o = oracle.oracle_on(p)
    assert_same(r, o, FULL)
    base = oracle.oracle_on(mesh)
    assert sorted(csr_cycles(r["offsets"], r["verts"])) == sorted(csr_cycles(base["offsets"], base["verts"]))


def test_single_tip_polygon_with_a_lobe(ctx):
    """Mesh 32 of the batched workload (656,631 uniform points) has a short
    polygon with one barrier-edge tip whose cycle also runs twice along a
    barrier edge away from the tip's slit (a lobe of the region hangs off
    that edge). The single-tip path must leave it to the region path, which
    marks that edge BARRIER like the oracle."""
    _say("batched mesh 32: single-tip polygon with a lobe")
    from meshgen.gen import batch_points, batch_sizes, mesh_from_points
    mesh = mesh_from_points(batch_points(32, int(batch_sizes(2000)[32])))
    r = gpu_mesh(ctx, mesh)
    o = oracle.oracle_on(mesh)
    assert o["stats"]["nonsimple_final"] >= 1
    assert_same(r, o, FULL)


@pytest.mark.parametrize("name", ["pslg20k", "pslg200k"])
def test_pslg_workloads(ctx, name):
    """Triangulations of planar straight-line graphs (8 circular holes, 6
    cracks): segment sides labelled like boundary edges, regions never
    crossing a segment, cracks as barrier edges with tips at their ends."""
    _say(f"workload {name}")
    mesh = config_mesh(name)
    o = oracle.oracle_on(mesh)
    r = gpu_mesh(ctx, mesh)
    assert_same(r, o, FULL)
    assert r["stats"]["splits"] == o["stats"]["splits"] > 0


def test_pslg_segment_flags_validated(ctx):
    """Segment flags on one half-edge of an edge only: polylla_validate
    reports ETOPO."""
    _say("pslg: asymmetric segment flags")
    from paper_2204_05438_amd import lib
    mesh = config_mesh("pslg20k")
    tri = lib.Tri.from_mesh(mesh)
    assert ctx.validate(tri) == lib.OK
    h = int(np.nonzero((mesh.fixed > 0) & (mesh.twin >= 0))[0][0])
    tri.fixed[h] = 0
    assert ctx.validate(tri) == lib.ETOPO


def test_batched_pslg(ctx):
    """A batch mixing PSLG meshes (segments) and plain meshes (no segments),
    cut into several groups, each mesh against the oracle."""
    _say("batched: PSLG and plain meshes")
    from meshgen.gen import pslg_mesh
    from paper_2204_05438_amd import lib
    meshes = []
    for k in range(12):
        if k % 3 == 2:
            meshes.append(random_mesh(4000 + k, 500 + 300 * k, "uniform"))
        else:
            meshes.append(pslg_mesh(800 + 700 * k, 2 + k % 3, 1 + k % 4, 60 + k))
    batch = lib.Batch.from_meshes(meshes)
    labels = lib.Labels.empty(batch)
    ctx.set_param(lib.PARAM_BATCH_GROUP_HE, 40000)
    try:
        out = ctx.mesh_batched(batch, labels)
        ctx.status()
    finally:
        ctx.set_param(lib.PARAM_BATCH_GROUP_HE, (1 << 30) - (1 << 24))
    check_batch_against_oracle(meshes, out, labels, batch.he_off_host.numpy())


def gpu_lepp(ctx, mesh):
    from paper_2204_05438_amd import lib
    term, length = ctx.lepp(lib.Tri.from_mesh(mesh))
    ctx.status()
    return term.cpu().numpy(), length.cpu().numpy()


@pytest.mark.parametrize("name", ["fan7_tip", "square", "square_segment"])
def test_lepp_golden(ctx, name):
    _say(f"lepp golden {name}")
    mesh, g = golden(name)
    term, length = gpu_lepp(ctx, mesh)
    assert term.tolist() == g["lepp_terminal"] and length.tolist() == g["lepp_length"]


def test_lepp_long_paths(ctx):
    """Paths far longer than the chase's 32 steps, finished by pointer
    jumping: the spiral fan's closed-form lengths, and the oracle."""
    _say("lepp spiral fans")
    for n in (40, 300, 5000):
        mesh = spiral_fan(n)
        term, length = gpu_lepp(ctx, mesh)
        expect = np.array([n - i for i in range(n - 1)] + [2], np.int32)
        assert (term == 3 * n - 4).all() and np.array_equal(length, expect), n
        ot, ol = oracle.oracle_lepp(mesh)
        assert np.array_equal(term, ot) and np.array_equal(length, ol)


@pytest.mark.parametrize("name", ["random", "uniform10k", "pslg20k", "mixed200k", "grid10m"])
def test_lepp_against_oracle(ctx, name):
    """Longest-edge propagation paths against the oracle."""
    _say(f"lepp {name}")
    meshes = ([random_mesh(6000 + k, [20, 300, 3000][k % 3], ["uniform", "cluster", "lattice"][k % 3])
               for k in range(6)] if name == "random" else [config_mesh(name)])
    for mesh in meshes:
        term, length = gpu_lepp(ctx, mesh)
        ot, ol = oracle.oracle_lepp(mesh)
        assert np.array_equal(term, ot) and np.array_equal(length, ol)


def test_uniform5m_large_regions(ctx):
    """5M uniform points: two regions exceed the LDS of the 1024-thread
    kernel at the default limits and are built by the global-memory path."""
    _say("uniform5m (regions beyond the workgroup LDS)")
    mesh = config_mesh("uniform5m")
    o = oracle.oracle_on(mesh)
    r = gpu_mesh(ctx, mesh)
    assert r["stats"]["fallback"] >= 1 and r["stats"]["lane"] == 0, r["stats"]
    assert_same(r, o, FULL)
    assert r["stats"]["splits"] == o["stats"]["splits"]


def test_workload_grid10m(ctx):
    """The benchmark workload at full size, in the benchmark's configuration."""
    _say("workload grid10m")
    mesh = config_mesh("grid10m")
    r = gpu_mesh(ctx, mesh)
    _say("grid10m: oracle")
    o = oracle.oracle_on(mesh)
    assert_same(r, o, FULL)
    assert r["stats"]["general_big"] > 0


def test_deterministic(ctx):
    _say("determinism mixed200k x3")
    mesh = config_mesh("mixed200k")
    runs = [gpu_mesh(ctx, mesh) for _ in range(3)]
    for r in runs[1:]:
        assert_same(r, runs[0], FULL)


def test_capacity_error(ctx):
    _say("capacity error")
    from paper_2204_05438_amd import lib
    mesh = random_mesh(5, 400, "uniform")
    tri = lib.Tri.from_mesh(mesh)
    out = lib.Polys.empty(tri, cap_polys=10, cap_verts=40)
    ctx.mesh(tri, None, out)
    assert ctx.status(raise_on_error=False) == lib.ECAPACITY
    # the context is usable afterwards
    r = gpu_mesh(ctx, mesh)
    assert_same(r, oracle.oracle_on(mesh), FULL)


def test_layout_errors(ctx):
    _say("layout errors")
    from paper_2204_05438_amd import lib
    mesh, _ = golden("square")
    tri = lib.Tri.from_mesh(mesh)
    assert ctx.validate(tri) == lib.OK
    bad = lib.Tri(tri.xy, tri.twin.clone(), tri.next, tri.origin)
    bad.twin[2] = 4
    assert ctx.validate(bad) == lib.ETOPO
    badn = lib.Tri(tri.xy, tri.twin, tri.next.clone(), tri.origin)
    badn.next[0] = 2
    assert ctx.validate(badn) == lib.ELAYOUT
    short = lib.Tri(tri.xy, tri.twin[:5], tri.next[:5], tri.origin[:5])
    with pytest.raises(lib.PolyllaError):
        ctx.mesh(short)
    # out-of-range twin inside the hot path: reported, no fault
    badr = lib.Tri(tri.xy, tri.twin.clone(), tri.next, tri.origin)
    badr.twin[2] = 1000
    ctx.mesh(badr)
    assert ctx.status(raise_on_error=False) == lib.ETOPO


def check_batch_against_oracle(meshes, out, labels=None, he_off=None, oracle_outputs=None):
    """Every mesh's polygons in a batched output (mesh-local ids) equal the
    oracle's for that mesh alone."""
    off, verts, start, po = (x.cpu().numpy() if x is not None else None for x in out.trimmed())
    he = labels.he.cpu().numpy() if labels is not None else None
    assert po[0] == 0 and po[-1] == off.size - 1
    for k, m in enumerate(meshes):
        o = oracle_outputs[k] if oracle_outputs is not None else oracle.oracle_on(m)
        a, b = int(po[k]), int(po[k + 1])
        got_off = off[a:b + 1] - off[a]
        assert np.array_equal(got_off, o["offsets"]), k
        assert np.array_equal(verts[off[a]:off[b]], o["verts"]), k
        if start is not None:
            assert np.array_equal(start[a:b], o["start"]), k
        if he is not None:
            assert np.array_equal(he[he_off[k]:he_off[k + 1]], o["he"]), k


@pytest.mark.parametrize("walk_cap,lds_max,mem_max,group", [(4, 4096, 65536, 0), (24, 4096, 65536, 0),
                                                            (24, 32, 65536, 0), (24, 32, 32, 0), (4, 32, 32, 0),
                                                            (24, 4096, 65536, 3), (24, 4096, 65536, 30000)])
def test_batched_equals_per_mesh(ctx, walk_cap, lds_max, mem_max, group):
    """A batch of uneven meshes (mesh-local indices) gives each mesh its own
    polygons, also with the region limits lowered (regions of the batch take
    the global-memory and one-lane paths) and with the batch cut into groups
    of one mesh each (group 3) or of about 30000 half-edges."""
    _say(f"batched 40 meshes walk_cap {walk_cap} lds_max {lds_max} mem_max {mem_max} group {group}")
    from paper_2204_05438_amd import lib
    rng = np.random.default_rng(11)
    meshes = [random_mesh(300 + k, int(n), ["uniform", "cluster", "grid", "lattice"][k % 4])
              for k, n in enumerate(np.rint(10 ** rng.uniform(0.8, 3.6, 40)))]
    meshes.insert(7, empty_mesh())
    ctx.set_param(lib.PARAM_WALK_CAP, walk_cap)
    ctx.set_param(lib.PARAM_REGION_LDS_MAX, lds_max)
    ctx.set_param(lib.PARAM_REGION_MEM_MAX, mem_max)
    if group:
        ctx.set_param(lib.PARAM_BATCH_GROUP_HE, group)
    try:
        batch = lib.Batch.from_meshes(meshes)
        labels = lib.Labels.empty(batch)
        out = ctx.mesh_batched(batch, labels)
        ctx.status()
        _say(f"  stats {ctx.stats()}")
    finally:
        ctx.set_param(lib.PARAM_WALK_CAP, 24)
        ctx.set_param(lib.PARAM_REGION_LDS_MAX, 4096)
        ctx.set_param(lib.PARAM_REGION_MEM_MAX, 65536)
        ctx.set_param(lib.PARAM_BATCH_GROUP_HE, (1 << 30) - (1 << 24))
    check_batch_against_oracle(meshes, out, labels, batch.he_off_host.numpy())
    st = ctx.stats()
    assert st["seeds"] == sum(oracle.oracle_on(m)["stats"]["seeds"] for m in meshes)


@pytest.mark.parametrize("emit_max", [0, 1030])
def test_emitter_direct_stores(ctx, emit_max):
    """Emitter tiles with more output polygons than the LDS staging holds
    write offsets and start half-edges directly: with the limit lowered to
    0 (every tile) or 1030 (a full tile of 1024 polygon records with more
    than 6 splits goes direct, the others stay in LDS), single meshes and a
    batch (int64 CSR, mesh-local ids) still equal the oracle."""
    from paper_2204_05438_amd import lib
    _say(f"emitter direct stores emit_max {emit_max}")
    ctx.set_param(lib.PARAM_EMIT_LDS_MAX, emit_max)
    try:
        for k, kind in enumerate(["uniform", "cluster", "lattice"]):
            mesh = random_mesh(2100 + k, 20000, kind)
            assert_same(gpu_mesh(ctx, mesh), oracle.oracle_on(mesh), FULL)
        rng = np.random.default_rng(12)
        meshes = [random_mesh(2200 + k, int(n), ["uniform", "cluster", "lattice"][k % 3])
                  for k, n in enumerate(np.rint(10 ** rng.uniform(1.0, 3.8, 24)))]
        meshes.insert(5, empty_mesh())
        batch = lib.Batch.from_meshes(meshes)
        labels = lib.Labels.empty(batch)
        out = ctx.mesh_batched(batch, labels)
        ctx.status()
    finally:
        ctx.set_param(lib.PARAM_EMIT_LDS_MAX, 1536)
    check_batch_against_oracle(meshes, out, labels, batch.he_off_host.numpy())


def test_batched_recipe_against_oracle(ctx):
    """120 meshes of the batched workload's recipe (uniform points, sizes
    log-uniform, here in [1e3, 2e4]) in one call, each against the oracle."""
    _say("batched recipe, 120 meshes")
    from meshgen.gen import batch_points, mesh_from_points
    from paper_2204_05438_amd import lib
    sizes = np.rint(10 ** np.random.default_rng(4).uniform(3.0, 4.3, 120)).astype(int)
    meshes = [mesh_from_points(batch_points(m, int(n))) for m, n in enumerate(sizes)]
    batch = lib.Batch.from_meshes(meshes)
    labels = lib.Labels.empty(batch)
    out = ctx.mesh_batched(batch, labels)
    ctx.status()
    check_batch_against_oracle(meshes, out, labels, batch.he_off_host.numpy())


def test_batched_bad_mesh_reported(ctx):
    """A local twin or origin outside its own mesh is reported (ETOPO), not
    taken as an index into a neighbouring mesh."""
    _say("batched: out-of-range local index")
    from paper_2204_05438_amd import lib
    meshes = [random_mesh(40 + k, 200, "uniform") for k in range(3)]
    for field, value in (("twin", None), ("origin", None)):
        batch = lib.Batch.from_meshes(meshes)
        H0 = meshes[0].n_halfedges
        arr = getattr(batch, field)
        if field == "twin":
            arr[H0 + 5] = meshes[1].n_halfedges + 2   # a half-edge of mesh 2 in global numbering
        else:
            arr[H0 + 5] = meshes[1].n_vertices + 1
        ctx.mesh_batched(batch)
        assert ctx.status(raise_on_error=False) == lib.ETOPO, field
    batch = lib.Batch.from_meshes(meshes)
    out = ctx.mesh_batched(batch)
    ctx.status()
    check_batch_against_oracle(meshes, out)


def test_batched_capacity_error(ctx):
    """Too small an output: ECAPACITY and every poly_off entry -1."""
    _say("batched: capacity error")
    from paper_2204_05438_amd import lib
    meshes = [random_mesh(60 + k, 300, "uniform") for k in range(4)]
    batch = lib.Batch.from_meshes(meshes)
    for group in (0, 3):
        if group:
            ctx.set_param(lib.PARAM_BATCH_GROUP_HE, group)
        try:
            out = lib.BatchOut.empty(batch, cap_polys=50, cap_verts=200)
            ctx.mesh_batched(batch, None, out)
            assert ctx.status(raise_on_error=False) == lib.ECAPACITY
            assert (out.poly_off.cpu().numpy() == -1).all()
        finally:
            ctx.set_param(lib.PARAM_BATCH_GROUP_HE, (1 << 30) - (1 << 24))
    out = ctx.mesh_batched(batch)
    ctx.status()
    check_batch_against_oracle(meshes, out)


def test_batched_graph_replay(ctx):
    """polylla_mesh_batched captured in a HIP graph: every replay, with eager
    work and synchronisation between replays, equals the eager call (also
    with the batch cut into several groups)."""
    _say("batched graph replay, 24 meshes")
    from paper_2204_05438_amd import lib
    rng = np.random.default_rng(21)
    kinds = ["uniform", "cluster", "grid", "lattice"]
    meshes = [random_mesh(600 + k, int(n), kinds[k % 4])
              for k, n in enumerate(np.rint(10 ** rng.uniform(1.0, 3.7, 24)))]
    batch = lib.Batch.from_meshes(meshes)
    for group in (0, 20000):
        if group:
            ctx.set_param(lib.PARAM_BATCH_GROUP_HE, group)
        labels = lib.Labels.empty(batch)
        out = lib.BatchOut.empty(batch)

        def snapshot():
            off, verts, start, po = (x.cpu().numpy().copy() for x in out.trimmed())
            return off, verts, start, po, labels.he.cpu().numpy().copy()

        try:
            ctx.mesh_batched(batch, labels, out)
            ctx.status()
            ref = snapshot()
            side = torch.cuda.Stream()
            side.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(side):
                ctx.mesh_batched(batch, labels, out)
            torch.cuda.current_stream().wait_stream(side)
            torch.cuda.synchronize()
            graph = torch.cuda.CUDAGraph()
            with torch.cuda.graph(graph):
                ctx.mesh_batched(batch, labels, out)
            for rep in range(3):
                out.verts.fill_(-1)
                out.offsets.fill_(-1)
                out.poly_off.fill_(-7)
                labels.he.zero_()
                torch.cuda.synchronize()
                graph.replay()
                torch.cuda.synchronize()
                assert ctx.status(raise_on_error=False) == lib.OK, rep
                got = snapshot()
                for a, b, name in zip(got, ref, ["offsets", "verts", "start", "poly_off", "he"]):
                    assert np.array_equal(a, b), (group, rep, name)
            del graph
        finally:
            ctx.set_param(lib.PARAM_BATCH_GROUP_HE, (1 << 30) - (1 << 24))
    check_batch_against_oracle(meshes, out)


def test_batched_beyond_2e31_halfedges(ctx):
    """One mesh replicated on the device until the batch holds more than 2^31
    half-edges (int64 offsets, several groups): every copy's polygons equal
    that mesh's oracle output."""
    from paper_2204_05438_amd import lib
    mesh = config_mesh("mixed200k")
    H, V = mesh.n_halfedges, mesh.n_vertices
    n = (1 << 31) // H + 2
    _say(f"batched: {n} copies of mixed200k, {n * H} half-edges")
    o = oracle.oracle_on(mesh)
    dev = torch.device("cuda")
    ho = torch.arange(n + 1, dtype=torch.int64) * H
    vo = torch.arange(n + 1, dtype=torch.int64) * V
    batch = lib.Batch(xy=torch.from_numpy(mesh.xy).to(dev).repeat(n, 1),
                      twin=torch.from_numpy(mesh.twin).to(dev).repeat(n),
                      origin=torch.from_numpy(mesh.origin).to(dev).repeat(n),
                      vtx_off=vo.to(dev), he_off=ho.to(dev), vtx_off_host=vo, he_off_host=ho)
    F1, S1 = o["offsets"].size - 1, o["verts"].size
    out = lib.BatchOut.empty(batch, cap_polys=n * F1, cap_verts=n * S1, with_start=False)
    ctx.mesh_batched(batch, None, out)
    ctx.status()
    _say(f"  stats {ctx.stats()}")
    assert out.counts.tolist() == [n * F1, n * S1]
    po = out.poly_off
    assert torch.equal(po, torch.arange(n + 1, dtype=torch.int64, device=dev) * F1)
    ref_off = torch.from_numpy(o["offsets"].astype(np.int64)).to(dev)
    ref_verts = torch.from_numpy(o["verts"]).to(dev)
    for k in range(n):
        got_off = out.offsets[k * F1:(k + 1) * F1 + 1] - k * S1
        assert torch.equal(got_off, ref_off), k
        assert torch.equal(out.verts[k * S1:(k + 1) * S1], ref_verts), k


@pytest.mark.parametrize("items", [1, 2, 4])
def test_longest_items_param(ctx, items):
    """Each triangles-per-thread setting of the longest-edge kernel gives the
    oracle's labels and polygons (sizes that leave ragged tails)."""
    from paper_2204_05438_amd import lib
    ctx.set_param(lib.PARAM_LONGEST_ITEMS, items)
    try:
        for n, kind in ((37, "uniform"), (1001, "lattice"), (4097, "cluster")):
            _say(f"longest items {items} {kind} n {n}")
            mesh = random_mesh(5100 + n, n, kind)
            assert_same(gpu_mesh(ctx, mesh), oracle.oracle_on(mesh), FULL)
        with pytest.raises(lib.PolyllaError):
            ctx.set_param(lib.PARAM_LONGEST_ITEMS, 3)
    finally:
        ctx.set_param(lib.PARAM_LONGEST_ITEMS, 2)
