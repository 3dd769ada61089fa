"""Pins of the CPU oracle against hand-derived values, brute force on tiny
meshes and invariants that hold at any size. No GPU involved."""
import math

import numpy as np
import pytest

import oracle
from bruteforce import BARRIER, FRONTIER, REPAIRED, TERMINAL, Brute, canonical, csr_cycles
from fixtures import empty_mesh, golden, golden_names, random_mesh, spiral_fan
from meshgen.gen import config_mesh, mesh_from_points


def run(mesh):
    return oracle.oracle_on(mesh)


@pytest.mark.parametrize("name", golden_names())
def test_golden_fixture(name):
    mesh, g = golden(name)
    o = run(mesh)
    assert o["he"].tolist() == g["he"]
    assert o["tri"].tolist() == g["tri"]
    assert o["vtx"].tolist() == g["vtx"]
    assert csr_cycles(o["pre_offsets"], o["pre_verts"]) == [tuple(c) for c in g["pre"]]
    assert csr_cycles(o["offsets"], o["verts"]) == [tuple(c) for c in g["final"]]


def test_empty_mesh():
    o = run(empty_mesh())
    assert o["offsets"].tolist() == [0] and o["verts"].size == 0


def test_layout_errors():
    mesh, _ = golden("square")
    bad = mesh.twin.copy()
    bad[2] = 4  # twin no longer an involution
    o = oracle.oracle_mesh(mesh.xy, bad, mesh.next, mesh.origin, check=False)
    assert o["rc"] == -3
    nx = mesh.next.copy()
    nx[0] = 2
    o = oracle.oracle_mesh(mesh.xy, mesh.twin, nx, mesh.origin, check=False)
    assert o["rc"] == -2
    o = oracle.oracle_mesh(mesh.xy, mesh.twin[:5], mesh.next[:5], mesh.origin[:5], check=False)
    assert o["rc"] == -2


def _compare_with_brute(mesh):
    o = run(mesh)
    b = Brute(mesh).mesh_pipeline()
    # labels before repair: LONGEST, FRONTIER, TERMINAL, BORDER, CONSTRAINED, SEED
    pre_mask = 1 | 2 | 4 | 8 | 64
    he_pre = o["he"] & pre_mask
    he_pre = np.where(o["he"] & REPAIRED, he_pre & np.uint8(0xFF ^ FRONTIER), he_pre)
    assert np.array_equal(he_pre, b["he"])
    assert np.array_equal(o["tri"], b["seed"])
    # polygons before repair: same cycles, one per region, listed by seed
    pre = csr_cycles(o["pre_offsets"], o["pre_verts"])
    assert sorted(pre) == sorted(canonical(c) for c in b["pre"])
    assert len(pre) == len(set(b["comp"])) == int(o["tri"].sum())
    # polygons after repair
    fin = csr_cycles(o["offsets"], o["verts"])
    assert sorted(fin) == sorted(canonical(c) for c in b["final"])
    # repaired edges: exactly those the brute-force pass loop added
    tri = mesh.origin.reshape(-1, 3)
    rep = {frozenset((int(tri[h // 3][h % 3]), int(tri[h // 3][(h % 3 + 1) % 3])))
           for h in np.nonzero(o["he"] & REPAIRED)[0]}
    assert rep == b["extra"]
    # barrier edges and barrier-edge tips of the polygons before repair
    assert np.array_equal(o["he"] & BARRIER, b["barrier"])
    assert set(np.nonzero(o["vtx"] & 1)[0].tolist()) == b["tips"]
    return o


def with_segments(mesh, seed, frac):
    """The mesh with a seeded random subset of its interior edges made
    segments of the input (both half-edges flagged)."""
    rng = np.random.default_rng(seed)
    o, tw = mesh.origin, mesh.twin
    h = np.arange(o.size)
    inner = np.nonzero((tw >= 0) & (h < tw))[0]
    pick = inner[rng.random(inner.size) < frac]
    fixed = np.zeros(o.size, np.uint8)
    fixed[pick] = 1
    fixed[tw[pick]] = 1
    mesh.fixed = fixed
    return mesh


@pytest.mark.parametrize("kind", ["uniform", "cluster", "grid", "lattice"])
@pytest.mark.parametrize("seed", range(8))
def test_oracle_vs_bruteforce_segments(kind, seed):
    """Input segments (a planar straight-line graph): each side of a segment
    is labelled like a boundary edge; labels, regions, barrier edges, tips
    and the repair against the brute force."""
    n = [8, 15, 30, 50, 80, 120, 200, 300][seed]
    frac = [0.05, 0.1, 0.2, 0.35][seed % 4]
    _compare_with_brute(with_segments(random_mesh(3000 + 17 * seed, n, kind), 5 + seed, frac))


@pytest.mark.parametrize("kind", ["uniform", "cluster", "grid", "lattice"])
@pytest.mark.parametrize("seed", range(12))
def test_oracle_vs_bruteforce(kind, seed):
    n = [6, 12, 25, 40, 60, 90, 120, 160, 200, 250, 300, 20][seed]
    _compare_with_brute(random_mesh(1000 * seed + 7, n, kind))


# Tiny meshes chosen (by their seeds) because they reach the rare corners of
# the repair: a split at a smaller tip that removes a larger tip of the same
# polygon (fewer splits than tips: Algorithm 4 repeated per Algorithm 1 finds
# the second tip gone on the next pass), and a region that touches itself at a
# vertex without a barrier edge (a pinched cycle, which the tip rule leaves as
# it is). The brute force decides every expected value.
KILLED_TIP_CASES = [("cluster", 30, 143), ("cluster", 30, 229), ("cluster", 30, 112),
                    ("uniform", 30, 193), ("cluster", 30, 118)]
PINCH_CASES = [("cluster", 30, 383), ("cluster", 60, 315), ("cluster", 100, 130)]


@pytest.mark.parametrize("kind,n,seed", KILLED_TIP_CASES)
def test_killed_tip_vs_bruteforce(kind, n, seed):
    mesh = random_mesh(seed * 7919 + n, n, kind)
    o = _compare_with_brute(mesh)
    b = Brute(mesh).mesh_pipeline()
    assert len(b["tips"]) > len(b["extra"]), "the case must remove a tip without a split"
    assert o["stats"]["tips"] == len(b["tips"]) and o["stats"]["splits"] == len(b["extra"])


@pytest.mark.parametrize("kind,n,seed", PINCH_CASES)
def test_pinched_region_vs_bruteforce(kind, n, seed):
    mesh = random_mesh(seed * 7919 + n, n, kind)
    o = _compare_with_brute(mesh)
    b = Brute(mesh).mesh_pipeline()
    pinched = [c for c in b["final"] if len(set(c)) < len(c)]
    assert pinched, "the case must keep a cycle with a repeated vertex"
    assert o["stats"]["nonsimple_final"] == len(pinched)


def test_bruteforce_sees_repairs():
    # the random cases above must actually exercise the repair
    total = 0
    for seed in range(12):
        o = run(random_mesh(1000 * seed + 7, 300, "uniform"))
        total += o["stats"]["splits"]
    assert total > 0


def _invariants(mesh, o):
    T = mesh.n_tri
    H = mesh.n_halfedges
    he, tri = o["he"], o["tri"]
    R = int(tri.sum())
    tw = mesh.twin
    # each triangle has exactly one longest edge
    assert np.all((he.reshape(T, 3) & 1).sum(1) == 1)
    # terminal edges are the mutual longest edges; seeds = terminal edges (once)
    inner = tw >= 0
    mutual = inner & (he & 1 > 0) & (he[np.where(inner, tw, 0)] & 1 > 0)
    border_term = (~inner) & (he & 1 > 0)
    assert np.array_equal((he & TERMINAL) > 0, mutual | border_term)
    assert R == int(mutual.sum()) // 2 + int(border_term.sum())
    # frontier edges before repair: E - T + R (each region is a tree of k-1 internal edges)
    E = (H + int((~inner).sum())) // 2
    pre_front = ((he & FRONTIER) > 0) & ((he & REPAIRED) == 0)
    n_front_edges = (int(pre_front.sum()) + int((pre_front & ~inner).sum())) // 2
    assert n_front_edges == E - T + R
    # sum of cycle lengths: T + 2F before and after repair
    Fp = len(o["pre_offsets"]) - 1
    F = len(o["offsets"]) - 1
    assert Fp == R
    assert o["pre_verts"].size == T + 2 * Fp
    assert o["verts"].size == T + 2 * F
    # every split adds one frontier edge and one polygon
    assert int((he & REPAIRED).sum() // REPAIRED) == 2 * (F - Fp)
    # Euler on the frontier graph of the final mesh (convex domain)
    fr = (he & FRONTIER) > 0
    Ef = (int(fr.sum()) + int((fr & ~inner).sum())) // 2
    Vf = np.unique(mesh.origin[fr]).size
    assert Vf - Ef + F == 1
    # areas: each cycle is CCW and the areas add up to the triangulation's
    xy = mesh.xy
    P = mesh.origin.reshape(T, 3)
    a, b, c = xy[P[:, 0]], xy[P[:, 1]], xy[P[:, 2]]
    tri_area = 0.5 * ((b[:, 0] - a[:, 0]) * (c[:, 1] - a[:, 1]) - (b[:, 1] - a[:, 1]) * (c[:, 0] - a[:, 0]))
    off, v = o["offsets"], o["verts"]
    L = np.diff(off)
    x, y = xy[v, 0], xy[v, 1]
    nxt = np.arange(v.size) + 1
    nxt[off[1:] - 1] = off[:-1]
    cross = x * y[nxt] - x[nxt] * y
    areas = 0.5 * np.add.reduceat(cross, off[:-1]) if F else np.zeros(0)
    assert np.all(areas > 0)
    assert math.isclose(areas.sum(), tri_area.sum(), rel_tol=1e-9)
    # no tip remains; cycles start at their smallest vertex
    starts = v[off[:-1]]
    for i in range(F):
        cyc = v[off[i]:off[i + 1]]
        assert starts[i] == cyc.min()
        n = cyc.size
        assert not np.any(cyc == np.roll(cyc, -2)) or n < 3
    # a triangle with three frontier edges is a polygon on its own
    three = np.nonzero(((he.reshape(T, 3) & FRONTIER) > 0).all(1))[0]
    polys3 = {tuple(v[off[i]:off[i + 1]]) for i in np.nonzero(L == 3)[0]}
    for t in three[:1000]:
        assert canonical(tuple(int(x) for x in P[t])) in polys3
    # barrier edges are frontier edges with both half-edges on one polygon before repair
    bar = (he & BARRIER) > 0
    assert np.all(fr[bar]) and np.all(bar[tw[bar]])


@pytest.mark.parametrize("name", ["uniform10k", "mixed50k", "grid120x"])
def test_invariants_workloads(name):
    mesh = config_mesh(name)
    _invariants(mesh, run(mesh))


@pytest.mark.slow
def test_invariants_1m():
    mesh = config_mesh("mixed1m")
    _invariants(mesh, run(mesh))


def test_rotation_and_relabel_invariance():
    """Renumbering triangles and rotating their vertex triples only permutes
    half-edge indices; away from exact length ties the polygons must not change."""
    mesh = random_mesh(99, 400, "uniform")
    o1 = run(mesh)
    rng = np.random.default_rng(5)
    T = mesh.n_tri
    perm = rng.permutation(T)
    rot = rng.integers(0, 3, T)
    tris = mesh.origin.reshape(T, 3)[perm]
    tris = np.stack([tris[np.arange(T), (rot + k) % 3] for k in range(3)], 1)
    from meshgen.gen import mesh_from_triangles
    m2 = mesh_from_triangles(mesh.xy, tris)
    o2 = run(m2)
    assert sorted(csr_cycles(o1["offsets"], o1["verts"])) == sorted(csr_cycles(o2["offsets"], o2["verts"]))


@pytest.mark.parametrize("n,seed", [(600, 1), (1500, 2), (3000, 3)])
def test_oracle_vs_bruteforce_pslg(n, seed):
    """Triangulations of planar straight-line graphs (holes and cracks, the
    generator's recipe at small sizes) against the brute force."""
    from meshgen.gen import pslg_mesh, validate
    mesh = pslg_mesh(n, 3, 3, seed)
    validate(mesh)
    assert mesh.meta["holes"] == 3 and mesh.meta["cracks"] == 3
    o = _compare_with_brute(mesh)
    assert o["stats"]["splits"] > 0


def test_pslg_regions_stay_inside_the_domain():
    """Every polygon of a PSLG mesh lies inside the domain: its vertex cycle
    never runs along a segment's two sides except as a barrier edge, every
    triangle is in one region, and the polygons' areas add up to the
    triangulation's (holes excluded)."""
    from meshgen.gen import config_mesh
    mesh = config_mesh("pslg20k")
    o = run(mesh)
    he = o["he"]
    fx = mesh.fixed.astype(bool)
    assert np.all((he[fx & (mesh.twin >= 0)] & FRONTIER) > 0)
    assert np.array_equal((he & 64) > 0, fx & (mesh.twin >= 0))
    T = mesh.n_tri
    P = mesh.origin.reshape(T, 3)
    xy = mesh.xy
    a, b, c = xy[P[:, 0]], xy[P[:, 1]], xy[P[:, 2]]
    tri_area = 0.5 * ((b[:, 0] - a[:, 0]) * (c[:, 1] - a[:, 1]) - (b[:, 1] - a[:, 1]) * (c[:, 0] - a[:, 0]))
    off, v = o["offsets"], o["verts"]
    x, y = xy[v, 0], xy[v, 1]
    nxt = np.arange(v.size) + 1
    nxt[off[1:] - 1] = off[:-1]
    areas = 0.5 * np.add.reduceat(x * y[nxt] - x[nxt] * y, off[:-1])
    assert np.all(areas > 0)
    assert math.isclose(areas.sum(), tri_area.sum(), rel_tol=1e-9)
    assert v.size == T + 2 * (off.size - 1)



@pytest.mark.parametrize("name", ["fan7_tip", "square", "square_segment"])
def test_lepp_golden(name):
    mesh, g = golden(name)
    term, length = oracle.oracle_lepp(mesh)
    assert term.tolist() == g["lepp_terminal"]
    assert length.tolist() == g["lepp_length"]


@pytest.mark.parametrize("kind", ["uniform", "cluster", "grid", "lattice"])
@pytest.mark.parametrize("seed", range(6))
def test_lepp_vs_bruteforce(kind, seed):
    """Lepp of every triangle against the brute force (with and without input
    segments); every path ends at a terminal edge (TERMINAL bit), and all the
    triangles of one terminal-edge region end at the same edge."""
    mesh = random_mesh(5100 + seed, [10, 40, 90, 160, 250, 400][seed], kind)
    if seed % 2:
        mesh = with_segments(mesh, seed, 0.15)
    term, length = oracle.oracle_lepp(mesh)
    b = Brute(mesh)
    assert [(int(x), int(y)) for x, y in zip(term, length)] == b.lepp()
    o = run(mesh)
    assert np.all(o["he"][term] & TERMINAL)
    lg, he, seed_flags = b.labels()
    front = {(t, i) for t in range(b.T) for i in range(3) if he[3 * t + i] & FRONTIER}
    comp = b.regions(lambda t, i: (t, i) in front)
    by_region = {}
    for t, r in enumerate(comp):
        assert by_region.setdefault(r, term[t]) == term[t]
    assert len(by_region) == int(o["tri"].sum())


@pytest.mark.parametrize("n", [7, 40, 300])
def test_lepp_spiral_fan_closed_form(n):
    """A fan whose spokes grow by 0.001 per step: every path runs to the last
    spoke, n - i triangles from triangle i (2 from the last one)."""
    term, length = oracle.oracle_lepp(spiral_fan(n))
    assert (term == 3 * n - 4).all()
    assert length.tolist() == [n - i for i in range(n - 1)] + [2]
