"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

The oracle computes the power cells of paper Sec. 3 Eq. 1 clipped to a box.
None of these tests retypes its formulas: each compares it with something
independent -- an exact-rational vertex enumeration, closed forms of box
slabs and of cube/half-space intersections, Qhull (Delaunay and the lifted
convex hull of Aurenhammer's lifting map), and invariants any partition of
the box into cells must satisfy.
"""
import itertools
from fractions import Fraction as Q

import numpy as np
import pytest

from oracle import brute
from paper_2605_06408_amd import workloads as wl

UNIT = np.array([0.0, 0.0, 0.0, 1.0, 1.0, 1.0])


def _cell_lists(res):
    n = len(res["vol"])
    return [res["nbr"][res["nbr_off"][i]:res["nbr_off"][i + 1]] for i in range(n)]


# ---------------------------------------------------------------- closed forms

def test_single_site_is_the_box(oracle_mod):
    box = np.array([-1.0, 0.5, 2.0, 3.0, 1.5, 2.25])
    r = oracle_mod.cells(np.array([[0.2, 0.7, 2.1]], np.float32), None, box)
    c = oracle_mod.cell_view(r, 0)
    assert c["vol"] == pytest.approx(4.0 * 1.0 * 0.25, rel=1e-14)
    np.testing.assert_allclose(c["centroid"], [1.0, 1.0, 2.125], rtol=1e-14)
    assert len(c["vert"]) == 8 and len(c["nbr"]) == 0
    assert [f[0] for f in c["facets"]] == [-6, -5, -4, -3, -2, -1]
    corners = {tuple(v) for v in c["vert"]}
    assert corners == set(itertools.product([-1.0, 3.0], [0.5, 1.5], [2.0, 2.25]))


@pytest.mark.parametrize("w0,w1", [(0.0, 0.0), (0.1, 0.0), (0.0, 0.3), (0.05, 0.2), (0.7, 0.0), (0.0, 0.7)])
def test_two_sites_axis_aligned(oracle_mod, w0, w1):
    # p0=(1/4,1/2,1/2), p1=(3/4,1/2,1/2): the radical plane is x = 1/2 + w0 - w1,
    # so cell 0 is the slab [0, x*] x [0,1]^2 (clamped to the box).
    xyz = np.array([[0.25, 0.5, 0.5], [0.75, 0.5, 0.5]], np.float32)
    w = np.array([w0, w1], np.float32)
    xs = min(max(0.5 + float(w[0]) - float(w[1]), 0.0), 1.0)
    r = oracle_mod.cells(xyz, w, UNIT)
    assert r["vol"][0] == pytest.approx(xs, abs=1e-15)
    assert r["vol"][1] == pytest.approx(1.0 - xs, abs=1e-15)
    for i, (lo, hi) in enumerate([(0.0, xs), (xs, 1.0)]):
        if hi > lo:
            np.testing.assert_allclose(r["centroid"][i], [(lo + hi) / 2, 0.5, 0.5], rtol=1e-14)
            assert list(_cell_lists(r)[i]) == [1 - i] if 0 < xs < 1 else True
        else:
            assert r["flags"][i] & oracle_mod.FLAG_EMPTY
            np.testing.assert_array_equal(r["centroid"][i], xyz[i].astype(np.float64))


def _cube_halfspace_volume(a, b):
    """Volume of [0,1]^3 intersected with {x : a.x <= b}, all a_k != 0, by
    inclusion-exclusion over the cube's corners (exact rationals)."""
    a = [Q(x) for x in a]
    b = Q(b)
    for k in range(3):
        if a[k] < 0:  # reflect x_k -> 1 - x_k
            b -= a[k]
            a[k] = -a[k]
    tot = Q(0)
    for v in itertools.product([0, 1], repeat=3):
        t = b - sum(a[k] * v[k] for k in range(3))
        if t > 0:
            tot += (-1) ** sum(v) * t ** 3
    return tot / (6 * a[0] * a[1] * a[2])


@pytest.mark.parametrize("seed", range(6))
def test_two_sites_general_direction(oracle_mod, seed):
    rng = np.random.default_rng(seed)
    xyz = rng.random((2, 3)).astype(np.float32)
    w = (rng.normal(size=2) * 0.05).astype(np.float32)
    p0 = [Q(float(c)) for c in xyz[0]]
    p1 = [Q(float(c)) for c in xyz[1]]
    a = [2 * (p1[k] - p0[k]) for k in range(3)]
    b = sum(c * c for c in p1) - sum(c * c for c in p0) + Q(float(w[0])) - Q(float(w[1]))
    v0 = _cube_halfspace_volume(a, b)
    r = oracle_mod.cells(xyz, w, UNIT)
    assert r["vol"][0] == pytest.approx(float(v0), rel=1e-12, abs=1e-15)
    assert r["vol"][1] == pytest.approx(float(1 - v0), rel=1e-12, abs=1e-15)


# ----------------------------------------------------- exact vertex enumeration

def _brute_cases():
    rng = np.random.default_rng(7)
    cases = []
    for seed in range(3):
        xyz, _, box = wl.uniform(11, seed)
        cases.append(("voronoi", xyz, None, box))
    for seed in range(3):
        xyz, _, box = wl.uniform(10, 10 + seed)
        w = (rng.random(10) * 0.06).astype(np.float32)
        cases.append(("power", xyz, w, box))
    xyz = (rng.random((10, 3)) * 1.4 - 0.2).astype(np.float32)  # some sites outside the box
    cases.append(("outside", xyz, (rng.random(10) * 0.02).astype(np.float32), np.array([0.1, 0.0, 0.05, 0.9, 1.0, 0.8])))
    xyz = rng.random((9, 3)).astype(np.float32)
    xyz[6] = xyz[2]
    w = np.zeros(9, np.float32)
    cases.append(("coincident_equal", xyz, w, UNIT))
    w = w.copy()
    w[6] = 0.01
    cases.append(("coincident_heavier", xyz, w, UNIT))
    return cases


@pytest.mark.parametrize("case", _brute_cases(), ids=lambda c: c[0])
def test_against_exact_vertex_enumeration(oracle_mod, case):
    _, xyz, w, box = case
    r = oracle_mod.cells(xyz, w, box)
    for i in range(len(xyz)):
        ex = brute.cell(xyz, w, box, i)
        c = oracle_mod.cell_view(r, i)
        assert not ex["degenerate"]
        assert bool(c["flags"] & oracle_mod.FLAG_EMPTY) == ex["empty"]
        keys = [tuple(int(x) for x in k) for k in c["vert_code"]]
        assert keys == sorted(ex["vertices"].keys()), i
        for k, pos in zip(keys, c["vert"]):
            np.testing.assert_allclose(pos, [float(x) for x in ex["vertices"][k]], rtol=0, atol=1e-13)
        assert set(int(x) for x in c["nbr"]) == ex["nbr"]
        assert c["vol"] == pytest.approx(float(ex["vol"]), rel=1e-12, abs=1e-16)


def test_coincident_rule(oracle_mod):
    xyz, _, box = wl.uniform(40, 3)
    dup = np.vstack([xyz, xyz[[5]]])
    base = oracle_mod.cells(xyz, None, box)
    r = oracle_mod.cells(dup, None, box)
    # equal weights: the lower index (5) keeps its cell, the copy (40) is empty
    assert r["flags"][40] & oracle_mod.FLAG_EMPTY
    np.testing.assert_array_equal(r["vol"][:40], base["vol"])
    w = np.zeros(41, np.float32)
    w[40] = 1e-3
    r2 = oracle_mod.cells(dup, w, box)
    assert r2["flags"][5] & oracle_mod.FLAG_EMPTY and not r2["flags"][40] & oracle_mod.FLAG_EMPTY


# ------------------------------------------------------------- library pins

def test_voronoi_adjacency_matches_qhull_delaunay(oracle_mod):
    from scipy.spatial import Delaunay
    xyz, _, box = wl.uniform(3000, 11)
    r = oracle_mod.cells(xyz, None, box)
    tri = Delaunay(xyz.astype(np.float64))
    nb = [set() for _ in range(len(xyz))]
    for s in tri.simplices:
        for a, b in itertools.combinations(s, 2):
            nb[a].add(int(b))
            nb[b].add(int(a))
    lists = _cell_lists(r)
    checked = 0
    for i in range(len(xyz)):
        codes = r["facet_code"][r["facet_off"][i]:r["facet_off"][i + 1]]
        if codes.min() < 0 or r["margin"][i] < 1e-6:
            continue  # touches the box, or too close to degenerate for Qhull
        assert set(int(x) for x in lists[i]) == nb[i], i
        checked += 1
    assert checked > 1500


def _lower_hull_edges(xyz, w):
    from scipy.spatial import ConvexHull
    p = xyz.astype(np.float64)
    lifted = np.hstack([p, (p * p).sum(1, keepdims=True) - w.astype(np.float64)[:, None]])
    hull = ConvexHull(lifted)
    nb = [set() for _ in range(len(xyz))]
    on_lower = np.zeros(len(xyz), bool)
    for s, eq in zip(hull.simplices, hull.equations):
        if eq[3] < 0:  # facet faces downward in the lifted coordinate
            on_lower[s] = True
            for a, b in itertools.combinations(s, 2):
                nb[a].add(int(b))
                nb[b].add(int(a))
    return nb, on_lower


@pytest.mark.parametrize("law", ["paper_gaussian", "lognormal"])
def test_power_adjacency_matches_lifted_hull(oracle_mod, law):
    n = 2000
    rng = np.random.default_rng(5)
    xyz = rng.random((n, 3)).astype(np.float32)
    if law == "paper_gaussian":
        from scipy.spatial import cKDTree
        d, _ = cKDTree(xyz).query(xyz, k=2)
        dnn = np.median(d[:, 1])
        w = rng.normal(0.0, dnn * dnn / 3.0, size=n).astype(np.float32)
    else:
        w = wl.power_uniform(n, 5)[1]
    r = oracle_mod.cells(xyz, w, UNIT)
    nb, on_lower = _lower_hull_edges(xyz, w)
    empty = (r["flags"] & oracle_mod.FLAG_EMPTY) != 0
    # a site off the lower hull has no cell anywhere, so none inside the box
    assert np.all(empty[~on_lower])
    lists = _cell_lists(r)
    checked = 0
    for i in range(n):
        codes = r["facet_code"][r["facet_off"][i]:r["facet_off"][i + 1]]
        if empty[i] or codes.min() < 0 or r["margin"][i] < 1e-6:
            continue
        assert set(int(x) for x in lists[i]) == nb[i], i
        checked += 1
    assert checked > (50 if law == "lognormal" else 1000)


# ------------------------------------------------------------------ invariants

def _invariant_sets():
    xyz, _, box = wl.uniform(1500, 2)
    yield "voronoi", xyz, None, box
    xyz, w, box = wl.power_uniform(1500, 2)
    yield "power_lognormal", xyz, w, box
    xyz, _, box = wl.clustered(3000, 4)
    yield "clustered", xyz, None, box
    xyz, _, box = wl.surface(3000, 4)
    yield "surface", xyz, None, box


@pytest.mark.parametrize("case", list(_invariant_sets()), ids=lambda c: c[0])
def test_partition_invariants(oracle_mod, case):
    _, xyz, w, box = case
    r = oracle_mod.cells(xyz, w, box)
    n = len(xyz)
    bvol = np.prod(box[3:] - box[:3])
    bcen = (box[:3] + box[3:]) / 2
    assert r["vol"].sum() == pytest.approx(bvol, rel=1e-12)
    np.testing.assert_allclose((r["vol"][:, None] * r["centroid"]).sum(0), bvol * bcen, rtol=1e-11)
    assert np.all(r["vol"] >= 0)
    lists = _cell_lists(r)
    sets = [set(int(x) for x in l) for l in lists]
    for i in range(n):
        assert list(lists[i]) == sorted(lists[i])
        for j in sets[i]:
            assert i in sets[j], (i, j)  # symmetric neighbour relation
    empty = (r["flags"] & oracle_mod.FLAG_EMPTY) != 0
    for i in np.nonzero(empty)[0]:
        assert len(sets[i]) == 0 and r["vol"][i] == 0
        np.testing.assert_array_equal(r["centroid"][i], xyz[i].astype(np.float64))
    for i in range(n):
        if empty[i]:
            continue
        v0, v1 = r["vert_off"][i], r["vert_off"][i + 1]
        f0, f1 = r["facet_off"][i], r["facet_off"][i + 1]
        nv, nf = v1 - v0, f1 - f0
        sizes = np.diff(r["fv_off"][f0:f1 + 1])
        assert sizes.sum() == 3 * nv and nf == nv // 2 + 2  # simple polytope, Euler
        # every facet is CCW seen from outside: its Newell normal points along
        # the outward normal (p_j - p_i for a site, the axis for a box face)
        verts = r["vert"][v0:v1]
        for f in range(f0, f1):
            ring = verts[r["fv"][r["fv_off"][f]:r["fv_off"][f + 1]]]
            nrm = np.cross(ring, np.roll(ring, -1, axis=0)).sum(0)
            code = r["facet_code"][f]
            if code >= 0:
                out = xyz[code].astype(np.float64) - xyz[i].astype(np.float64)
            else:
                ax = (-code - 1) // 2
                out = np.zeros(3)
                out[ax] = 1.0 if (-code - 1) % 2 else -1.0
            assert np.dot(nrm, out) > 0, (i, code)


def test_shared_facets_agree(oracle_mod):
    xyz, w, box = wl.power_uniform(800, 9)
    w = (w * 0.05).astype(np.float32)  # moderate weights: few empty cells
    r = oracle_mod.cells(xyz, w, box)
    def facet(i, j):
        f0, f1 = r["facet_off"][i], r["facet_off"][i + 1]
        fs = [f for f in range(f0, f1) if r["facet_code"][f] == j]
        assert len(fs) == 1
        f = fs[0]
        idx = r["fv"][r["fv_off"][f]:r["fv_off"][f + 1]]
        v0 = r["vert_off"][i]
        return r["vert"][v0 + idx]
    lists = _cell_lists(r)
    for i in range(len(xyz)):
        for j in lists[i]:
            if j < i:
                continue
            a, b = facet(i, j), facet(j, i)
            assert len(a) == len(b)
            # same polygon traversed in opposite directions
            b = b[::-1]
            k = int(np.argmin(np.abs(b - a[0]).sum(1)))
            np.testing.assert_allclose(np.roll(b, -k, axis=0), a, rtol=0, atol=1e-12)


def test_empty_power_sphere(oracle_mod):
    xyz, w, box = wl.power_uniform(700, 3)
    w = (w * 0.1).astype(np.float32)
    r = oracle_mod.cells(xyz, w, box)
    p = xyz.astype(np.float64)
    wd = w.astype(np.float64)
    for i in range(len(xyz)):
        v0, v1 = r["vert_off"][i], r["vert_off"][i + 1]
        for v, codes in zip(r["vert"][v0:v1], r["vert_code"][v0:v1]):
            if codes.min() < 0:
                continue
            pw = ((p - v) ** 2).sum(1) - wd
            ref = pw[i]
            scale = ((p[i] - v) ** 2).sum() + abs(wd[i]) + 1e-30
            # the four sites of a dual tetrahedron share the power distance ...
            np.testing.assert_allclose(pw[codes], ref, rtol=0, atol=1e-12 * scale)
            # ... and no other site is closer in power distance
            assert pw.min() >= ref - 1e-12 * scale


def test_equal_weights_reproduce_voronoi(oracle_mod):
    xyz, _, box = wl.uniform(500, 1)
    a = oracle_mod.cells(xyz, None, box)
    b = oracle_mod.cells(xyz, np.full(500, 0.125, np.float32), box)
    for k in ["nbr_off", "nbr", "vert", "vert_code", "fv", "vol", "centroid"]:
        np.testing.assert_array_equal(a[k], b[k])


# ------------------------------------------------------------ metamorphic

@pytest.mark.parametrize("k", [3, -2])
def test_power_of_two_scaling_is_exact(oracle_mod, k):
    xyz, w, box = wl.power_uniform(600, 8)
    w = (w * 0.1).astype(np.float32)
    s = np.float32(2.0 ** k)
    a = oracle_mod.cells(xyz, w, box)
    b = oracle_mod.cells(xyz * s, w * s * s, box * float(s))
    for key in ["nbr_off", "nbr", "vert_code", "facet_code", "fv", "flags"]:
        np.testing.assert_array_equal(a[key], b[key])
    np.testing.assert_array_equal(a["vert"] * float(s), b["vert"])
    np.testing.assert_array_equal(a["vol"] * float(s) ** 3, b["vol"])
    np.testing.assert_array_equal(a["centroid"] * float(s), b["centroid"])


def test_permutation_equivariance(oracle_mod):
    xyz, w, box = wl.power_uniform(600, 4)
    w = (w * 0.1).astype(np.float32)
    perm = np.random.default_rng(0).permutation(600)
    a = oracle_mod.cells(xyz, w, box)
    b = oracle_mod.cells(xyz[perm], w[perm], box)
    la, lb = _cell_lists(a), _cell_lists(b)
    for t in range(600):
        i = perm[t]
        if a["margin"][i] < 1e-6:
            continue
        assert sorted(perm[lb[t]].tolist()) == la[i].tolist()
        assert b["vol"][t] == pytest.approx(a["vol"][i], rel=1e-12)
        np.testing.assert_allclose(b["centroid"][t], a["centroid"][i], rtol=1e-12)


def test_weight_shift_invariance(oracle_mod):
    xyz, _, box = wl.uniform(500, 6)
    rng = np.random.default_rng(6)
    w = (rng.integers(0, 2 ** 18, size=500) * 2.0 ** -24).astype(np.float32)  # exact under +0.25
    a = oracle_mod.cells(xyz, w, box)
    b = oracle_mod.cells(xyz, w + np.float32(0.25), box)
    assert np.all((w + np.float32(0.25)).astype(np.float64) - 0.25 == w.astype(np.float64))
    for k in ["nbr_off", "nbr", "vert", "vert_code", "fv", "vol", "centroid"]:
        np.testing.assert_array_equal(a[k], b[k])


# ------------------------------------------------------------ lattices

@pytest.mark.parametrize("m", [4, 8])
def test_regular_lattice_gives_exact_cubes(oracle_mod, m):
    # dyadic spacing: the sites and every cell face are exact in FP32 and FP64
    g = (np.arange(m) + 0.5) / m
    xyz = np.array(list(itertools.product(g, g, g)), np.float32)
    r = oracle_mod.cells(xyz, None, UNIT)
    np.testing.assert_allclose(r["vol"], 1.0 / m ** 3, rtol=1e-14)
    np.testing.assert_allclose(r["centroid"], xyz.astype(np.float64), rtol=0, atol=1e-15)
    assert np.all(r["flags"] & oracle_mod.FLAG_DEGENERATE)  # 8 cells meet at every vertex
    assert np.all(r["margin"] == 0)


def test_jittered_lattice_gives_near_unit_cubes(oracle_mod):
    m = 6
    rng = np.random.default_rng(3)
    g = np.arange(m) + 0.5
    xyz = np.array(list(itertools.product(g, g, g))) + rng.uniform(-0.02, 0.02, size=(m ** 3, 3))
    xyz = xyz.astype(np.float32)
    box = np.array([0.0, 0.0, 0.0, m, m, m], float)
    r = oracle_mod.cells(xyz, None, box)
    assert r["vol"].sum() == pytest.approx(m ** 3, rel=1e-13)
    assert np.all(np.abs(r["vol"] - 1.0) < 0.15)
    np.testing.assert_allclose(r["centroid"], xyz.astype(np.float64), atol=0.05)
    lists = _cell_lists(r)
    idx = {tuple(np.floor(x).astype(int)): i for i, x in enumerate(xyz)}
    for key, i in idx.items():
        for ax in range(3):
            for d in (-1, 1):
                nb = list(key)
                nb[ax] += d
                if tuple(nb) in idx:  # face-adjacent lattice cells always share a facet
                    assert idx[tuple(nb)] in lists[i]
