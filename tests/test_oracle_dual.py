"""Pins of the oracle's dual tetrahedra (the regular triangulation of the
weighted sites, paper Sec. 3; the Delaunay tetrahedralisation for equal
weights), against Qhull and against the empty-orthosphere definition by
brute force over all four-site subsets.

A tetrahedron is listed when its power centre (the diagram vertex it is dual
to) lies strictly inside the box."""
import itertools

import numpy as np
import pytest

from paper_2605_06408_amd import workloads as wl

UNIT = np.array([0.0, 0.0, 0.0, 1.0, 1.0, 1.0])


def _inside(z, box, pad):
    return bool(np.all(z > box[:3] + pad) and np.all(z < box[3:] - pad))


def test_equal_weights_match_qhull_delaunay(oracle_mod):
    from scipy.spatial import Delaunay
    xyz, _, box = wl.uniform(600, 21)
    box = np.asarray(box, np.float64)
    got = {tuple(r) for r in oracle_mod.tetrahedra(oracle_mod.cells(xyz, None, box)).tolist()}
    p = xyz.astype(np.float64)
    want, near = set(), set()
    for s in Delaunay(p).simplices:
        a = p[s[1:]] - p[s[0]]
        rhs = 0.5 * (a * a).sum(1)
        z = p[s[0]] + np.linalg.solve(a, rhs)  # circumcentre
        key = tuple(sorted(int(x) for x in s))
        if _inside(z, box, 1e-9):
            want.add(key)
        elif _inside(z, box, -1e-9):
            near.add(key)  # centre on the box surface within rounding: either way
    assert len(want) > 1000
    assert want <= got and got - want <= near


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_regular_tets_by_empty_orthosphere(oracle_mod, seed):
    """Brute force over all 4-subsets: a subset is a regular tetrahedron with
    its power centre z in the box iff z (equal power distance |z - p|^2 - w to
    all four) has a strictly larger power distance to every other site."""
    n = 26
    rng = np.random.default_rng(100 + seed)
    xyz = rng.random((n, 3)).astype(np.float32)
    w = (rng.normal(0.0, 0.02, n)).astype(np.float32)
    p = xyz.astype(np.float64)
    wd = w.astype(np.float64)
    want = set()
    for q in itertools.combinations(range(n), 4):
        q = list(q)
        a = 2.0 * (p[q[1:]] - p[q[0]])
        rhs = (p[q[1:]] ** 2).sum(1) - wd[q[1:]] - (p[q[0]] ** 2).sum() + wd[q[0]]
        if abs(np.linalg.det(a)) < 1e-12:
            continue
        z = np.linalg.solve(a, rhs)
        if not _inside(z, UNIT, 0.0):
            continue
        pw = ((p - z) ** 2).sum(1) - wd
        ref = pw[q[0]]
        others = np.delete(pw, q)
        gap = others.min() - ref
        assert abs(gap) > 1e-9, "seed gives a near-degenerate subset"
        if gap > 0:
            want.add(tuple(q))
    got = {tuple(r) for r in oracle_mod.tetrahedra(oracle_mod.cells(xyz, w, UNIT)).tolist()}
    assert len(want) >= 3
    assert got == want


def test_each_tet_is_a_vertex_of_its_four_cells(oracle_mod):
    xyz, w, box = wl.power_uniform(1500, 8)
    r = oracle_mod.cells(xyz, w, box)
    tets = oracle_mod.tetrahedra(r)
    seen = set()
    for i in range(len(xyz)):
        for c in r["vert_code"][r["vert_off"][i]:r["vert_off"][i + 1]]:
            if c[0] >= 0:
                seen.add((i,) + tuple(int(x) for x in c))
    # every all-site vertex of a cell is one tetrahedron seen from one of its sites
    assert len(seen) == 4 * len(tets)
    for t in tets.tolist():
        assert t == sorted(t) and len(set(t)) == 4
        for k in range(4):
            assert (t[k],) + tuple(t[:k] + t[k + 1:]) in seen


def test_no_tets_without_four_sites(oracle_mod):
    xyz = np.array([[0.2, 0.3, 0.4], [0.7, 0.6, 0.5], [0.4, 0.8, 0.1]], np.float32)
    assert oracle_mod.tetrahedra(oracle_mod.cells(xyz, None, UNIT)).shape == (0, 4)


def test_weighted_match_qhull_lifted_lower_hull(oracle_mod):
    """The regular triangulation is the projection of the lower convex hull of
    the lifted points (p, |p|^2 - w) (Aurenhammer's lifting map): its facets
    whose power centre lies in the box are the oracle's tetrahedra."""
    from scipy.spatial import ConvexHull
    xyz, w, box = wl.power_uniform(1500, 9)
    w = (w * 0.3).astype(np.float32)
    box = np.asarray(box, np.float64)
    got = {tuple(r) for r in oracle_mod.tetrahedra(oracle_mod.cells(xyz, w, box)).tolist()}
    p = xyz.astype(np.float64)
    wd = w.astype(np.float64)
    hull = ConvexHull(np.hstack([p, (p * p).sum(1, keepdims=True) - wd[:, None]]))
    want, near = set(), set()
    for s, eq in zip(hull.simplices, hull.equations):
        if eq[3] >= 0:
            continue  # upper hull
        a = 2.0 * (p[s[1:]] - p[s[0]])
        rhs = (p[s[1:]] ** 2).sum(1) - wd[s[1:]] - (p[s[0]] ** 2).sum() + wd[s[0]]
        z = np.linalg.solve(a, rhs)  # power centre
        key = tuple(sorted(int(x) for x in s))
        if _inside(z, box, 1e-9):
            want.add(key)
        elif _inside(z, box, -1e-9):
            near.add(key)
    assert len(want) > 500
    assert want <= got and got - want <= near
