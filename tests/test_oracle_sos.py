"""Pins of the symbolically perturbed exact oracle (oracle/sos.py), on the CPU.

1. On inputs in general position it is the exact cell: vertices, exact
   positions, neighbours and exact volumes equal those of the exact-rational
   vertex enumeration (oracle/brute.py), a different algorithm.
2. On exactly degenerate inputs (dyadic lattices, where eight cells meet at
   every vertex; four sites around a line through box faces; equal non-zero
   weights; sites on a common sphere) it equals an explicit perturbation: the
   vertex enumeration run on the weights w_k + delta^(k+1) with a small but
   finite delta = 2^-64 (exact rationals), which puts the input in general
   position.  For delta small enough the sign of every perturbed predicate
   is that of its lowest-order non-zero term, which is what the symbolic rule
   takes.
3. The perturbed cells form a partition: volumes and first moments sum to
   those of the box exactly, neighbours are symmetric, every cell is a simple
   polytope (F = V/2 + 2), a vertex of four sites appears in all four cells,
   and a shared facet has the same vertices from both sides.
4. The dual of a lattice is a triangulation: the tetrahedra cover the
   lattice's hull exactly once (absolute volumes sum to its volume, every
   triangle is shared by two tetrahedra or lies on the hull).
5. Planted mistakes in the sign rule (own-site term dropped, priority
   reversed, ties kept inside) each fail one of these pins.
"""
import itertools
from fractions import Fraction as Q

import numpy as np
import pytest

from oracle import brute, sos

UNIT = np.array([0.0, 0.0, 0.0, 1.0, 1.0, 1.0])


def lattice(m, h=0.25, off=0.125):
    g = off + h * np.arange(m)
    return np.array([[a, b, c] for a in g for b in g for c in g], np.float32)


def _degenerate_cases():
    # site order shuffled, so that no symmetry of the configuration maps the
    # perturbation's priority order onto another one
    L3 = lattice(3)[np.random.default_rng(3).permutation(27)]
    box3 = np.array([0.0, 0.0, 0.0, 0.75, 0.75, 0.75])
    # four sites around the vertical line x = y = 1/2: eight planes meet the
    # box faces z = 0 and z = 1 at one point
    four = np.array([[0.25, 0.25, 0.5], [0.75, 0.25, 0.5], [0.25, 0.75, 0.5], [0.75, 0.75, 0.5],
                     [0.5, 0.5, 0.125]], np.float32)
    # eight cube corners and the centre: the centre's cell vertices are met
    # by four sites each
    cube = np.array([[0.25 + 0.5 * (c & 1), 0.25 + 0.5 * ((c >> 1) & 1), 0.25 + 0.5 * ((c >> 2) & 1)]
                     for c in range(8)] + [[0.5, 0.5, 0.5]], np.float32)[np.random.default_rng(4).permutation(9)]
    L2 = lattice(2, 0.5, 0.25)
    return {
        "lattice3": (L3, None, box3, [0, 4, 13, 22]),
        "line_through_box_faces": (four, None, UNIT, list(range(5))),
        "cube_and_centre": (cube, None, UNIT, list(range(9))),
        "lattice2_equal_weights": (L2, np.full(8, 1.0 / 64, np.float32), UNIT, list(range(8))),
    }


def _explicit(xyz, w, box, ids, delta=Q(1, 2 ** 64)):
    base = [Q(0)] * len(xyz) if w is None else [Q(float(v)) for v in w]
    wp = [base[k] + delta ** (k + 1) for k in range(len(xyz))]
    return {i: brute.cell(xyz, wp, box, i) for i in ids}


@pytest.mark.parametrize("kind", ["voronoi", "power", "outside"])
def test_general_position_equals_exact_enumeration(kind):
    rng = np.random.default_rng({"voronoi": 0, "power": 1, "outside": 2}[kind])
    n = 12
    xyz = rng.random((n, 3)).astype(np.float32)
    w = None
    box = UNIT
    if kind == "power":
        w = (0.02 * rng.lognormal(0.0, 0.75, n) ** 2).astype(np.float32)
    if kind == "outside":
        box = np.array([0.1, 0.1, 0.1, 0.9, 0.8, 0.9])
        w = (0.01 * rng.random(n)).astype(np.float32)
    res = sos.cells(xyz, w, box)
    for i in range(n):
        b = brute.cell(xyz, w, box, i)
        assert not b["degenerate"]
        s = res[i]
        assert s["empty"] == b["empty"]
        assert s["vertices"] == b["vertices"]
        assert s["nbr"] == sorted(b["nbr"])
        assert s["vol"] == b["vol"]


@pytest.mark.parametrize("name", list(_degenerate_cases()))
def test_degenerate_inputs_equal_an_explicit_perturbation(name):
    xyz, w, box, ids = _degenerate_cases()[name]
    res = sos.cells(xyz, w, box, ids)
    exp = _explicit(xyz, w, box, ids)
    for i in ids:
        b, s = exp[i], res[i]
        assert not b["degenerate"], (name, i)  # the explicit perturbation is generic
        assert b["empty"] == s["empty"]
        assert set(b["vertices"]) == set(s["vertices"]), (name, i)
        assert sorted(b["nbr"]) == s["nbr"], (name, i)
        assert abs(float(b["vol"] - s["vol"])) <= 1e-12


def _invariants(xyz, w, box):
    res = sos.cells(xyz, w, box)
    bv = [Q(float(np.float32(v))) for v in box]
    vol_box = (bv[3] - bv[0]) * (bv[4] - bv[1]) * (bv[5] - bv[2])
    assert sum(c["vol"] for c in res.values()) == vol_box
    for k in range(3):
        mom = sum(c["vol"] * c["centroid"][k] for c in res.values())
        assert mom == vol_box * (bv[k] + bv[3 + k]) / 2
    for i, c in res.items():
        if c["empty"]:
            continue
        assert len(c["facets"]) == len(c["vertices"]) // 2 + 2  # simple polytope
        for j in c["nbr"]:
            assert i in res[j]["nbr"]
            # the shared facet: the same vertices seen from both sides
            mine = {tuple(sorted((set(k) - {j}) | {i})) for k in c["facets"][j]}
            assert mine == set(res[j]["facets"][i])
        for key in c["vertices"]:
            if key[0] >= 0:  # four sites meet: the vertex is in all four cells
                quad = sorted(key + (i,))
                for s in key:
                    assert tuple(q for q in quad if q != s) in res[s]["vertices"]
    return res


@pytest.mark.parametrize("name", list(_degenerate_cases()))
def test_perturbed_cells_form_a_partition(name):
    xyz, w, box, _ = _degenerate_cases()[name]
    _invariants(xyz, w, box)


def test_dual_of_a_lattice_is_a_triangulation():
    L, _, box, _ = _degenerate_cases()["lattice3"]
    res = _invariants(L, None, box)
    tets = sos.tetrahedra(res)
    P = [tuple(Q(float(c)) for c in p) for p in L]
    total = Q(0)
    faces = {}
    for t in tets:
        a, b, c, d = (P[k] for k in t)
        u = [b[k] - a[k] for k in range(3)]
        v = [c[k] - a[k] for k in range(3)]
        z = [d[k] - a[k] for k in range(3)]
        total += abs(u[0] * (v[1] * z[2] - v[2] * z[1]) - u[1] * (v[0] * z[2] - v[2] * z[0])
                     + u[2] * (v[0] * z[1] - v[1] * z[0])) / 6
        for f in itertools.combinations(t, 3):
            faces[f] = faces.get(f, 0) + 1
    lo, hi = Q(1, 8), Q(5, 8)
    assert total == (hi - lo) ** 3
    for f, cnt in faces.items():
        assert cnt in (1, 2)
        if cnt == 1:  # a boundary triangle lies on one face of the hull
            assert any(all(P[k][ax] == side for k in f) for ax in range(3) for side in (lo, hi)), f


def _mutants():
    good = sos._side

    def no_own_term(pl, tri, h, i):
        A, B, C = (pl[t] for t in tri)
        H = pl[h]
        bc, ca, ab = sos._cross(B.a, C.a), sos._cross(C.a, A.a), sos._cross(A.a, B.a)
        det = sos._dot(A.a, bc)
        hb = (sos._dot(H.a, bc), sos._dot(H.a, ca), sos._dot(H.a, ab))
        S = A.b * hb[0] + B.b * hb[1] + C.b * hb[2] - H.b * det
        if S == 0:
            deriv = {H.site: Q(det) / 2}
            for X, g in zip((A, B, C), hb):
                if X.site is not None:
                    deriv[X.site] = -Q(g) / 2
            for k in sorted(deriv):
                if deriv[k] != 0:
                    S = deriv[k]
                    break
        return 1 if (S > 0) == (det > 0) and S != 0 else -1

    def reversed_priority(pl, tri, h, i):
        A, B, C = (pl[t] for t in tri)
        H = pl[h]
        bc, ca, ab = sos._cross(B.a, C.a), sos._cross(C.a, A.a), sos._cross(A.a, B.a)
        det = sos._dot(A.a, bc)
        hb = (sos._dot(H.a, bc), sos._dot(H.a, ca), sos._dot(H.a, ab))
        S = A.b * hb[0] + B.b * hb[1] + C.b * hb[2] - H.b * det
        if S == 0:
            deriv = {H.site: Q(det) / 2}
            own = -Q(det)
            for X, g in zip((A, B, C), hb):
                if X.site is not None:
                    deriv[X.site] = -Q(g) / 2
                    own += g
            deriv[i] = own / 2
            for k in sorted(deriv, reverse=True):
                if deriv[k] != 0:
                    S = deriv[k]
                    break
        return 1 if (S > 0) == (det > 0) and S != 0 else -1

    def ties_inside(pl, tri, h, i):
        A, B, C = (pl[t] for t in tri)
        H = pl[h]
        bc, ca, ab = sos._cross(B.a, C.a), sos._cross(C.a, A.a), sos._cross(A.a, B.a)
        det = sos._dot(A.a, bc)
        S = A.b * sos._dot(H.a, bc) + B.b * sos._dot(H.a, ca) + C.b * sos._dot(H.a, ab) - H.b * det
        return 1 if S != 0 and (S > 0) == (det > 0) else -1

    assert good is not None
    return {"no_own_term": no_own_term, "reversed_priority": reversed_priority, "ties_inside": ties_inside}


@pytest.mark.parametrize("mutant", list(_mutants()))
def test_planted_sign_rule_mistakes_are_caught(monkeypatch, mutant):
    monkeypatch.setattr(sos, "_side", _mutants()[mutant])
    caught = False
    for name, (xyz, w, box, ids) in _degenerate_cases().items():
        try:
            test_degenerate_inputs_equal_an_explicit_perturbation(name)
            _invariants(xyz, w, box)
        except (AssertionError, RuntimeError, KeyError, ValueError, ZeroDivisionError):
            caught = True
            break
    assert caught, mutant
