"""Power cells of symbolically perturbed weights, in exact rational
arithmetic -- TEST INFRASTRUCTURE ONLY (imported by tests/ only).

Reading of exact degeneracies.  The paper defines the cell of a site (Sec. 3,
Eq. 1) and its neighbours for sites in general position; it gives no rule
for five or more sites on one power sphere, or a plane through a vertex.
Here the weights are perturbed symbolically: w_k -> w_k + delta^(k+1) for an
infinitesimal delta > 0 and original index k (Simulation of Simplicity,
Edelsbrunner and Muecke 1990).  Every cell is then the exact cell of the
perturbed sites, which are in general position: every vertex joins exactly
three planes and no vertex lies on a fourth, neighbour relations are
symmetric, and the dual is a proper regular triangulation.  The geometry
reported is the limit delta -> 0, so facets of zero area and coincident
vertices appear where the unperturbed diagram is degenerate.

Sign rule.  In the frame of p_i a vertex y where planes A, B, C meet (normals
a_A, a_B, a_C, offsets b_A, b_B, b_C) solves M y = b, and with
bc = a_B x a_C, ca = a_C x a_A, ab = a_A x a_B, det = a_A . bc it is
y = (b_A bc + b_B ca + b_C ab) / det.  Against the plane H of site m,
    S = det (a_H . y - b_H) = b_A a_H.bc + b_B a_H.ca + b_C a_H.ab - b_H det,
and y is outside H iff S det > 0.  S is linear in the offsets, and a site
plane's offset b_X = (|a_X|^2 + w_i - w_x) / 2 is linear in the weights, so
under the perturbation S(delta) = S + sum_k (dS/dw_k) delta^(k+1) exactly:
    dS/dw_x = -(a_H . cross_X) / 2   for X in {A, B, C} the plane of site x
                                      (cross_A = bc, cross_B = ca, cross_C = ab)
    dS/dw_m = det / 2
    dS/dw_i = (sum over site planes X of a_H . cross_X - det) / 2
(box planes do not depend on weights).  If S = 0 its sign is that of the
derivative of smallest index k among the non-zero ones; dS/dw_m is never
zero, so every test is decided.

The cell is clipped plane by plane in exact rationals (Fractions built from
the FP32 inputs); a candidate whose plane distance exceeds the largest
vertex distance of the current cell cannot cut it and is skipped.  The
clipping itself is the plain half-space intersection: with every sign decided
the polytope stays simple, so an edge is the pair of planes two vertices
share, and a removed vertex next to a kept one across edge {P, Q} yields the
vertex (H, P, Q).  Tiny inputs only.
"""
from __future__ import annotations

from fractions import Fraction as Q

import numpy as np


def _cross(u, v):
    return (u[1] * v[2] - u[2] * v[1], u[2] * v[0] - u[0] * v[2], u[0] * v[1] - u[1] * v[0])


def _dot(u, v):
    return u[0] * v[0] + u[1] * v[1] + u[2] * v[2]


def _sign(x) -> int:
    return (x > 0) - (x < 0)


class _Plane:
    __slots__ = ("a", "b", "code", "site")

    def __init__(self, a, b, code, site):
        self.a, self.b, self.code, self.site = a, b, code, site


def _losers(P, W):
    """Sites sharing a position with another of larger perturbed weight (the
    larger weight, or on equal weights the lower index): empty cells, and
    their planes constrain nobody (the winner's plane is the same or
    tighter)."""
    out = set()
    groups = {}
    for j, p in enumerate(P):
        groups.setdefault(p, []).append(j)
    for g in groups.values():
        if len(g) > 1:
            win = max(g, key=lambda j: (W[j], -j))
            out.update(j for j in g if j != win)
    return out


def _side(pl, tri, h, i) -> int:
    """+1 if the vertex of planes tri lies outside plane h (perturbed), else -1."""
    A, B, C = (pl[t] for t in tri)
    H = pl[h]
    bc, ca, ab = _cross(B.a, C.a), _cross(C.a, A.a), _cross(A.a, B.a)
    det = _dot(A.a, bc)
    hb = (_dot(H.a, bc), _dot(H.a, ca), _dot(H.a, ab))
    S = A.b * hb[0] + B.b * hb[1] + C.b * hb[2] - H.b * det
    if S == 0:
        deriv = {H.site: Q(det, 2)}
        own = -det
        for X, g in zip((A, B, C), hb):
            if X.site is not None:
                deriv[X.site] = -Q(g, 2) if not isinstance(g, Q) else -g / 2
                own += g
        deriv[i] = Q(own) / 2
        for k in sorted(deriv):
            if deriv[k] != 0:
                S = deriv[k]
                break
    return 1 if _sign(S) == _sign(det) else -1


def _solve(pl, tri):
    A, B, C = (pl[t] for t in tri)
    bc, ca, ab = _cross(B.a, C.a), _cross(C.a, A.a), _cross(A.a, B.a)
    det = _dot(A.a, bc)
    return tuple((A.b * bc[k] + B.b * ca[k] + C.b * ab[k]) / det for k in range(3))


def _pairs(tri):
    a, b, c = tri
    return (frozenset((a, b)), frozenset((b, c)), frozenset((a, c)))


def _clip(pl, verts, h, i):
    """Cuts the cell (dict: frozenset of 3 plane indices -> position) by plane
    h.  Returns 'none', 'changed' or 'empty'."""
    side = {v: _side(pl, tuple(sorted(v)), h, i) for v in verts}
    out = [v for v, s in side.items() if s > 0]
    if not out:
        return "none"
    if len(out) == len(verts):
        return "empty"
    ends = {}
    for v in verts:
        for pr in _pairs(tuple(v)):
            ends.setdefault(pr, []).append(v)
    new = {}
    for v in out:
        for pr in _pairs(tuple(v)):
            e = ends[pr]
            if len(e) != 2:
                raise RuntimeError("cell %d: edge %s has %d vertices (not a simple polytope)" % (i, sorted(pr), len(e)))
            u = e[0] if e[1] == v else e[1]
            if side[u] < 0:
                key = frozenset(pr | {h})
                new[key] = _solve(pl, tuple(sorted(key)))
    for v in out:
        del verts[v]
    verts.update(new)
    return "changed"


def _exact_inputs(xyz, w, box):
    P = [tuple(Q(float(c)) for c in row) for row in np.asarray(xyz)]
    if w is None:
        W = [Q(0)] * len(P)
    else:
        W = [x if isinstance(x, Q) else Q(float(x)) for x in w]
    B = [Q(float(np.float32(v))) for v in box]
    return P, W, B


def cell(xyz, w, box, i, _inputs=None):
    """The perturbed cell of site i: dict with 'empty', 'vertices' (ascending
    code triple -> exact global position), 'nbr' (sorted site ids), 'facets'
    (code -> ring of vertex code triples, in cyclic order), 'vol' and
    'centroid' (exact, the delta -> 0 limit)."""
    P, W, B = _inputs if _inputs is not None else _exact_inputs(xyz, w, box)
    losers = _losers(P, W)
    res = dict(empty=True, vertices={}, nbr=[], facets={}, vol=Q(0), centroid=P[i])
    if i in losers:
        return res
    pi, wi = P[i], W[i]
    pl = []
    for ax in range(3):
        lo = [0, 0, 0]
        lo[ax] = -1
        pl.append(_Plane(tuple(lo), pi[ax] - B[ax], -(2 * ax + 1), None))
        hi = [0, 0, 0]
        hi[ax] = 1
        pl.append(_Plane(tuple(hi), B[3 + ax] - pi[ax], -(2 * ax + 2), None))
    verts = {}
    for c in range(8):
        tri = frozenset((c & 1, 2 + ((c >> 1) & 1), 4 + ((c >> 2) & 1)))
        verts[tri] = _solve(pl, tuple(sorted(tri)))
    cand = []
    for j, p in enumerate(P):
        if j == i or j in losers:
            continue
        a = tuple(p[k] - pi[k] for k in range(3))
        a2 = _dot(a, a)
        if a2 == 0:
            continue
        b = (a2 + wi - W[j]) / 2
        cand.append((float(b) / float(a2) ** 0.5, j, a, b, a2))
    cand.sort(key=lambda t: (t[0], t[1]))
    r2 = max(_dot(y, y) for y in verts.values())
    for _, j, a, b, a2 in cand:
        # every point y of the cell has |y|^2 <= r2: the plane a.y = b with
        # b > 0 and b^2 > r2 |a|^2 cannot reach it (strictly, so no
        # infinitesimal perturbation can either)
        if b > 0 and b * b > r2 * a2:
            continue
        pl.append(_Plane(a, b, j, j))
        r = _clip(pl, verts, len(pl) - 1, i)
        if r == "empty":
            return res
        if r == "changed":
            r2 = max(_dot(y, y) for y in verts.values())
    res["empty"] = False
    code = lambda t: pl[t].code  # noqa: E731
    key = {v: tuple(sorted(code(t) for t in v)) for v in verts}
    res["vertices"] = {key[v]: tuple(pi[k] + verts[v][k] for k in range(3)) for v in verts}
    on = {}
    for v in verts:
        for t in v:
            on.setdefault(t, []).append(v)
    vol6 = Q(0)
    mom = [Q(0), Q(0), Q(0)]
    for t, vs in on.items():
        # ring: walk the facet's vertices along its edges {t, s}
        ring = [vs[0]]
        while len(ring) < len(vs):
            cur = ring[-1]
            nxt = [u for u in vs if u not in ring and len(u & cur) == 2]
            if not nxt:
                raise RuntimeError("cell %d: facet %d is not a cycle" % (i, code(t)))
            if len(ring) == 1:
                nxt = nxt[:1]
            ring.append(nxt[0])
        # counter-clockwise seen from outside where the facet has an area
        # (Newell's normal against the plane's outward normal); a facet of
        # zero area keeps the direction of the walk
        nn = [Q(0), Q(0), Q(0)]
        for q in range(len(ring)):
            c = _cross(verts[ring[q]], verts[ring[(q + 1) % len(ring)]])
            nn = [nn[k] + c[k] for k in range(3)]
        if _dot(nn, pl[t].a) < 0:
            ring.reverse()
        res["facets"][code(t)] = [key[v] for v in ring]
        if pl[t].site is not None:
            res["nbr"].append(pl[t].site)
        # signed pyramids from the site (frame origin; a power cell need not
        # contain its site) over the facet's triangles
        y0 = verts[ring[0]]
        for q in range(1, len(ring) - 1):
            y1, y2 = verts[ring[q]], verts[ring[q + 1]]
            d6 = _dot(y0, _cross(y1, y2))
            vol6 += d6
            for k in range(3):
                mom[k] += d6 * (y0[k] + y1[k] + y2[k]) / 4
    res["nbr"].sort()
    res["vol"] = vol6 / 6
    if vol6 != 0:
        res["centroid"] = tuple(pi[k] + mom[k] / vol6 for k in range(3))
    return res


def cells(xyz, w, box, ids=None):
    """Perturbed cells of the sites ids (default all)."""
    inputs = _exact_inputs(xyz, w, box)
    ids = range(len(inputs[0])) if ids is None else ids
    return {int(i): cell(xyz, w, box, int(i), inputs) for i in ids}


def tetrahedra(res):
    """Dual tetrahedra (i, j, k, l), i < j < k < l, from the cells in res
    (dict site -> cell): one per vertex of cell i whose three planes are sites
    above i."""
    out = []
    for i, c in sorted(res.items()):
        for key in sorted(c["vertices"]):
            if key[0] > i:
                out.append((i,) + key)
    return sorted(out)
