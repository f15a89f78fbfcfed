"""Exact-rational power cells by vertex enumeration -- TEST INFRASTRUCTURE ONLY.

An algorithm independent of the C++ clipper, used to pin it on tiny inputs.
The cell C_i of the power diagram (paper Sec. 3, Eq. 1) clipped to the box B
is the set of y (frame centred on p_i) with a_k . y <= b_k for the six box
half-spaces and for a_j = p_j - p_i, b_j = (|a_j|^2 + w_i - w_j) / 2 for
every j != i.  Its vertices are exactly the points where three of these
planes meet and all constraints hold; every such point is found by solving
all plane triples in exact rational arithmetic (``fractions.Fraction`` built
from the FP32 inputs, so no rounding anywhere).  O(P^4) per cell: tiny n only.

Returns, per cell, the set of vertices keyed by their ascending code triple,
the neighbour set (site planes carrying >= 3 distinct vertices), the exact
volume (tetrahedral fan over facets ordered by angle) and a flag telling
whether any point lies on more than three planes (not in general position).
"""
from __future__ import annotations

import itertools
import math
from fractions import Fraction as Q


def _weight(w, j):
    """Weight j as an exact rational: FP32 inputs, or Fractions as given (a
    test may pass exactly perturbed weights)."""
    if w is None:
        return Q(0)
    return w[j] if isinstance(w[j], Q) else Q(float(w[j]))


def _losers(xyz, w):
    """Sites sharing a position with a heavier site (or an equally heavy one
    of lower index): their cells are empty and their planes are implied by the
    winner's, so they constrain nobody."""
    out = set()
    groups = {}
    for j in range(len(xyz)):
        groups.setdefault(tuple(float(c) for c in xyz[j]), []).append(j)
    for g in groups.values():
        if len(g) > 1:
            win = max(g, key=lambda j: (_weight(w, j), -j))
            out.update(j for j in g if j != win)
    return out


def _planes(xyz, w, box, i):
    import numpy as np
    box = [float(np.float32(v)) for v in box]  # the clip box is an FP32 input
    p = [Q(float(c)) for c in xyz[i]]
    wi = _weight(w, i)
    pl = []
    for ax in range(3):
        lo = [Q(0)] * 3
        lo[ax] = Q(-1)
        pl.append((lo, p[ax] - Q(float(box[ax])), -(2 * ax + 1)))
        hi = [Q(0)] * 3
        hi[ax] = Q(1)
        pl.append((hi, Q(float(box[3 + ax])) - p[ax], -(2 * ax + 2)))
    losers = _losers(xyz, w)
    for j in range(len(xyz)):
        if j == i or j in losers:
            continue
        a = [Q(float(xyz[j][k])) - p[k] for k in range(3)]
        d2 = sum(c * c for c in a)
        if d2 == 0:
            continue
        wj = _weight(w, j)
        pl.append((a, (d2 + wi - wj) / 2, j))
    coincident_empty = i in losers
    return p, pl, coincident_empty


def _solve(A, B, C):
    (a, ba, _), (b, bb, _), (c, bc, _) = A, B, C

    def cross(u, v):
        return [u[1] * v[2] - u[2] * v[1], u[2] * v[0] - u[0] * v[2], u[0] * v[1] - u[1] * v[0]]

    bxc, cxa, axb = cross(b, c), cross(c, a), cross(a, b)
    det = sum(a[k] * bxc[k] for k in range(3))
    if det == 0:
        return None
    return tuple((ba * bxc[k] + bb * cxa[k] + bc * axb[k]) / det for k in range(3))


def cell(xyz, w, box, i):
    p, pl, emptied = _planes(xyz, w, box, i)
    res = dict(vertices={}, nbr=set(), vol=Q(0), degenerate=False, empty=True)
    if emptied:
        return res
    pts = {}
    for A, B, C in itertools.combinations(range(len(pl)), 3):
        y = _solve(pl[A], pl[B], pl[C])
        if y is None:
            continue
        ok = True
        for a, b, _ in pl:
            if sum(a[k] * y[k] for k in range(3)) > b:
                ok = False
                break
        if ok:
            pts.setdefault(y, set()).update((A, B, C))
    if not pts:
        return res
    res["empty"] = False
    onplane = {}
    for y, s in pts.items():
        if len(s) != 3:
            res["degenerate"] = True
        for q in s:
            onplane.setdefault(q, []).append(y)
        key = tuple(sorted(pl[q][2] for q in s))
        res["vertices"][key] = tuple(p[k] + y[k] for k in range(3))
    # exact volume: fan of tetrahedra from one vertex over every facet polygon
    ref = next(iter(pts))
    vol6 = Q(0)
    for q, ys in onplane.items():
        if len(ys) < 3:
            res["degenerate"] = True
            continue
        if pl[q][2] >= 0:
            res["nbr"].add(pl[q][2])
        a = pl[q][0]
        na = math.sqrt(float(sum(c * c for c in a)))
        nrm = [float(c) / na for c in a]
        cen = [sum(float(y[k]) for y in ys) / len(ys) for k in range(3)]
        m = min(range(3), key=lambda r: abs(nrm[r]))
        ax = [0.0, 0.0, 0.0]
        ax[m] = 1.0
        e1 = [nrm[1] * ax[2] - nrm[2] * ax[1], nrm[2] * ax[0] - nrm[0] * ax[2], nrm[0] * ax[1] - nrm[1] * ax[0]]
        e2 = [nrm[1] * e1[2] - nrm[2] * e1[1], nrm[2] * e1[0] - nrm[0] * e1[2], nrm[0] * e1[1] - nrm[1] * e1[0]]
        ring = sorted(ys, key=lambda y: math.atan2(sum((float(y[k]) - cen[k]) * e2[k] for k in range(3)),
                                                   sum((float(y[k]) - cen[k]) * e1[k] for k in range(3))))
        f0 = ring[0]
        for t in range(1, len(ring) - 1):
            u = [f0[k] - ref[k] for k in range(3)]
            v = [ring[t][k] - ref[k] for k in range(3)]
            z = [ring[t + 1][k] - ref[k] for k in range(3)]
            vol6 += (u[0] * (v[1] * z[2] - v[2] * z[1]) - u[1] * (v[0] * z[2] - v[2] * z[0])
                     + u[2] * (v[0] * z[1] - v[1] * z[0]))
    res["vol"] = vol6 / 6
    return res
