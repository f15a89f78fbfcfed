"""FP64 analytic gradients of cell volumes, centroids and vertices -- TEST
INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Derivatives are taken with the combinatorics of the diagram held fixed (the
cells' facet/vertex structure does not change under an infinitesimal move).
They follow from the cell definition (paper Sec. 3, Eq. 1), written in the
frame of the site p_i: C_i = {y : a_f . y <= b_f for every facet plane f},
with a_f = p_j - p_i and b_f = (|a_f|^2 + w_i - w_j) / 2 for the plane of
site j, and a_f = +-e_k, b_f = +-(B_k - p_i,k) for a face of the clip box.

Moving plane f by (da_f, db_f) moves a boundary point y of facet F_f along
the outward normal by (db_f - da_f . y) / |a_f|.  Integrating that speed over
the boundary (transport of the volume and first-moment integrals):

    dV = sum_f  (A_f db_f - A_f Y_f . da_f) / |a_f|
    dm = sum_f  (A_f Y_f db_f - S_f da_f) / |a_f|,      m = int_C y dV

with A_f the facet area, Y_f its centroid and S_f = int_F y y^T dA (frame of
p_i).  The centroid is c = p_i + m / V.  A vertex is x = p_i + M^-1 b with
the rows of M the normals a of its three planes, so for a gradient g on x,
d/db = M^-T g and d/da_k = -(M^-T g)_k y.  Finally the plane parameters
depend on the sites: da_f = dp_j - dp_i, db_f = a_f . da_f + (dw_i - dw_j)/2
for a site plane and db_f = -a_f . dp_i for a box face.

For an empty cell V = 0 and c = p_i.

When no clip box is given, the box is the bounding box of the sites, so its
faces move with the extreme sites: b_f = p_i,k - min_j p_j,k for a lower face
and max_j p_j,k - p_i,k for an upper one.  The sum over all cells of dL/db_f
for each face then goes, with sign -1 (lower) or +1 (upper), to the site
that attains that minimum or maximum (the lowest index among ties).

The closed forms that follow for the volume (dV_i/dw_j = -A_ij / (2 D_ij),
dV_i/dp_j = -(A_ij / D_ij)(X_ij - p_j) with X_ij the facet centroid) are
checked in the tests; the whole chain is pinned by FP64 central finite
differences through the oracle.
"""
from __future__ import annotations

import numpy as np

from . import cell_view, cells


def _plane(code, i, xyz, w, box):
    """Plane (a, b) of facet code `code` of cell i, frame of p_i, FP64."""
    p = xyz[i]
    if code >= 0:
        a = xyz[code] - p
        wi = 0.0 if w is None else w[i]
        wj = 0.0 if w is None else w[code]
        return a, 0.5 * (a @ a + (wi - wj))
    c = -code - 1
    ax, side = c >> 1, c & 1
    a = np.zeros(3)
    if side:
        a[ax] = 1.0
        return a, box[3 + ax] - p[ax]
    a[ax] = -1.0
    return a, p[ax] - box[ax]


def _facet_integrals(poly, a):
    """Area, area * centroid and second moment int y y^T dA of a planar polygon
    (vertices counter-clockwise seen along +a), by a triangle fan."""
    n = a / np.linalg.norm(a)
    A = 0.0
    AY = np.zeros(3)
    S = np.zeros((3, 3))
    p0 = poly[0]
    for t in range(1, len(poly) - 1):
        p1, p2 = poly[t], poly[t + 1]
        at = 0.5 * (np.cross(p1 - p0, p2 - p0) @ n)
        s = p0 + p1 + p2
        A += at
        AY += at * s / 3.0
        S += at / 12.0 * (np.outer(p0, p0) + np.outer(p1, p1) + np.outer(p2, p2) + np.outer(s, s))
    return A, AY, S


def cell_partials(xyz, w, box, res, t, g_vol=0.0, g_cen=None, g_vert_fn=None, box_db=None):
    """Contributions of cell t of an oracle result to dL/dp and dL/dw, for
    L = g_vol V_i + g_cen . c_i + sum_v phi(x_v) with grad phi = g_vert_fn.
    g_vert_fn(x [k,3], codes [k,3], i) gives the gradient on the cell's
    vertices (positions, ascending plane codes, site).
    Returns {site: (dL/dp (3,), dL/dw)}, the box faces held fixed; with
    ``box_db`` (an array of 6) dL/db_f of the cell's box faces is added to
    box_db[-code - 1]."""
    i = int(res["ids"][t])
    cv = cell_view(res, t)
    gc = np.zeros(3) if g_cen is None else np.asarray(g_cen, float)
    out = {}

    def add(site, gp, gw):
        if site not in out:
            out[site] = [np.zeros(3), 0.0]
        out[site][0] = out[site][0] + gp
        out[site][1] = out[site][1] + gw

    add(i, gc, 0.0)  # c = p_i + m / V, and c = p_i for an empty cell
    if len(cv["vert"]) == 0:
        return {k: (v[0], v[1]) for k, v in out.items()}
    p = xyz[i]
    y = cv["vert"] - p
    planes = {}
    integ = {}
    for code, idx in cv["facets"]:
        a, b = _plane(code, i, xyz, w, box)
        planes[code] = (a, b)
        integ[code] = _facet_integrals(y[idx], a)
    # V and m from the facets: pyramids with apex at the site
    V = sum(planes[c][1] * integ[c][0] / (3.0 * np.linalg.norm(planes[c][0])) for c in planes)
    m = sum(planes[c][1] * integ[c][1] / (4.0 * np.linalg.norm(planes[c][0])) for c in planes)
    dA = {c: np.zeros(3) for c in planes}   # dL/da_f
    dB = {c: 0.0 for c in planes}           # dL/db_f
    if V != 0.0:
        # L = g_vol V + gc . (p_i + m / V)
        alpha = g_vol - gc @ m / (V * V)
        gamma = gc / V
        for c, (a, b) in planes.items():
            D = np.linalg.norm(a)
            A, AY, S = integ[c]
            dB[c] += (alpha * A + gamma @ AY) / D
            dA[c] += -(alpha * AY + S @ gamma) / D
    if g_vert_fn is not None:
        gv = np.asarray(g_vert_fn(cv["vert"], cv["vert_code"], i), float)
        for v in range(len(y)):
            codes = [int(c) for c in cv["vert_code"][v]]
            M = np.array([planes[c][0] for c in codes])
            g = np.linalg.solve(M.T, gv[v])
            for k, c in enumerate(codes):
                dB[c] += g[k]
                dA[c] += -g[k] * y[v]
            add(i, gv[v], 0.0)
    for c, (a, b) in planes.items():
        if c >= 0:
            gp = dA[c] + dB[c] * a
            add(c, gp, -0.5 * dB[c])
            add(i, -gp, 0.5 * dB[c])
        else:
            add(i, -dB[c] * a, 0.0)
            if box_db is not None:
                box_db[-c - 1] += dB[c]
    return {k: (v[0], v[1]) for k, v in out.items()}


def backward(xyz, w, box, g_vol=None, g_cen=None, g_vert_fn=None, ids=None, fp64=False):
    """dL/dp [n,3] and dL/dw [n] for L = sum_i g_vol_i V_i + g_cen_i . c_i
    + sum over all vertices phi(x) (grad phi = g_vert_fn(x, codes, i), see
    ``cell_partials``).  ``box`` None: the box is the sites' bounding box and
    its faces carry gradient to the extreme sites (all cells are needed).

    With ``ids`` the gradients are exact only at those sites: the cells of
    the sites and of all their neighbours are computed (a site's gradient
    collects contributions from every cell that has it as a neighbour, which
    by symmetry of the diagram are its own neighbours)."""
    dt = np.float64 if fp64 else np.float32
    x64 = np.asarray(xyz, dt).astype(np.float64)
    w64 = None if w is None else np.asarray(w, dt).astype(np.float64)
    moving_box = box is None
    if moving_box:
        if ids is not None:
            raise ValueError("a box that follows the sites needs every cell (ids=None)")
        box = np.concatenate([x64.min(axis=0), x64.max(axis=0)])
    box64 = np.asarray(box, dt).astype(np.float64)
    n = len(x64)
    box_db = np.zeros(6) if moving_box else None
    if ids is None:
        need = np.arange(n)
    else:
        first = cells(xyz, w, box, ids=np.asarray(ids, np.int64), margin=False, fp64=fp64)
        need = np.unique(np.concatenate([np.asarray(ids, np.int64), first["nbr"]]))
    res = cells(xyz, w, box, ids=need, margin=False, fp64=fp64)
    gp = np.zeros((n, 3))
    gw = np.zeros(n)
    for t in range(len(need)):
        i = int(need[t])
        part = cell_partials(x64, w64, box64, res, t,
                             0.0 if g_vol is None else float(g_vol[i]),
                             None if g_cen is None else g_cen[i], g_vert_fn, box_db)
        for s, (a, b) in part.items():
            gp[s] += a
            gw[s] += b
    if moving_box:
        for c in range(6):
            ax, side = c >> 1, c & 1
            col = x64[:, ax]
            j = int(np.argmax(col)) if side else int(np.argmin(col))  # first index among ties
            gp[j, ax] += box_db[c] if side else -box_db[c]
    return gp, gw, res


def loss_value(xyz, w, box, g_vol=None, g_cen=None, phi=None, fp64=True):
    """L = sum_i g_vol_i V_i + g_cen_i . c_i + sum over all vertices
    phi(x, codes, i): the function whose gradient ``backward`` returns (for
    finite differences)."""
    res = cells(xyz, w, box, margin=False, fp64=fp64)
    L = 0.0
    if g_vol is not None:
        L += float(np.dot(g_vol, res["vol"]))
    if g_cen is not None:
        L += float(np.sum(g_cen * res["centroid"]))
    if phi is not None:
        for t in range(len(res["ids"])):
            v0, v1 = res["vert_off"][t], res["vert_off"][t + 1]
            if v1 > v0:
                L += float(np.sum(phi(res["vert"][v0:v1], res["vert_code"][v0:v1], int(res["ids"][t]))))
    return L
