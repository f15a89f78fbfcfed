"""Pins of the oracle's robustness margin (the certificate that decides which
cells the bit-exact parity gate covers).

What the margin promises: a cell with margin >= tau keeps its combinatorics
(emptiness, neighbours, vertex plane-triples, facet rings) when every plane of
its definition (Sec. 3, Eq. 1 in the frame of the site: a = p_j - p_i,
b = (|a|^2 + w_i - w_j) / 2, and the six box faces) is perturbed by a relative
amount well below tau.  This is the perturbation that FP32 rounding of the
local-frame planes makes, so it is what "in general position at the
precision compared" means.  The tests check that promise directly, and check
on constructed near-degenerate inputs that the margin shrinks with the
distance to the degeneracy, with the conditioning of the vertex and, for
empty power cells, with the weight still missing to make the cell non-empty.

Constructions (all Voronoi unless stated, box [0,1]^3, FP64 inputs):
  * co-spherical: sites i, j, k, l with circumcentre v (a vertex of all four
    cells), and a fifth site on the same sphere, placed in the normal cone of
    cell i at v (so its plane only touches the cell, at v), then moved
    radially out by a relative delta: the cell keeps the same combinatorics
    and v lies about delta * R from the fifth site's plane;
  * box face: the same four sites rotated so that an axis lies in that normal
    cone, and the box face of that axis placed delta * R outside v;
  * sliver: i, j, k on a circle of radius rho and l lifted off its plane by
    theta * rho, so v moves by about rho / theta times any perturbation of
    the planes; a fifth site as in the co-spherical case;
  * hidden power site: two sites, the second so heavy that the first cell is
    empty until w_i rises by exactly dw.
"""
import numpy as np
import pytest

import oracle

BOX = np.array([0.0, 0.0, 0.0, 1.0, 1.0, 1.0])


# ------------------------------------------------------------------ helpers

def canon(res, t):
    """Combinatorics of cell t of an oracle result, in canonical form."""
    v = oracle.cell_view(res, t)
    keys = [tuple(k) for k in v["vert_code"].tolist()]
    fac = []
    for code, ring in v["facets"]:
        rr = [keys[q] for q in ring]
        s = min(range(len(rr)), key=lambda q: rr[q])
        fac.append((code, tuple(rr[s:] + rr[:s])))
    return bool(v["flags"] & oracle.FLAG_EMPTY), tuple(v["nbr"].tolist()), tuple(sorted(keys)), tuple(sorted(fac))


def perturb_for_cell(xyz, w, box, i, eps, rng):
    """Inputs whose planes in the frame of site i differ from the original
    ones by a relative amount of at most about eps: every other site moves by
    up to eps times its distance from p_i, every weight by up to
    eps (|a|^2 + |w_j - w_i|), every box face by up to eps times its distance
    from p_i.  Site i itself stays (a common translation changes nothing)."""
    x = np.asarray(xyz, np.float64)
    p = x[i].copy()
    a = x - p
    d = np.linalg.norm(a, axis=1)
    u = rng.normal(size=a.shape)
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    x2 = x + u * (eps * d * rng.uniform(0.0, 1.0, len(d)))[:, None]
    x2[i] = p
    w2 = None
    if w is not None:
        wd = np.asarray(w, np.float64)
        w2 = wd + eps * (d ** 2 + np.abs(wd - wd[i])) * rng.uniform(-1.0, 1.0, len(d))
        w2[i] = wd[i]
    b = np.asarray(box, np.float64)
    b2 = b + eps * np.abs(b - np.concatenate([p, p])) * rng.uniform(-1.0, 1.0, 6)
    return x2, w2, b2


def lattice(m, jitter, seed):
    """m^3 sites at the centres of a regular grid of [0,1]^3, each moved by up
    to `jitter` grid spacings per axis (near co-spherical groups of eight)."""
    rng = np.random.default_rng(seed)
    g = (np.stack(np.meshgrid(*[np.arange(m)] * 3, indexing="ij"), -1).reshape(-1, 3) + 0.5) / m
    return (g + rng.uniform(-1.0, 1.0, g.shape) * jitter / m).astype(np.float32)


def sliver(theta, delta, rho=0.2):
    """Four sites with circumcentre v (flatness theta) and a fifth site on
    their circumsphere in the normal cone of cell 0 at v, moved radially
    outward by the relative amount delta.  Returns (sites [5,3], v)."""
    c = np.array([0.5, 0.5, 0.5])
    ang = np.radians([0.0, 100.0, 220.0, 300.0])
    P = np.stack([c + rho * np.array([np.cos(t), np.sin(t), 0.0]) for t in ang])
    P[3, 2] += theta * rho
    # circumcentre: on the axis of the circle, equidistant from the lifted site
    v = c + np.array([0.0, 0.0, theta * rho / 2.0])
    assert np.allclose(np.linalg.norm(P - v, axis=1), np.linalg.norm(P[0] - v))
    # a direction inside the cone spanned by the normals of cell 0's planes at
    # v; the ray from p_0 along it meets the sphere again at q
    d = (P[1:4] - P[0]).sum(0)
    q = P[0] + 2.0 * np.dot(v - P[0], d) / np.dot(d, d) * d
    q = v + (q - v) * (1.0 + delta)
    return np.vstack([P, q[None]]), v


def rotation(u, t):
    """Rotation matrix taking direction u to direction t (Rodrigues)."""
    u = u / np.linalg.norm(u)
    t = t / np.linalg.norm(t)
    k = np.cross(u, t)
    s, c = np.linalg.norm(k), np.dot(u, t)
    K = np.array([[0.0, -k[2], k[1]], [k[2], 0.0, -k[0]], [-k[1], k[0], 0.0]])
    return np.eye(3) + K + K @ K * ((1.0 - c) / s ** 2)


def box_face_case(delta):
    """Four sites rotated so that +y lies in the normal cone of cell 0 at
    their circumcentre v; the y_max face of the box at delta * R above v."""
    P, v = sliver(1.0, 1.0)
    P = P[:4]
    c = np.array([0.5, 0.5, 0.5])
    Rm = rotation((P[1:4] - P[0]).sum(0), np.array([0.0, 1.0, 0.0]))
    P = (P - c) @ Rm.T + c
    v = (v - c) @ Rm.T + c
    box = BOX.copy()
    box[4] = v[1] + delta * np.linalg.norm(v - P[0])
    return P, box


def margin0(xyz, w=None, box=BOX):
    r = oracle.cells(xyz, w, box, fp64=True)
    return float(r["margin"][0]), r


# ------------------------------------------------------------------ the promise

def _stability_inputs():
    rng = np.random.default_rng(3)
    x = rng.uniform(0.0, 1.0, (300, 3)).astype(np.float32)
    w = ((rng.lognormal(0.0, 0.75, 300) * 0.05) ** 2).astype(np.float32)
    sl, _ = sliver(1e-3, 1e-4)
    fb, fbox = box_face_case(3e-6)
    return {
        "lattice_j1e-2": (lattice(6, 1e-2, 1), None, BOX),
        "lattice_j1e-3": (lattice(6, 1e-3, 1), None, BOX),
        "lattice_j1e-5": (lattice(6, 1e-5, 1), None, BOX),
        "uniform": (x, None, BOX),
        "power_lognormal": (x, w, BOX),
        "sliver": (sl, None, BOX),
        "box_face": (fb, None, fbox),
    }


STABILITY = _stability_inputs()


@pytest.mark.parametrize("name", sorted(STABILITY))
@pytest.mark.parametrize("tau", [1e-3, 1e-5, 1e-7])
def test_certified_cells_survive_perturbation(name, tau):
    """Every cell certified at tau keeps its combinatorics under three random
    relative perturbations of size tau / 10 of the planes that define it."""
    xyz, w, box = STABILITY[name]
    res = oracle.cells(xyz, w, box)
    cert = np.nonzero(res["margin"] >= tau)[0]
    rng = np.random.default_rng(17)
    pick = rng.choice(cert, min(30, len(cert)), replace=False) if len(cert) else []
    changed = []
    for i in pick:
        ref = canon(res, i)
        for _ in range(3):
            x2, w2, b2 = perturb_for_cell(xyz, w, box, int(i), tau / 10.0, rng)
            r2 = oracle.cells(x2, w2, b2, ids=[int(i)], fp64=True)
            if canon(r2, 0) != ref:
                changed.append(int(i))
                break
    assert not changed, "cells certified at %g changed under a %g perturbation: %s" % (tau, tau / 10, changed)


def test_perturbation_reaches_uncertified_cells():
    """The perturbation is strong enough to matter: on the near-degenerate
    lattice (jitter 1e-5 grid spacings) perturbations of 1e-4 change most
    cells, none of which the margin certifies at 1e-3."""
    xyz = lattice(6, 1e-5, 1)
    res = oracle.cells(xyz, None, BOX)
    assert (res["margin"] >= 1e-3).sum() == 0
    rng = np.random.default_rng(5)
    ids = rng.choice(len(xyz), 20, replace=False)
    moved = 0
    for i in ids:
        x2, w2, b2 = perturb_for_cell(xyz, None, BOX, int(i), 1e-4, rng)
        moved += canon(oracle.cells(x2, w2, b2, ids=[int(i)], fp64=True), 0) != canon(res, int(i))
    assert moved >= 10


# ------------------------------------------------------------------ constructions

@pytest.mark.parametrize("case", ["cospherical", "box_face"])
def test_margin_proportional_to_offset(case):
    """A vertex that lies delta * R from a plane it is not on (a fifth
    co-spherical site moved out by delta, or a box face delta * R away) gives
    a margin proportional to delta over four decades, and of the order of
    delta (between delta / 100 and delta), with unchanged combinatorics."""
    ms, combos = [], set()
    for delta in (1e-3, 1e-4, 1e-5, 1e-6, 1e-7):
        if case == "cospherical":
            P, _ = sliver(1.0, delta)
            m, r = margin0(P)
        else:
            P, box = box_face_case(delta)
            m, r = margin0(P, None, box)
        ms.append(m / delta)
        combos.add(canon(r, 0))
    ms = np.array(ms)
    assert len(combos) == 1
    assert ms.max() / ms.min() < 1.05, ms
    assert 1e-2 <= ms.min() and ms.max() <= 1.0, ms


def test_box_face_is_the_limiting_plane():
    """In the box-face construction the limiting plane is the box face: the
    cell has no facet on it, and moving the face away raises the margin."""
    P, box = box_face_case(1e-6)
    m, r = margin0(P, None, box)
    assert all(code != -4 for code, _ in oracle.cell_view(r, 0)["facets"])
    box2 = box.copy()
    box2[4] += 0.5
    m2, _ = margin0(P, None, box2)
    assert m2 > 1e3 * m


def test_margin_reflects_vertex_conditioning():
    """The sliver's vertex moves by about rho / theta times a relative
    perturbation of its planes, so a valid certificate must shrink with theta
    at a fixed plane offset: from theta = 0.1 to 0.001 it falls by at least
    20x (the plane offset itself barely changes)."""
    m = {th: margin0(sliver(th, 3e-5)[0])[0] for th in (1e-1, 1e-2, 1e-3)}
    assert m[1e-2] < 0.3 * m[1e-1]
    assert m[1e-3] < 0.05 * m[1e-1]


@pytest.mark.parametrize("dw_rel,level", [(3e-2, 1e-3), (3e-4, 1e-5), (3e-6, 1e-7), (3e-9, 1e-10), (3e-13, 0.0)])
def test_empty_cell_certificate_level(dw_rel, level):
    """Site 0 at the box centre, site 1 a distance l = 0.1 along x with weight
    w_1 = 0.11 + dw: cell 0 is empty exactly while w_0 < dw (its plane then
    lies beyond the box face x = 0).  The certificate raises w_0 by
    tau (l^2 + |w_0|) = 0.01 tau at tau = 1e-3, 1e-5, 1e-7, 1e-10 and reports
    the largest tau at which the cell stays empty."""
    dw = 0.01 * dw_rel
    xyz = np.array([[0.5, 0.5, 0.5], [0.6, 0.5, 0.5]])
    w = np.array([0.0, 0.11 + dw])
    m, r = margin0(xyz, w)
    assert r["flags"][0] & oracle.FLAG_EMPTY
    assert m == level
    # and the cell really is non-empty once w_0 exceeds dw
    w2 = w.copy()
    w2[0] = 2.0 * dw
    _, r2 = margin0(xyz, w2)
    assert not r2["flags"][0] & oracle.FLAG_EMPTY
