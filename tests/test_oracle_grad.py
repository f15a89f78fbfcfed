"""Pins of the FP64 analytic gradient oracle (oracle/grad.py): FP64 central
finite differences through the oracle's cells, and the closed forms of the
two-site case (paper Sec. 3, Eq. 1)."""
import numpy as np
import pytest

from oracle import cells
from oracle import grad as og

BOX = np.array([0.0, 0.0, 0.0, 1.0, 1.0, 1.0])


def _phi(x, codes, i):
    # a smooth vertex loss with a non-trivial gradient, plus a term linear in
    # each vertex with a coefficient keyed by the vertex (cell, planes)
    key = (np.asarray(codes, np.int64) * np.array([3, 5, 7])).sum(axis=1) + 11 * i
    lin = np.stack([np.sin(key), np.cos(key), np.sin(2.0 * key)], axis=1)
    return 0.5 * np.sum((x - 0.3) ** 2, axis=1) + np.sin(3.0 * x[:, 0]) + np.sum(lin * x, axis=1)


def _dphi(x, codes, i):
    key = (np.asarray(codes, np.int64) * np.array([3, 5, 7])).sum(axis=1) + 11 * i
    g = x - 0.3
    g[:, 0] += 3.0 * np.cos(3.0 * x[:, 0])
    return g + np.stack([np.sin(key), np.cos(key), np.sin(2.0 * key)], axis=1)


def _problem(n, seed, weighted):
    rng = np.random.default_rng(seed)
    xyz = rng.random((n, 3))
    w = None
    if weighted:
        s = 0.5 * n ** (-1.0 / 3.0)
        w = (s * np.exp(0.75 * rng.normal(size=n))) ** 2
    g_vol = rng.normal(size=n)
    g_cen = rng.normal(size=(n, 3))
    return xyz, w, g_vol, g_cen


def _fd(xyz, w, g_vol, g_cen, phi, h=1e-6):
    n = len(xyz)
    gp = np.zeros((n, 3))
    gw = np.zeros(n)
    for k in range(n):
        for c in range(3):
            xp, xm = xyz.copy(), xyz.copy()
            xp[k, c] += h
            xm[k, c] -= h
            gp[k, c] = (og.loss_value(xp, w, BOX, g_vol, g_cen, phi) - og.loss_value(xm, w, BOX, g_vol, g_cen, phi)) / (2 * h)
        if w is not None:
            wp, wm = w.copy(), w.copy()
            wp[k] += h
            wm[k] -= h
            gw[k] = (og.loss_value(xyz, wp, BOX, g_vol, g_cen, phi) - og.loss_value(xyz, wm, BOX, g_vol, g_cen, phi)) / (2 * h)
    return gp, gw


@pytest.mark.parametrize("weighted", [False, True])
@pytest.mark.parametrize("with_vertices", [False, True])
def test_gradient_matches_finite_differences(weighted, with_vertices):
    xyz, w, g_vol, g_cen = _problem(24, 7 if weighted else 3, weighted)
    phi = _phi if with_vertices else None
    dphi = _dphi if with_vertices else None
    gp, gw, res = og.backward(xyz, w, BOX, g_vol, g_cen, dphi, fp64=True)
    assert not np.any(res["flags"] & 2), "test input must be in general position"
    fp, fw = _fd(xyz, w, g_vol, g_cen, phi)
    scale = np.abs(fp).max()
    assert np.abs(gp - fp).max() <= 1e-6 * scale
    if weighted:
        assert np.abs(gw - fw).max() <= 1e-6 * max(np.abs(fw).max(), 1.0)


def test_gradient_of_empty_power_cells():
    # a light site next to a heavy one has an empty cell: V = 0, c = p
    xyz = np.array([[0.3, 0.5, 0.5], [0.32, 0.5, 0.5], [0.8, 0.4, 0.6], [0.6, 0.8, 0.3]])
    w = np.array([0.05, 0.0, 0.0, 0.01])
    r = cells(xyz, w, BOX, fp64=True)
    assert r["flags"][1] & 1
    g_vol = np.array([0.3, -1.0, 0.7, 0.2])
    g_cen = np.arange(12, dtype=float).reshape(4, 3) / 10.0
    gp, gw, _ = og.backward(xyz, w, BOX, g_vol, g_cen, fp64=True)
    fp, fw = _fd(xyz, w, g_vol, g_cen, None)
    assert np.abs(gp - fp).max() <= 1e-6 * np.abs(fp).max()
    assert np.abs(gw - fw).max() <= 1e-6 * np.abs(fw).max()
    np.testing.assert_allclose(gp[1], g_cen[1], rtol=0, atol=1e-12)


def test_two_sites_closed_form():
    # sites (1/4, 1/2, 1/2) and (3/4, 1/2, 1/2): the separating plane is
    # x = 1/2 + (w0 - w1) (D = 1/2), so V0 = 1/2 + w0 - w1 and the facet has
    # area A = 1 with centroid (X, 1/2, 1/2)
    xyz = np.array([[0.25, 0.5, 0.5], [0.75, 0.5, 0.5]])
    w = np.array([0.05, 0.0])
    X = 0.5 + 0.05
    gp, gw, _ = og.backward(xyz, w, BOX, np.array([1.0, 0.0]), None, fp64=True)
    # dV0/dw1 = -A / (2 D) = -1, dV0/dw0 = +1
    assert gw == pytest.approx([1.0, -1.0], abs=1e-12)
    # dV0/dp1 = -(A / D)(X_f - p1); dV0/dp0 = (A / D)(X_f - p0)
    Xf = np.array([X, 0.5, 0.5])
    np.testing.assert_allclose(gp[1], -(1.0 / 0.5) * (Xf - xyz[1]), atol=1e-12)
    np.testing.assert_allclose(gp[0], (1.0 / 0.5) * (Xf - xyz[0]), atol=1e-12)
    # V0 = X = (x0 + x1)/2 + (w0 - w1) / (2 (x1 - x0)), so
    # dV0/dx0 = 1/2 + (w0 - w1) / (2 D^2) and dV0/dx1 = 1/2 - (w0 - w1) / (2 D^2)
    assert gp[0][0] == pytest.approx(0.5 + 0.05 / (2 * 0.25), abs=1e-12)
    assert gp[1][0] == pytest.approx(0.5 - 0.05 / (2 * 0.25), abs=1e-12)


def test_volume_weight_closed_form_on_random_power_diagram():
    # dV_i/dw_j = -A_ij / (2 D_ij) for every neighbour j, and
    # dV_i/dw_i = sum_j A_ij / (2 D_ij) (box facets do not depend on weights)
    xyz, w, _, _ = _problem(40, 11, True)
    r = cells(xyz, w, BOX, fp64=True)
    for i in (0, 5, 17):
        g_vol = np.zeros(len(xyz))
        g_vol[i] = 1.0
        gp, gw, _ = og.backward(xyz, w, BOX, g_vol, None, fp64=True)
        cv = __import__("oracle").cell_view(r, i)
        expect = np.zeros(len(xyz))
        for code, idx in cv["facets"]:
            if code < 0:
                continue
            poly = cv["vert"][idx]
            # polygon area by the shoelace formula in 3D (independent of the fan code)
            area = 0.5 * np.linalg.norm(sum(np.cross(poly[k], poly[(k + 1) % len(poly)]) for k in range(len(poly))))
            D = np.linalg.norm(xyz[code] - xyz[i])
            expect[code] -= area / (2 * D)
            expect[i] += area / (2 * D)
        np.testing.assert_allclose(gw, expect, atol=1e-12)


@pytest.mark.parametrize("weighted", [False, True])
def test_gradient_with_box_of_the_sites(weighted):
    """No clip box given: the box is the sites' bounding box, so moving an
    extreme site moves a box face too.  Finite differences recompute that box
    from the perturbed sites."""
    xyz, w, g_vol, g_cen = _problem(20, 13 if weighted else 5, weighted)
    gp, gw, res = og.backward(xyz, w, None, g_vol, g_cen, fp64=True)
    assert not np.any(res["flags"] & 2), "test input must be in general position"
    h = 1e-6
    fp = np.zeros_like(gp)
    for k in range(len(xyz)):
        for c in range(3):
            xp, xm = xyz.copy(), xyz.copy()
            xp[k, c] += h
            xm[k, c] -= h
            fp[k, c] = (og.loss_value(xp, w, None, g_vol, g_cen) - og.loss_value(xm, w, None, g_vol, g_cen)) / (2 * h)
    assert np.abs(gp - fp).max() <= 1e-6 * np.abs(fp).max()
    # the box term matters here: with the box held fixed the extreme sites differ
    gfix, _, _ = og.backward(xyz, w, np.concatenate([xyz.min(0), xyz.max(0)]), g_vol, g_cen, fp64=True)
    ext = np.unique(np.concatenate([xyz.argmin(0), xyz.argmax(0)]))
    assert np.abs(gfix[ext] - fp[ext]).max() > 1e-3 * np.abs(fp).max()
