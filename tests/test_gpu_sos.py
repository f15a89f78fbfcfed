"""GPU builds with the symbolic perturbation (vd_options.perturb = 1) against
the exact symbolically perturbed oracle (oracle/sos.py), on exactly
degenerate inputs: dyadic lattices (eight cells at every vertex), cube
corners around a centre, four sites around a line through two box faces,
equal non-zero weights.  Every cell must match exactly: empty flag,
neighbours, vertex plane-triples, facet rings (cyclic order; orientation
where the facet has an area), and the dual tetrahedra; volumes and centroids
within 1e-5.  On inputs in general position the option changes nothing.
"""
import numpy as np
import pytest

from oracle import sos

from .parity import gpu_build, to_numpy
from .test_oracle_sos import _degenerate_cases, lattice

pytestmark = pytest.mark.gpu


def _cases():
    c = dict(_degenerate_cases())
    rng = np.random.default_rng(11)
    L4 = lattice(4, 0.125, 0.0625)[rng.permutation(64)]
    c["lattice4_shuffled"] = (L4, None, np.array([0.0, 0.0, 0.0, 0.5, 0.5, 0.5]), None)
    L5 = lattice(5, 0.125, 0.0625)
    c["lattice5"] = (L5, None, np.array([0.0, 0.0, 0.0, 0.625, 0.625, 0.625]), None)
    # a lattice inside a larger box: the outer cells reach the box faces
    c["lattice3_in_unit_box"] = (lattice(3), None, np.array([0.0, 0.0, 0.0, 1.0, 1.0, 1.0]), None)
    return c


def _ring_match(g_ring, o_ring, oriented):
    n = len(o_ring)
    if len(g_ring) != n:
        return False
    if g_ring[0] not in o_ring:
        return False
    k = o_ring.index(g_ring[0])
    fwd = [o_ring[(k + t) % n] for t in range(n)]
    if g_ring == fwd:
        return True
    bwd = [o_ring[(k - t) % n] for t in range(n)]
    return not oriented and g_ring == bwd


def _has_area(res_cell, ring):
    P = [res_cell["vertices"][k] for k in ring]
    nn = [0, 0, 0]
    for q in range(len(P)):
        a, b = P[q], P[(q + 1) % len(P)]
        nn[0] += a[1] * b[2] - a[2] * b[1]
        nn[1] += a[2] * b[0] - a[0] * b[2]
        nn[2] += a[0] * b[1] - a[1] * b[0]
    return any(x != 0 for x in nn)


@pytest.mark.parametrize("name", list(_cases()))
def test_perturbed_build_matches_the_exact_oracle(name):
    import torch
    import paper_2605_06408_amd as vd
    xyz, w, box, _ = _cases()[name]
    n = len(xyz)
    ctx = vd.Context(0)
    x = torch.from_numpy(np.ascontiguousarray(xyz)).cuda()
    ww = None if w is None else torch.from_numpy(np.ascontiguousarray(w, np.float32)).cuda()
    d = ctx.build(x, ww, bbox=[float(v) for v in box], perturb=1)
    tets = ctx.tetrahedra().cpu().numpy()
    torch.cuda.synchronize()
    g = to_numpy(d)
    res = sos.cells(xyz, w, box)
    assert d.sizes["n_uncertain"] == 0 and d.sizes["n_failed"] == 0
    assert d.sizes["n_perturbed"] > 0  # these inputs do have exact ties
    for i in range(n):
        o = res[i]
        empty = bool(g["flags"][i] & vd.FLAG_EMPTY)
        assert empty == o["empty"], (name, i)
        nb = g["nbr"][g["nbr_off"][i]:g["nbr_off"][i + 1]].tolist()
        assert nb == o["nbr"], (name, i, nb, o["nbr"])
        vs, ve = g["vert_off"][i], g["vert_off"][i + 1]
        keys = [tuple(int(c) for c in r) for r in g["vert_planes"][vs:ve]]
        assert sorted(keys) == sorted(o["vertices"]), (name, i)
        for f in range(g["facet_off"][i], g["facet_off"][i + 1]):
            code = int(g["facet_nbr"][f])
            ring = [keys[int(v) - vs] for v in g["fv"][g["fv_off"][f]:g["fv_off"][f + 1]]]
            o_ring = o["facets"][code]
            assert _ring_match(ring, o_ring, _has_area(o, o_ring)), (name, i, code)
        if not o["empty"]:
            ov = float(o["vol"])
            assert abs(float(g["vol"][i]) - ov) <= 1e-5 * ov
            ell = max(float(np.abs(np.asarray(box, float)).max()), 1e-30)
            oc = np.array([float(c) for c in o["centroid"]])
            assert np.abs(g["centroid"][i] - oc).max() <= 1e-5 * ell
            for k, y in zip(keys, g["vert"][vs:ve]):
                ox = np.array([float(c) for c in o["vertices"][k]])
                assert np.abs(y - ox).max() <= 1e-6 * ell
    assert sorted(map(tuple, tets.tolist())) == sos.tetrahedra(res)
    ctx.close()


@pytest.mark.parametrize("kind", ["uniform", "power"])
def test_perturbation_changes_nothing_in_general_position(kind):
    from paper_2605_06408_amd import workloads as wl
    xyz, w, box = (wl.uniform(3000, 7) if kind == "uniform" else wl.power_uniform(3000, 7))
    if w is not None:
        w = (w * 0.05).astype(np.float32)
    a = to_numpy(gpu_build(xyz, w, box, precision=2))
    d = gpu_build(xyz, w, box, perturb=1)
    b = to_numpy(d)
    assert d.sizes["n_perturbed"] == 0
    for k in ("nbr_off", "nbr", "facet_off", "facet_nbr", "fv_off", "fv", "vert_off", "vert", "vert_planes", "vol",
              "centroid"):
        assert np.array_equal(a[k], b[k]), k


def test_perturbed_lattice_at_size():
    """A 16^3 dyadic lattice (4096 sites, every diagram vertex shared by eight
    cells) built with the perturbation: properties that hold at any size.
    Every cell is the cube of side h about its site (zero-area facets add
    nothing), the perturbed cells are simple polytopes (F = V/2 + 2) with
    symmetric neighbours, and the dual tetrahedra tile the lattice's hull
    exactly once: their absolute volumes (exact in FP64 for these
    coordinates) sum to the hull's, and every triangle is shared by two
    tetrahedra or lies on the hull."""
    import itertools
    import torch
    import paper_2605_06408_amd as vd
    m, h = 16, 1.0 / 16
    xyz = lattice(m, h, h / 2)
    box = np.array([0.0, 0.0, 0.0, 1.0, 1.0, 1.0])
    ctx = vd.Context(0)
    d = ctx.build(torch.from_numpy(xyz).cuda(), None, bbox=[float(v) for v in box], perturb=1)
    tets = ctx.tetrahedra().cpu().numpy().astype(np.int64)
    torch.cuda.synchronize()
    g = to_numpy(d)
    n = len(xyz)
    assert d.sizes["n_uncertain"] == 0 and d.sizes["n_failed"] == 0 and d.sizes["n_perturbed"] > 0
    assert np.abs(g["vol"].astype(np.float64) / h ** 3 - 1.0).max() <= 1e-6
    assert np.abs(g["centroid"].astype(np.float64) - xyz).max() <= 1e-6
    nv = np.diff(g["vert_off"])
    nf = np.diff(g["facet_off"])
    assert np.all(nf == nv // 2 + 2)
    rows = np.repeat(np.arange(n), np.diff(g["nbr_off"]))
    pairs = set(zip(rows.tolist(), g["nbr"].tolist()))
    assert all((j, i) in pairs for i, j in pairs)
    P = xyz.astype(np.float64)
    a, b, c, e = (P[tets[:, k]] for k in range(4))
    vol = np.abs(np.einsum("ij,ij->i", b - a, np.cross(c - a, e - a))) / 6.0
    lo, hi = h / 2, 1.0 - h / 2
    assert vol.sum() == pytest.approx((hi - lo) ** 3, rel=1e-12)
    faces = {}
    for t in tets.tolist():
        for f in itertools.combinations(t, 3):
            faces[f] = faces.get(f, 0) + 1
    assert set(faces.values()) <= {1, 2}
    for f, cnt in faces.items():
        if cnt == 1:
            q = P[list(f)]
            assert any(np.all(q[:, ax] == s) for ax in range(3) for s in (lo, hi)), f
    ctx.close()
