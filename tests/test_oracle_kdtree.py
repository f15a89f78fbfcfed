"""The oracle's k-d tree candidate mode against its brute-force mode.

Both take the candidates of a cell in increasing plane distance d_ij (Sec. 4.2,
Eq. 2; ties by index) and stop once d_ij exceeds the cell's largest vertex
distance; the tree only finds them faster (best-first over a median-split
k-d tree keyed by the node bound of Sec. 4.2.2).  The clip sequence is then
the same, so every output, the robustness margin included, must agree bit
for bit.  Brute force is itself pinned by tests/test_oracle_pins.py."""
import numpy as np
import pytest

import oracle
from paper_2605_06408_amd import workloads as wl

KEYS = ["nbr_off", "nbr", "vert_off", "vert", "vert_code", "facet_off", "facet_code", "fv_off", "fv", "vol",
        "centroid", "flags", "margin"]


@pytest.mark.parametrize("name,n", [("uniform", 20000), ("clustered", 20000), ("surface", 8000),
                                    ("power_uniform", 20000), ("power_clustered", 20000),
                                    ("paper_clusters_w", 10000)])
def test_kdtree_mode_is_bit_identical(name, n):
    if name == "paper_clusters_w":
        xyz, w, box = wl.make("paper_clusters10_w_1m", 4, n)
    else:
        xyz, w, box = getattr(wl, name)(n, 3)
    a = oracle.cells(xyz, w, box, candidates="brute")
    b = oracle.cells(xyz, w, box, candidates="kdtree")
    for k in KEYS:
        assert np.array_equal(a[k], b[k]), k
    assert (a["flags"] & oracle.FLAG_EMPTY).sum() < n


def test_kdtree_mode_on_coincident_and_tiny_inputs():
    """Coincident sites (losers dropped, twins flagged), sites outside the box,
    and inputs smaller than one tree leaf."""
    rng = np.random.default_rng(8)
    xyz = rng.random((3000, 3)).astype(np.float32)
    xyz[10:20] = xyz[5]
    xyz[100:103] = xyz[7]
    w = (rng.random(3000) * 1e-4).astype(np.float32)
    w[100] = 0.01
    xyz[200:210] += 0.5  # outside the box
    box = np.array([0, 0, 0, 1, 1, 1.0])
    for ww in (None, w):
        a = oracle.cells(xyz, ww, box, candidates="brute")
        b = oracle.cells(xyz, ww, box, candidates="kdtree")
        for k in KEYS:
            assert np.array_equal(a[k], b[k]), k
    for n in (1, 2, 5, 9):
        a = oracle.cells(xyz[:n], None, box, candidates="brute")
        b = oracle.cells(xyz[:n], None, box, candidates="kdtree")
        for k in KEYS:
            assert np.array_equal(a[k], b[k]), (n, k)


def test_kdtree_mode_on_sampled_cells():
    """A sample of cells (ids) of a larger set, as the full-size parity tests
    and the CPU baseline use it."""
    xyz, w, box = wl.make("power_clustered_1m", 1, 60000)
    ids = np.sort(np.random.default_rng(2).choice(len(xyz), 800, replace=False))
    a = oracle.cells(xyz, w, box, ids=ids, candidates="brute")
    b = oracle.cells(xyz, w, box, ids=ids, candidates="kdtree")
    for k in KEYS:
        assert np.array_equal(a[k], b[k]), k


def test_session_with_a_moved_site_matches_a_fresh_run():
    """oracle.Session keeps the sites and the k-d tree across calls and can
    move one site first (finite differences): its cells equal those of a
    brute-force run on a copy with that site moved."""
    xyz, w, box = wl.make("power_clustered_1m", 0, 60000)
    x64, w64 = xyz.astype(np.float64), w.astype(np.float64)
    S = oracle.Session(x64, w64, box, candidates="kdtree")
    rng = np.random.default_rng(0)
    nonempty = np.nonzero((oracle.cells(xyz, w, box, ids=np.arange(0, 60000, 7), margin=False)["flags"] & 1) == 0)[0] * 7
    for k in list(rng.choice(60000, 10, replace=False)) + list(rng.choice(nonempty, 10, replace=False)):
        k = int(k)
        pk = x64[k] + rng.normal(size=3) * 1e-4
        wk = w64[k] * (1.0 + 1e-3)
        nb = oracle.cells(x64, w64, box, ids=[k], fp64=True)["nbr"]
        ids = np.unique(np.concatenate([[k], nb, rng.choice(60000, 5)]))
        a = S.cells(ids, margin=True, moved=(k, pk, wk))
        x2, w2 = x64.copy(), w64.copy()
        x2[k], w2[k] = pk, wk
        b = oracle.cells(x2, w2, box, ids=ids, fp64=True, candidates="brute")
        for q in KEYS:
            assert np.array_equal(a[q], b[q]), (k, q)
        # and the site is back in place afterwards
        c = S.cells(ids, margin=True)
        d = oracle.cells(x64, w64, box, ids=ids, fp64=True, candidates="brute")
        for q in KEYS:
            assert np.array_equal(c[q], d[q]), (k, q)
