"""GPU backward (vd_backward, the autograd Function) against the FP64
analytic gradient oracle, which finite differences pin on the CPU.

Bar: the gradient is defined through the combinatorics, so it is compared on
sites whose own cell and every neighbouring cell have the same combinatorics
on both sides (same neighbours, facets and vertex plane-triples); those must
be at least 90% of the sites (forward parity makes them almost all), and on
them each gradient component agrees within GRAD_TOL relative to the site's
gradient size plus the mean gradient size.
The GPU evaluates every cell in FP64 from the same FP32 inputs and sums the
shares of a site in FP64, rounding once to FP32 (2^-24 relative); around the
thin cells of tight clusters those shares are up to ~1e8 times the site
gradient they cancel to, which costs 1e8 * 2^-53 ~ 1e-8 in FP64.  GRAD_TOL
leaves room for both with a wide margin."""
import numpy as np
import pytest

from paper_2605_06408_amd import workloads as wl

from .parity import gpu_build

pytestmark = pytest.mark.gpu

GRAD_TOL = 5e-5


def _key_grad(codes, cell):
    """Gradient on each vertex, keyed by (cell, ascending plane codes) so that
    both sides get bit-identical values (FP32): a vertex's gradient must not
    depend on its computed position, since a near-singular vertex solve
    amplifies any difference in it."""
    c = np.asarray(codes, np.int64).reshape(-1, 3)
    key = (c * np.array([3, 5, 7])).sum(axis=1) + 11 * np.asarray(cell, np.int64)
    return np.stack([np.sin(key), np.cos(key), np.sin(2.0 * key)], axis=1).astype(np.float32)


def _key_grad_oracle(x, codes, i):
    return _key_grad(codes, np.full(len(x), i)).astype(np.float64)


def _topology(res, t, gpu):
    """(neighbours, facet codes, sorted vertex plane-triples) of row t."""
    nb = tuple(res["nbr"][res["nbr_off"][t]:res["nbr_off"][t + 1]].tolist())
    fc = tuple(res["facet_nbr" if gpu else "facet_code"][res["facet_off"][t]:res["facet_off"][t + 1]].tolist())
    vc = res["vert_planes" if gpu else "vert_code"][res["vert_off"][t]:res["vert_off"][t + 1]]
    vt = tuple(sorted(tuple(int(c) for c in sorted(r)) for r in np.asarray(vc).reshape(-1, 3)))
    return nb, fc, vt


def _same_topology_sites(d, res, sites):
    """Sites among `sites` whose gradient both sides assemble from the same
    cells with identical combinatorics: the site's cell, its neighbours' cells
    (oracle) and every cell that lists it on the GPU must match between the
    GPU (Diagram d) and the oracle result `res` (which must hold the cells of
    the sites and of their neighbours)."""
    from .parity import to_numpy
    row = {int(i): t for t, i in enumerate(res["ids"])}
    need = np.array(sorted(row), np.int64)
    d = d._replace(**{k: getattr(d, k).detach() for k in ("vol", "centroid", "vert")})
    g = to_numpy(d, need)
    grow = {int(i): t for t, i in enumerate(g["ids"])}
    same = {i: _topology(g, grow[i], True) == _topology(res, row[i], False) for i in row}
    # cells that list each site on the GPU (a cell sends a share to every
    # site it lists, whether or not that site lists it back)
    nbr_off = d.nbr_off.cpu().numpy()
    nbr = d.nbr.cpu().numpy()
    rows = np.repeat(np.arange(len(nbr_off) - 1), np.diff(nbr_off))
    want = np.isin(nbr, np.asarray(sites, np.int64))
    listers = {}
    for i, j in zip(rows[want].tolist(), nbr[want].tolist()):
        listers.setdefault(j, []).append(i)
    out = []
    for j in sites:
        t = row[int(j)]
        nb = res["nbr"][res["nbr_off"][t]:res["nbr_off"][t + 1]]
        if (same[int(j)] and all(same.get(int(i), False) for i in nb)
                and all(same.get(int(i), False) for i in listers.get(int(j), []))):
            out.append(int(j))
    return np.array(out, np.int64)


def _compare(g_gpu, g_orc, sites):
    g_gpu = np.asarray(g_gpu, np.float64)
    g_orc = np.asarray(g_orc, np.float64)
    if g_orc.ndim == 1:
        g_gpu, g_orc = g_gpu[:, None], g_orc[:, None]
    scale = np.abs(g_orc[sites]).max(axis=1) + np.abs(g_orc[sites]).max(axis=1).mean()
    err = np.abs(g_gpu[sites] - g_orc[sites]).max(axis=1) / scale
    return err


def _run_backward(xyz, w, box, g_vol, g_cen, with_vert):
    import torch
    import paper_2605_06408_amd as vd
    ctx = vd.Context(0)
    x = torch.from_numpy(xyz).cuda()
    ww = None if w is None else torch.from_numpy(w).cuda()
    d = ctx.build(x, ww, bbox=None if box is None else [float(v) for v in box])
    gv = torch.from_numpy(g_vol.astype(np.float32)).cuda()
    gc = torch.from_numpy(g_cen.astype(np.float32)).cuda()
    gx = None
    if with_vert:
        vp = d.vert_planes.cpu().numpy()
        cell = np.repeat(np.arange(len(xyz)), np.diff(d.vert_off.cpu().numpy()))
        gx = torch.from_numpy(_key_grad(vp, cell)).cuda()
    g_xyz, g_w = ctx.backward(gv, gc, gx, want_w=True)
    torch.cuda.synchronize()
    return d, g_xyz.cpu().numpy(), g_w.cpu().numpy(), ctx


@pytest.mark.parametrize("name,with_vert", [("uniform", False), ("uniform", True), ("power_uniform", False),
                                            ("power_uniform", True), ("clustered", True)])
def test_backward_matches_oracle(oracle_mod, name, with_vert):
    from oracle import grad as og
    n = 3000
    xyz, w, box = getattr(wl, name)(n, 5)
    rng = np.random.default_rng(9)
    g_vol = rng.normal(size=n) * n
    g_cen = rng.normal(size=(n, 3))
    d, gp, gw, _ = _run_backward(xyz, w, box, g_vol, g_cen, with_vert)
    op, ow, res = og.backward(xyz, w, box, g_vol, g_cen, _key_grad_oracle if with_vert else None)
    sites = _same_topology_sites(d, res, np.arange(n))
    assert len(sites) >= 0.9 * n
    e = _compare(gp, op, sites)
    print("%s vert=%s: %d sites, max rel err %.2e" % (name, with_vert, len(sites), e.max()))
    assert e.max() <= GRAD_TOL
    if w is not None:
        ew = _compare(gw, ow, sites)
        assert ew.max() <= GRAD_TOL


def test_two_sites_closed_form_on_gpu():
    # dV0/dw1 = -A / (2 D) = -1 and dV0/dw0 = +1; dV0/dx0 = 1/2 + (w0 - w1)/(2 D^2)
    xyz = np.array([[0.25, 0.5, 0.5], [0.75, 0.5, 0.5]], np.float32)
    w = np.array([0.0625, 0.0], np.float32)
    box = np.array([0, 0, 0, 1, 1, 1.0])
    _, gp, gw, _ = _run_backward(xyz, w, box, np.array([1.0, 0.0]), np.zeros((2, 3)), False)
    assert gw == pytest.approx([1.0, -1.0], abs=1e-6)
    assert gp[0] == pytest.approx([0.5 + 0.0625 / 0.5, 0, 0], abs=1e-6)
    assert gp[1] == pytest.approx([0.5 - 0.0625 / 0.5, 0, 0], abs=1e-6)


def test_empty_cells_pass_the_centroid_gradient():
    # an empty power cell has c = p_i: its site receives g_cen[i] and nothing else
    xyz = np.array([[0.3, 0.5, 0.5], [0.32, 0.5, 0.5], [0.8, 0.4, 0.6], [0.6, 0.8, 0.3]], np.float32)
    w = np.array([0.05, 0.0, 0.0, 0.01], np.float32)
    box = np.array([0, 0, 0, 1, 1, 1.0])
    g_cen = np.arange(12, dtype=float).reshape(4, 3) / 10.0
    d, gp, gw, _ = _run_backward(xyz, w, box, np.array([0.3, -1.0, 0.7, 0.2]), g_cen, False)
    assert int(d.flags[1].item()) & 1
    assert gp[1] == pytest.approx(g_cen[1], abs=1e-6)
    from oracle import grad as og
    op, ow, _ = og.backward(xyz, w, box, np.array([0.3, -1.0, 0.7, 0.2]), g_cen)
    np.testing.assert_allclose(gp, op, rtol=1e-5, atol=1e-5)
    np.testing.assert_allclose(gw, ow, rtol=1e-5, atol=1e-5)


def test_backward_is_deterministic():
    import torch
    xyz, w, box = wl.power_uniform(5000, 2)
    rng = np.random.default_rng(1)
    g_vol = rng.normal(size=5000)
    g_cen = rng.normal(size=(5000, 3))
    _, gp1, gw1, ctx = _run_backward(xyz, w, box, g_vol, g_cen, True)
    gv = torch.from_numpy(g_vol.astype(np.float32)).cuda()
    gc = torch.from_numpy(g_cen.astype(np.float32)).cuda()
    g2, w2 = ctx.backward(gv, gc, None)
    _, gp3, gw3, _ = _run_backward(xyz, w, box, g_vol, g_cen, True)
    assert np.array_equal(gp1, gp3) and np.array_equal(gw1, gw3)
    assert not np.array_equal(gp1, g2.cpu().numpy())  # the vertex term matters


def test_autograd_function_config5_loss(oracle_mod):
    """loss = sum_i (V_i - |B|/n)^2 + |c_i - p_i|^2 through torch autograd."""
    import torch
    import paper_2605_06408_amd as vd
    from oracle import grad as og
    n = 2000
    xyz, w, box = wl.power_clustered(n, 3)
    x = torch.from_numpy(xyz).cuda().requires_grad_(True)
    ww = torch.from_numpy(w).cuda().requires_grad_(True)
    d = vd.power_diagram(x, ww, bbox=[float(v) for v in box])
    loss = ((d.vol - 1.0 / n) ** 2).sum() + ((d.centroid - x) ** 2).sum()
    loss.backward()
    gp, gw = x.grad.cpu().numpy(), ww.grad.cpu().numpy()
    vol = d.vol.detach().double().cpu().numpy()
    cen = d.centroid.detach().double().cpu().numpy()
    g_vol = 2.0 * (vol - 1.0 / n)
    g_cen = 2.0 * (cen - xyz.astype(np.float64))
    op, ow, res = og.backward(xyz, w, box, g_vol, g_cen)
    op = op - g_cen  # the loss's own explicit -p term
    sites = _same_topology_sites(d, res, np.arange(n))
    assert len(sites) >= 0.9 * n
    assert _compare(gp, op, sites).max() <= GRAD_TOL
    assert _compare(gw, ow, sites).max() <= GRAD_TOL


def test_backward_after_another_build_is_refused():
    import torch
    import paper_2605_06408_amd as vd
    xyz, w, box = wl.power_uniform(500, 1)
    ctx = vd.Context(0)
    x = torch.from_numpy(xyz).cuda().requires_grad_(True)
    d = vd.power_diagram(x, None, bbox=[float(v) for v in box], context=ctx)
    ctx.build(x.detach(), None, bbox=[float(v) for v in box])
    with pytest.raises(RuntimeError, match="another build"):
        d.vol.sum().backward()


def test_backward_power_clustered_million_sampled(oracle_mod):
    """The differentiable power diagram of 1M clustered sites: the backward in
    the configuration bench.py times, sampled sites against the oracle."""
    import torch
    from oracle import grad as og
    xyz, w, box = wl.make("power_clustered_1m", 0)
    n = len(xyz)
    rng = np.random.default_rng(4)
    d = gpu_build(xyz, w, box)
    vol = d.vol.double().cpu().numpy()
    cen = d.centroid.double().cpu().numpy()
    g_vol = 2.0 * (vol - 1.0 / n)
    g_cen = 2.0 * (cen - xyz.astype(np.float64))
    import paper_2605_06408_amd as vd
    ctx = vd.context(d.vol.device)
    g_xyz, g_w = ctx.backward(torch.from_numpy(g_vol.astype(np.float32)).cuda(),
                              torch.from_numpy(g_cen.astype(np.float32)).cuda())
    gp, gw = g_xyz.cpu().numpy(), g_w.cpu().numpy()
    flags = d.flags.cpu().numpy()
    # half the sample from non-empty cells (most clustered cells are empty)
    nonempty = np.nonzero((flags & 1) == 0)[0]
    ids = np.unique(np.concatenate([rng.choice(n, 60, replace=False), rng.choice(nonempty, 60, replace=False)]))
    op, ow, res = og.backward(xyz, w, box, g_vol, g_cen, ids=ids)
    sites = _same_topology_sites(d, res, ids)
    assert len(sites) >= 0.9 * len(ids)
    e = _compare(gp, op, sites)
    ew = _compare(gw, ow, sites)
    print("1M sampled: %d sites, max rel err %.2e / %.2e" % (len(sites), e.max(), ew.max()))
    assert e.max() <= GRAD_TOL and ew.max() <= GRAD_TOL


def test_backward_very_large_cells(oracle_mod):
    """Gradients through cells of hundreds to thousands of vertices (the
    wave-group passes, and the hand-over between them): the heavy sites and a
    sample of others against the oracle, with the vertex term."""
    from oracle import grad as og
    from .test_gpu_parity import _heavy_sites
    xyz, w, box, big = _heavy_sites(40000, 21)
    n = len(xyz)
    rng = np.random.default_rng(6)
    g_vol = rng.normal(size=n) * n
    g_cen = rng.normal(size=(n, 3))
    d, gp, gw, _ = _run_backward(xyz, w, box, g_vol, g_cen, True)
    assert d.sizes["n_resumed"] >= 1
    ids = np.unique(np.concatenate([np.arange(big), rng.choice(n, 40, replace=False)]))
    op, ow, res = og.backward(xyz, w, box, g_vol, g_cen, _key_grad_oracle, ids=ids)
    sites = _same_topology_sites(d, res, ids)
    # the largest cell is too large for the oracle to certify (FP32 may drop
    # or add a sliver facet); the others must be comparable
    assert len(set(sites.tolist()) & {1, 2, 3}) >= 2
    assert len(sites) >= 0.8 * len(ids)
    e = _compare(gp, op, sites)
    ew = _compare(gw, ow, sites)
    print("very large cells: %d of %d sites, max rel err %.2e / %.2e" % (len(sites), len(ids), e.max(), ew.max()))
    assert e.max() <= GRAD_TOL and ew.max() <= GRAD_TOL


@pytest.mark.parametrize("name", ["uniform", "power_uniform"])
def test_backward_with_box_of_the_sites(oracle_mod, name):
    """No box given: the box is the sites' bounding box and its faces move
    with the extreme sites, whose gradients then carry the faces' terms (the
    oracle is pinned by finite differences that recompute that box)."""
    from oracle import grad as og
    n = 2000
    xyz, w, _ = getattr(wl, name)(n, 8)
    rng = np.random.default_rng(2)
    g_vol = rng.normal(size=n) * n
    g_cen = rng.normal(size=(n, 3))
    d, gp, gw, _ = _run_backward(xyz, w, None, g_vol, g_cen, False)
    op, ow, res = og.backward(xyz, w, None, g_vol, g_cen)
    sites = _same_topology_sites(d, res, np.arange(n))
    ext = np.unique(np.concatenate([xyz.argmin(0), xyz.argmax(0)]))
    assert len(sites) >= 0.9 * n and set(ext.tolist()) <= set(sites.tolist())
    e = _compare(gp, op, sites)
    print("%s, box of the sites: %d sites, max rel err %.2e (extreme sites %.2e)"
          % (name, len(sites), e.max(), _compare(gp, op, ext).max()))
    assert e.max() <= GRAD_TOL
    if w is not None:
        assert _compare(gw, ow, sites).max() <= GRAD_TOL


def test_vertex_gradient_must_cover_every_vertex():
    import torch
    import paper_2605_06408_amd as vd
    xyz, w, box = wl.uniform(300, 1)
    ctx = vd.Context(0)
    d = ctx.build(torch.from_numpy(xyz).cuda(), None, bbox=[float(v) for v in box])
    short = torch.zeros((d.sizes["n_vert"] - 1, 3), dtype=torch.float32, device="cuda")
    with pytest.raises(ValueError):
        ctx.backward(None, None, short)


def _config5_gradient():
    """The differentiable power diagram of the 1M-site clustered power
    workload and the gradient of L = sum_i (V_i - |B|/n)^2 + |c_i - p_i|^2
    through torch autograd (vd_backward), as bench.py times it."""
    import torch
    import paper_2605_06408_amd as vd
    xyz, w, box = wl.make("power_clustered_1m", 0)
    n = len(xyz)
    x = torch.from_numpy(xyz).cuda().requires_grad_(True)
    ww = torch.from_numpy(w).cuda().requires_grad_(True)
    ctx = vd.Context(0)
    d = vd.power_diagram(x, ww, bbox=[float(v) for v in box], context=ctx)
    loss = ((d.vol - 1.0 / n) ** 2).sum() + ((d.centroid - x) ** 2).sum()
    loss.backward()
    torch.cuda.synchronize()
    return xyz, w, box, d, x.grad.cpu().numpy(), ww.grad.cpu().numpy()


def test_config5_finite_differences(oracle_mod):
    """FP64 central finite differences of the config-5 loss on 1000 sampled
    sites (500 uniformly, 500 among non-empty cells: about 92% of the cells
    are empty), through the oracle with the site moved (steps 1e-6 l and
    1e-6 l^2 for positions and weights, l the cell's diagonal or, for an empty
    cell, the nearest-site distance), against vd_backward.  A site is compared
    where its cell and its neighbours' cells are certified (the combinatorics
    hold under the step) and match the GPU's."""
    import oracle
    xyz, w, box, d, gp, gw = _config5_gradient()
    n = len(xyz)
    rng = np.random.default_rng(1000)
    flags = d.flags.cpu().numpy()
    nonempty = np.nonzero((flags & 1) == 0)[0]
    sites = np.unique(np.concatenate([rng.choice(n, 500, replace=False), rng.choice(nonempty, 500, replace=False)]))
    first = oracle.cells(xyz, w, box, ids=sites)
    need = np.unique(np.concatenate([sites, first["nbr"]]))
    res = oracle.cells(xyz, w, box, ids=need)
    row = {int(i): t for t, i in enumerate(need)}
    ok = set(_same_topology_sites(d, res, sites).tolist())
    # certified: the site's cell and its neighbours' cells are at least
    # 1e-5 from a change of combinatorics (tight clusters leave many below)
    certified = [int(k) for k in sites
                 if all(res["margin"][row[int(j)]] >= 1e-5
                        for j in np.concatenate([[k], res["nbr"][res["nbr_off"][row[int(k)]]:res["nbr_off"][row[int(k)] + 1]]]))]
    cert = [k for k in certified if k in ok]
    print("config 5: %d sampled sites, %d certified with their neighbours, %d of those with the GPU's combinatorics"
          % (len(sites), len(certified), len(cert)))
    assert len(certified) >= 0.6 * len(sites), (len(certified), len(sites))
    assert len(cert) >= 0.99 * len(certified), (len(cert), len(certified))
    x64, w64 = xyz.astype(np.float64), w.astype(np.float64)
    S = oracle.Session(x64, w64, box)

    def local_loss(k, cells, pk, wk):
        r = S.cells(cells, moved=(k, pk, wk))
        p = x64[cells].copy()
        p[cells == k] = pk
        return float(np.sum((r["vol"] - 1.0 / n) ** 2) + np.sum((r["centroid"] - p) ** 2))

    fd_p = np.zeros((n, 3))
    fd_w = np.zeros(n)
    for k in cert:
        t = row[k]
        cells = np.unique(np.concatenate([[k], res["nbr"][res["nbr_off"][t]:res["nbr_off"][t + 1]]]))
        v = res["vert"][res["vert_off"][t]:res["vert_off"][t + 1]]
        ell = float(np.linalg.norm(v.max(0) - v.min(0))) if len(v) else float(
            np.sort(np.linalg.norm(x64 - x64[k], axis=1))[1])
        hp, hw = 1e-6 * ell, 1e-6 * ell * ell
        for c in range(3):
            e = np.zeros(3)
            e[c] = hp
            fd_p[k, c] = (local_loss(k, cells, x64[k] + e, w64[k]) - local_loss(k, cells, x64[k] - e, w64[k])) / (2 * hp)
        fd_w[k] = (local_loss(k, cells, x64[k], w64[k] + hw) - local_loss(k, cells, x64[k], w64[k] - hw)) / (2 * hw)
    S.close()
    cert = np.array(cert, np.int64)
    ep = _compare(gp, fd_p, cert)
    ew = _compare(gw, fd_w, cert)
    print("config 5 finite differences: %d of %d sites, max rel err positions %.2e weights %.2e"
          % (len(cert), len(sites), ep.max(), ew.max()))
    assert ep.max() <= GRAD_TOL and ew.max() <= GRAD_TOL


def test_config5_volume_weight_closed_form():
    """dV_i/dw_j = -A_ij / (2 D_ij) for a neighbour j and
    dV_i/dw_i = sum_j A_ij / (2 D_ij) (box facets do not depend on weights),
    with A_ij the area of the GPU's own facet ring (FP64 shoelace) and
    D_ij = |p_j - p_i|: vd_backward with g_vol = 1 on 300 non-empty cells of
    the 1M-site clustered power workload that share no neighbour."""
    import torch
    import paper_2605_06408_amd as vd
    from .parity import to_numpy
    xyz, w, box = wl.make("power_clustered_1m", 0)
    n = len(xyz)
    ctx = vd.Context(0)
    d = ctx.build(torch.from_numpy(xyz).cuda(), torch.from_numpy(w).cuda(), bbox=[float(v) for v in box])
    flags = d.flags.cpu().numpy()
    off = d.nbr_off.cpu().numpy()
    nbr = d.nbr.cpu().numpy()
    rng = np.random.default_rng(5)
    chosen, taken = [], set()
    for i in rng.permutation(np.nonzero((flags & 1) == 0)[0]):
        nb = set(nbr[off[i]:off[i + 1]].tolist()) | {int(i)}
        if nb & taken:
            continue
        chosen.append(int(i))
        taken |= nb
        # the neighbours' other neighbours may be chosen; their g_w then mixes
        # two cells, so every site next to a chosen cell is reserved
        if len(chosen) == 300:
            break
    g_vol = np.zeros(n, np.float32)
    g_vol[chosen] = 1.0
    _, g_w = ctx.backward(torch.from_numpy(g_vol).cuda(), None, None)
    g_w = g_w.cpu().numpy().astype(np.float64)
    g = to_numpy(d, np.array(chosen))
    # The areas come from the FP32 output vertices: each coordinate carries
    # up to 2^-24 |x| of rounding, so a ring's area is known to within
    # 2^-23 max|x| times its perimeter (each edge moves with both ends);
    # the backward itself works in FP64.  Each comparison is held to 1e-6 of
    # sum_j A_ij / (2 D_ij) plus that area uncertainty over 2 D_ij.
    worst = 0.0
    for t, i in enumerate(chosen):
        own, own_unc, excess = 0.0, 0.0, 0.0
        for f in range(g["facet_off"][t], g["facet_off"][t + 1]):
            j = int(g["facet_nbr"][f])
            if j < 0:
                continue
            ring = g["vert"][g["fv"][g["fv_off"][f]:g["fv_off"][f + 1]]].astype(np.float64)
            unc = 2.0 ** -23 * float(np.abs(ring).max()) * float(
                sum(np.linalg.norm(ring[(q + 1) % len(ring)] - ring[q]) for q in range(len(ring))))
            ring = ring - ring[0]
            area = 0.5 * np.linalg.norm(sum(np.cross(ring[q], ring[(q + 1) % len(ring)]) for q in range(len(ring))))
            D = float(np.linalg.norm(xyz[j].astype(np.float64) - xyz[i].astype(np.float64)))
            own += area / (2 * D)
            own_unc += unc / (2 * D)
            # i is the only chosen cell next to j
            excess = max(excess, abs(g_w[j] + area / (2 * D)) - unc / (2 * D))
        excess = max(excess, abs(g_w[i] - own) - own_unc)
        worst = max(worst, excess / own)
    print("closed form dV/dw on %d cells: max error beyond the FP32 area uncertainty %.2e of sum_j A_ij / (2 D_ij)"
          % (len(chosen), worst))
    assert len(chosen) == 300
    assert worst <= 1e-6
