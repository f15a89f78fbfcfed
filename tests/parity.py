"""Helpers for the GPU-vs-oracle parity tests (imported by tests only).

Both sides are brought to one canonical form per cell: neighbour ids
ascending; vertices keyed by their ascending triple of facet codes (site id
or box face -1..-6); facets keyed by code, each polygon as the cyclic list of
its vertex keys starting at the smallest key (orientation preserved).

Gate (readings of "bit-exact neighbours on inputs in general position" and
"1e-5 relative geometry"): a cell whose oracle margin is at least `tau` is
certified -- its combinatorics are far from any degeneracy at the precision
compared -- and must match exactly: empty flag, neighbour list, vertex keys
and facet polygons.  The plain FP32 form is gated at tau = 1e-5, the mixed
FP32/FP64 form (FP64 re-evaluation of doubtful signs) at TAU_MIXED = 1e-10.  On certified non-empty cells, vertices and centroids must
satisfy |x - x*|_inf / max(|x*|_inf, l) <= tol with l the diagonal of the
cell's bounding box, and volumes |V - V*| / V* <= tol.  Uncertified cells are
only counted.
"""
from __future__ import annotations

import numpy as np

TAU_FP32 = 1e-5
TAU_MIXED = 1e-10

FIELDS = ("nbr_off", "nbr", "facet_off", "facet_nbr", "fv_off", "fv", "vert_off", "vert", "vert_planes", "vol",
          "centroid", "flags")


def gpu_build(xyz, w, box, **kw):
    """Run the library on the GPU; returns the torch Diagram."""
    import torch
    import paper_2605_06408_amd as vd
    x = torch.from_numpy(np.ascontiguousarray(xyz, np.float32)).cuda()
    ww = None if w is None else torch.from_numpy(np.ascontiguousarray(w, np.float32)).cuda()
    d = vd.build(x, ww, bbox=None if box is None else [float(v) for v in box], **kw)
    torch.cuda.synchronize()
    return d


def to_numpy(d, ids=None) -> dict:
    """Whole diagram (ids None) or the rows of cells `ids`, as numpy arrays
    with re-based offsets.  Row gathering happens on the device."""
    import torch
    if ids is None:
        out = {k: getattr(d, k).cpu().numpy() for k in FIELDS}
        out["ids"] = np.arange(len(out["vol"]))
        out["vert_base"] = out["vert_off"][:-1].copy()
        return out
    dev = d.vol.device
    tid = torch.as_tensor(np.asarray(ids, np.int64), device=dev)

    def rows(off, sel):
        s, e = off[sel], off[sel + 1]
        ln = e - s
        new = torch.zeros(len(sel) + 1, dtype=torch.int64, device=dev)
        new[1:] = torch.cumsum(ln, 0)
        tot = int(new[-1].item())
        idx = torch.repeat_interleave(s - new[:-1], ln, output_size=tot) + torch.arange(tot, device=dev)
        return idx, new

    out = {}
    ni, out["nbr_off"] = rows(d.nbr_off, tid)
    out["nbr"] = d.nbr[ni]
    vi, out["vert_off"] = rows(d.vert_off, tid)
    out["vert"] = d.vert[vi]
    out["vert_planes"] = d.vert_planes[vi]
    fi, out["facet_off"] = rows(d.facet_off, tid)
    out["facet_nbr"] = d.facet_nbr[fi]
    fvi, out["fv_off"] = rows(d.fv_off, fi)
    # global vertex index -> index within the gathered vertex rows
    cell_of_facet = torch.repeat_interleave(torch.arange(len(tid), device=dev),
                                            out["facet_off"][1:] - out["facet_off"][:-1])
    cell_of_fv = torch.repeat_interleave(cell_of_facet, out["fv_off"][1:] - out["fv_off"][:-1])
    out["fv"] = d.fv[fvi].to(torch.int64) - d.vert_off[tid][cell_of_fv] + out["vert_off"][:-1][cell_of_fv]
    out["vol"] = d.vol[tid]
    out["centroid"] = d.centroid[tid]
    out["flags"] = d.flags[tid]
    out = {k: v.cpu().numpy() for k, v in out.items()}
    out["ids"] = np.asarray(ids, np.int64)
    out["vert_base"] = out["vert_off"][:-1].copy()
    return out


def _canon_gpu(g, t):
    v0, v1 = g["vert_off"][t], g["vert_off"][t + 1]
    keys = [tuple(int(c) for c in r) for r in g["vert_planes"][v0:v1]]
    verts = {k: g["vert"][v0 + j].astype(np.float64) for j, k in enumerate(keys)}
    facets = {}
    for f in range(g["facet_off"][t], g["facet_off"][t + 1]):
        idx = [int(x) - v0 for x in g["fv"][g["fv_off"][f]:g["fv_off"][f + 1]]]
        if not idx or min(idx) < 0 or max(idx) >= len(keys):
            facets[int(g["facet_nbr"][f])] = ("malformed",)
            continue
        ring = [keys[q] for q in idx]
        r = min(range(len(ring)), key=lambda q: ring[q])
        facets[int(g["facet_nbr"][f])] = tuple(ring[r:] + ring[:r])
    nbr = [int(x) for x in g["nbr"][g["nbr_off"][t]:g["nbr_off"][t + 1]]]
    return nbr, verts, facets, len(keys)


def _canon_oracle(o, t):
    v0, v1 = o["vert_off"][t], o["vert_off"][t + 1]
    keys = [tuple(int(c) for c in r) for r in o["vert_code"][v0:v1]]
    verts = {k: o["vert"][v0 + j] for j, k in enumerate(keys)}
    facets = {}
    for f in range(o["facet_off"][t], o["facet_off"][t + 1]):
        ring = [keys[int(x)] for x in o["fv"][o["fv_off"][f]:o["fv_off"][f + 1]]]
        r = min(range(len(ring)), key=lambda q: ring[q])
        facets[int(o["facet_code"][f])] = tuple(ring[r:] + ring[:r])
    nbr = [int(x) for x in o["nbr"][o["nbr_off"][t]:o["nbr_off"][t + 1]]]
    return nbr, verts, facets, len(keys)


def _poly_volume(verts: dict, facets: dict) -> float:
    """Volume of a closed polytope from its facet rings (FP64 fan)."""
    keys = list(verts)
    ref = verts[keys[0]]
    v6 = 0.0
    for ring in facets.values():
        if ring and ring[0] == "malformed":
            return float("nan")
        a = verts[ring[0]] - ref
        for t in range(1, len(ring) - 1):
            b = verts[ring[t]] - ref
            c = verts[ring[t + 1]] - ref
            v6 += float(np.dot(a, np.cross(b, c)))
    return v6 / 6.0


def compare(g: dict, o: dict, tau: float = 1e-5, tol: float = 1e-5, max_report: int = 5) -> dict:
    """Compare GPU rows `g` and oracle rows `o` for the same cells (same order)."""
    assert np.array_equal(g["ids"], o["ids"])
    rep = dict(cells=len(g["ids"]), certified=0, topo_fail=[], geo_fail=[], uncertified=0,
               uncertified_mismatch=0, max_vert_err=0.0, max_vol_err=0.0, max_cen_err=0.0, empty=0, tau=tau)
    # per certified non-empty cell: vertex (global, relative to max(|x*|, l)),
    # vertex in the cell's frame (relative to l), volume and centroid errors
    errs = {"vert": [], "vert_local": [], "vol": [], "cen": []}
    for t in range(len(g["ids"])):
        cert = o["margin"][t] >= tau
        ge = bool(g["flags"][t] & 1)
        oe = bool(o["flags"][t] & 1)
        rep["empty"] += int(oe)
        gn, gv, gf, _ = _canon_gpu(g, t)
        on, ov, of, _ = _canon_oracle(o, t)
        same = ge == oe and gn == on and set(gv) == set(ov) and gf == of
        if not cert:
            rep["uncertified"] += 1
            rep["uncertified_mismatch"] += int(not same)
            continue
        rep["certified"] += 1
        if not same:
            if len(rep["topo_fail"]) < max_report:
                rep["topo_fail"].append(dict(cell=int(g["ids"][t]), gpu_flags=int(g["flags"][t]), oracle_empty=oe,
                                             only_gpu=sorted(set(gn) - set(on)), only_oracle=sorted(set(on) - set(gn)),
                                             nbr_equal=gn == on, verts_equal=set(gv) == set(ov),
                                             margin=float(o["margin"][t])))
            else:
                rep["topo_fail"].append(int(g["ids"][t]))
            continue
        if oe:
            continue
        P = np.array(list(ov.values()))
        ell = float(np.linalg.norm(P.max(0) - P.min(0)))
        ve = max(float(np.max(np.abs(gv[k] - ov[k])) / max(float(np.max(np.abs(ov[k]))), ell)) for k in ov)
        vv = abs(float(g["vol"][t]) - float(o["vol"][t])) / float(o["vol"][t])
        c_ref = o["centroid"][t]
        ce = float(np.max(np.abs(g["centroid"][t].astype(np.float64) - c_ref))) / max(float(np.max(np.abs(c_ref))), ell)
        errs["vert"].append(ve)
        errs["vert_local"].append(max(float(np.max(np.abs(gv[k] - ov[k]))) for k in ov) / ell)
        errs["vol"].append(vv)
        errs["cen"].append(ce)
        rep["max_vert_err"] = max(rep["max_vert_err"], ve)
        rep["max_vol_err"] = max(rep["max_vol_err"], vv)
        rep["max_cen_err"] = max(rep["max_cen_err"], ce)
        if ve > tol or vv > tol or ce > tol:
            if len(rep["geo_fail"]) < max_report:
                rep["geo_fail"].append(dict(cell=int(g["ids"][t]), vert=ve, vol=vv, cen=ce,
                                            gpu_vol=float(g["vol"][t]), oracle_vol=float(o["vol"][t]),
                                            gpu_vol_from_own_vertices=_poly_volume(gv, gf),
                                            gpu_flags=int(g["flags"][t]), nv=len(gv)))
    rep["errs"] = {k: np.asarray(v, np.float64) for k, v in errs.items()}
    return rep


def error_table(rep: dict) -> dict:
    """p50 / p99 / max of each geometry error of a compare() report."""
    out = {}
    for k, v in rep["errs"].items():
        out[k] = [float(np.quantile(v, 0.5)), float(np.quantile(v, 0.99)), float(v.max())] if len(v) else None
    return out


def assert_parity(rep: dict, min_certified_frac: float = 0.9):
    msg = "parity report: %r" % {k: v for k, v in rep.items() if k != "errs"}
    print(msg)
    assert not rep["topo_fail"], msg
    assert not rep["geo_fail"], msg
    assert rep["certified"] >= min_certified_frac * rep["cells"], msg
