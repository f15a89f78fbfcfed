"""Throughput of the diagram construction on one MI355X.

One step = one full vd_build + vd_write (LBVH build, traversal and clipping,
prefix sums, CSR write-out of neighbours, facets, vertices, volumes and
centroids) over the whole site set, with the sites already resident in HBM.
Timing follows the paper's protocol (Sec. 5.2: warm-up runs, then the mean
of timed runs), bracketed by device synchronisation.

The headline `value` is the clustered 1M Voronoi workload.  Further legs,
each timed the same way: the 20M surface-like Voronoi workload and the
uniform 1M power workload (plain FP32 and mixed FP32/FP64 forms), the mixed
form on the headline workload, and one training step of the differentiable
1M clustered power diagram (forward, loss, hand-written backward).

Roofline.  Nothing here is a dense contraction; the work is FP32 vector
arithmetic, priced per counted work unit in lane operations (an FMA is one):
    W_alg = 4 N_cls + 36 N_vnew + 30 N_node + 15 N_site + 16 N_fin
(side tests, new vertices, BVH child-box tests, leaf site tests, final
vertices), against P_VALU = 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 39.3e12
lane operations per second (non-packed FP32; 78.6 TFLOP/s with FMA = 2).
The compulsory HBM bytes of a step are
    B_alg = 16 n (sites) + 24 n (Morton keys and indices) + 32 (2 n / l)
            (BVH nodes) + the exact output bytes,
against 8 TB/s; the roofline time is max(t_VALU, t_HBM).  The `roofline`
object prices the dominant kernel (the 64-vertex traversal+clip pass, timed by
HIP events on the library's stream) with its own work counters.

The CPU baseline is the FP64 oracle (k-d tree candidates, no robustness
margins, all host threads) on a random sample of the headline workload's
cells; the same oracle run on that sample, and one on a sample of the 20M
workload, are the FP64 reference of the error tables of both forms.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "cells/sec at 1M and 20M sites (Voronoi, power); fwd+bwd cells/sec"

# Lane operations (FMA = 1) per counted work unit.
W_COST = {"classify": 4, "new_vertex": 36, "node_test": 30, "site_test": 15, "final_vertex": 16}
P_VALU_TOPS = 39.3        # 256 CUs x 64 lanes x 2.4 GHz, 10^12 lane operations per second
PEAK_HBM_GBS = 8000.0     # MI355X HBM3E

# HBM traffic of the 64-vertex clip kernel per launch, from two rocprofv3 --pmc
# runs (FETCH_SIZE, WRITE_SIZE; KiB per dispatch) of bench.py on the named
# workload, each scaled by what the same counter reads for a plain 256 MiB
# device copy in the same run.  Valid only while the kernel source is unchanged.
TRAFFIC_MEASURED = {
    "sources_sha1": {"paper_2605_06408_amd/csrc/vd_clip.hip": "8b7a529a5af7ea0e90c41faeb3f8d35f56feccdd",
                     "paper_2605_06408_amd/csrc/vd_internal.h": "77d985737103a5e17fcf0f4b9b37769ea8224b30"},
    "workload": "clustered_1m", "fetch_kib": 54281.5, "write_kib": 1088839.78125, "fetch_scale": 2.0,
    "write_scale": 1.0,
}


def measured_traffic(workload: str):
    """Bytes per launch of the clip kernel, or None if not measured for this
    workload or the kernel changed since."""
    import hashlib
    t = TRAFFIC_MEASURED
    if t["workload"] != workload:
        return None
    for rel, sha in t["sources_sha1"].items():
        with open(os.path.join(ROOT, rel), "rb") as f:
            if hashlib.sha1(f.read()).hexdigest() != sha:
                return None
    return 1024.0 * (t["fetch_kib"] * t["fetch_scale"] + t["write_kib"] * t["write_scale"])


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="clustered_1m",
                    help="uniform_10k | clustered_1m | power_uniform_1m | surface_20m | power_clustered_1m, "
                         "or one of the paper's sets, paper_{uniform,gradient,clusters5,clusters10}[_w]_{1m,15m}")
    ap.add_argument("--n", type=int, default=None, help="override the site count")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--precision", type=int, default=1, help="1 fp32, 2 mixed fp32/fp64")
    ap.add_argument("--leaf-size", type=int, default=0)
    ap.add_argument("--culling", type=int, default=3)
    ap.add_argument("--traversal", type=int, default=1)
    ap.add_argument("--warm-start", type=int, default=0, help="K of the KNN warm start (0: none)")
    ap.add_argument("--weight-ratio", type=float, default=None,
                    help="replace the weights by w ~ N(0, (ratio * d_nn)^2), d_nn the median "
                         "nearest-neighbour distance (the paper's weight sweep)")
    ap.add_argument("--no-cpu-baseline", action="store_true", help="skip the oracle (baseline and error tables)")
    ap.add_argument("--no-extra", action="store_true",
                    help="only the headline workload: skip the other legs and the peak calibration")
    ap.add_argument("--leg-steps", type=int, default=None,
                    help="timed steps of the other legs (default: --steps, at most 10 on the 20M workload)")
    ap.add_argument("--bwd-config", default="power_clustered_1m",
                    help="workload of the fwd+bwd leg (differentiable power diagram)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target CPU time of the oracle sample")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run one plain 256 MiB device copy (reference for HBM byte counters)")
    return ap.parse_args()


def log(msg: str):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def w_alg(ctr: dict) -> float:
    """Algorithmic lane operations of a set of work counters."""
    return float(sum(ctr[k] * c for k, c in W_COST.items()))


def output_bytes(sz: dict) -> float:
    """Exact bytes of every output array of vd_write."""
    n = sz["n"]
    return float(24 * (n + 1) + 4 * sz["n_nbr"] + 4 * sz["n_facet"] + 8 * (sz["n_facet"] + 1) + 4 * sz["n_fv"]
                 + 24 * sz["n_vert"] + 17 * n)


def b_alg(sz: dict, leaf: int) -> float:
    n = sz["n"]
    return float(16 * n + 24 * n + 32 * (2 * n / leaf)) + output_bytes(sz)


def timed(step, steps: int, warmup: int) -> float:
    """Mean milliseconds of `step` over `steps` runs after `warmup` runs,
    bracketed by device synchronisation."""
    import torch
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1000.0 / steps


def run_leg(name, xyz, w, box, kw, steps, warmup, label, verbose=False):
    """Time full steps (build + write) of one workload; the per-phase HIP-event
    times come from the same steps, the work counters from one untimed
    counting build.  Returns the leg's report and its context."""
    import numpy as np
    import torch
    import paper_2605_06408_amd as vd
    n = len(xyz)
    dev = torch.device("cuda", 0)
    tx = torch.from_numpy(xyz).to(dev)
    tw = None if w is None else torch.from_numpy(w).to(dev)
    bbox = [float(v) for v in box]
    ctx = vd.Context(0)

    def step(profile=False, counters=False):
        sz = ctx.build_sizes(tx, tw, bbox, profile=profile, counters=counters, **kw)
        return ctx.write(sz)

    step(counters=True)  # counting adds scalar work: never timed
    torch.cuda.synchronize()
    ctr = ctx.counters()
    for _ in range(warmup):
        step(profile=True)
    torch.cuda.synchronize()
    phases = {k: 0.0 for k in vd.PHASES}
    clip_ms = []
    t0 = time.perf_counter()
    for k in range(steps):
        d = step(profile=True)
        tm = ctx.timings()
        if verbose:
            log("%s step %d: %.1f ms build" % (label, k, tm["build"]))
        clip_ms.append(tm["clip"])
        for q in phases:
            phases[q] += tm[q] / steps
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1000.0 / steps
    sizes = dict(d.sizes)
    leaf = kw.get("leaf_size") or 32
    # dominant kernel: the 64-vertex pass, priced with its own counters
    k_ms = float(np.mean(clip_ms))
    wk = w_alg(ctr["tier0"])
    kernel = {"kernel": "k_clip<1, 4, ...> (64-vertex pass)", "kernel_ms": k_ms, "w_alg": wk,
              "achieved_Tops": wk / (k_ms * 1e-3) / 1e12, "frac": wk / (k_ms * 1e-3) / 1e12 / P_VALU_TOPS}
    # whole step
    W = w_alg(ctr["total"])
    B = b_alg(sizes, leaf)
    t_valu, t_hbm = W / (P_VALU_TOPS * 1e12) * 1e3, B / (PEAK_HBM_GBS * 1e9) * 1e3
    rep = {"workload": name, "n": n, "value": n / (ms / 1000.0), "unit": "cells/s", "ms_per_step": ms,
           "kernel_ms_build": phases["build"], "phases_ms": phases,
           "step_roofline": {"w_alg": W, "b_alg": B, "t_valu_ms": t_valu, "t_hbm_ms": t_hbm,
                             "bound": "valu" if t_valu >= t_hbm else "hbm",
                             "frac": max(t_valu, t_hbm) / ms},
           "dominant_kernel": kernel, "counters": ctr, "sizes": sizes,
           "empty_frac": sizes["n_empty"] / n}
    fp = ctr["total"]
    if fp["classify"]:
        rep["fp64_side_test_frac"] = fp["fp64_test"] / fp["classify"]
    return rep, ctx, (tx, tw, bbox)


def fwd_bwd_leg(config: str, seed: int, kw, steps, warmup) -> dict:
    """One training step of the differentiable power diagram: forward
    (build + volumes/centroids/vertices), the loss
    L = sum_i (V_i - |B|/n)^2 + |c_i - p_i|^2 and its hand-written backward to
    positions and weights."""
    import numpy as np
    import torch
    import paper_2605_06408_amd as vd
    from paper_2605_06408_amd import workloads as wl
    xyz, w, box = wl.make(config, seed)
    n = len(xyz)
    bvol = float(np.prod(np.asarray(box[3:]) - np.asarray(box[:3])))
    x = torch.from_numpy(xyz).cuda().requires_grad_(True)
    ww = torch.from_numpy(w).cuda().requires_grad_(True)
    ctx = vd.Context(0)
    bbox = [float(v) for v in box]

    def fwd():
        return vd.power_diagram(x, ww, bbox=bbox, context=ctx, **kw)

    def step():
        x.grad = None
        ww.grad = None
        d = fwd()
        loss = ((d.vol - bvol / n) ** 2).sum() + ((d.centroid - x) ** 2).sum()
        loss.backward()

    ms_fwd = timed(lambda: fwd(), steps, warmup)
    ms = timed(step, steps, warmup)
    d = fwd()
    loss = ((d.vol - bvol / n) ** 2).sum() + ((d.centroid - x) ** 2).sum()
    loss.backward()
    torch.cuda.synchronize()
    tm = ctx.timings() if kw.get("profile") else {}
    out = {"workload": config, "n": n, "value": n / (ms / 1000.0), "unit": "cells/s", "ms_per_step": ms,
           "fwd_ms": ms_fwd, "fwd_value": n / (ms_fwd / 1000.0), "bwd_kernel_ms": tm.get("backward"),
           "empty_frac": ctx.last_sizes["n_empty"] / n, "dtype": "f32 in, f64 per-cell arithmetic"}
    ctx.close()
    return out


# ------------------------------------------------------------------ oracle

def _oracle_sample(xyz, w, box, m, rng, threads):
    import numpy as np
    import oracle
    ids = np.sort(rng.choice(len(xyz), min(m, len(xyz)), replace=False))
    t0 = time.perf_counter()
    res = oracle.cells(xyz, w, box, ids=ids, threads=threads, margin=True)
    return ids, res, time.perf_counter() - t0


def _error_table(d, res, ids, tau):
    """Per form: neighbour mismatches on cells the oracle certifies at tau and
    below it, and p50/p99/max geometry errors on certified non-empty cells
    (vertices matched by their plane-code triples; vertex and centroid errors
    relative to max(|x*|_inf, l), volumes relative, and the vertex error in the
    cell's frame relative to l, with l the cell's diagonal)."""
    import numpy as np
    import torch
    dev = d.vol.device
    tid = torch.as_tensor(ids, device=dev)
    nb_s, nb_e = d.nbr_off[tid].cpu().numpy(), d.nbr_off[tid + 1].cpu().numpy()
    v_s, v_e = d.vert_off[tid].cpu().numpy(), d.vert_off[tid + 1].cpu().numpy()
    nbr_idx = np.concatenate([np.arange(a, b) for a, b in zip(nb_s, nb_e)] + [np.zeros(0, np.int64)])
    v_idx = np.concatenate([np.arange(a, b) for a, b in zip(v_s, v_e)] + [np.zeros(0, np.int64)])
    nbr = d.nbr[torch.as_tensor(nbr_idx, device=dev)].cpu().numpy()
    vert = d.vert[torch.as_tensor(v_idx, device=dev)].cpu().numpy().astype(np.float64)
    vpl = d.vert_planes[torch.as_tensor(v_idx, device=dev)].cpu().numpy()
    vol = d.vol[tid].cpu().numpy().astype(np.float64)
    cen = d.centroid[tid].cpu().numpy().astype(np.float64)
    nb_o = np.concatenate([[0], np.cumsum(nb_e - nb_s)])
    v_o = np.concatenate([[0], np.cumsum(v_e - v_s)])
    cert = res["margin"] >= tau
    mism_c = mism_u = 0
    err = {"vert": [], "vert_local": [], "vol": [], "cen": []}
    for t in range(len(ids)):
        g_nb = nbr[nb_o[t]:nb_o[t + 1]].tolist()
        o_nb = res["nbr"][res["nbr_off"][t]:res["nbr_off"][t + 1]].tolist()
        gk = {tuple(r): vert[v_o[t] + q] for q, r in enumerate(vpl[v_o[t]:v_o[t + 1]].tolist())}
        ok = {tuple(r): res["vert"][res["vert_off"][t] + q]
              for q, r in enumerate(res["vert_code"][res["vert_off"][t]:res["vert_off"][t + 1]].tolist())}
        same = g_nb == o_nb and set(gk) == set(ok)
        if not cert[t]:
            mism_u += int(not same)
            continue
        mism_c += int(not same)
        if not same or not ok:
            continue
        P = np.array(list(ok.values()))
        ell = float(np.linalg.norm(P.max(0) - P.min(0)))
        dv = max(float(np.max(np.abs(gk[k] - ok[k]))) for k in ok)
        err["vert"].append(max(float(np.max(np.abs(gk[k] - ok[k]))) / max(float(np.max(np.abs(ok[k]))), ell)
                               for k in ok))
        err["vert_local"].append(dv / ell)
        err["vol"].append(abs(vol[t] - res["vol"][t]) / res["vol"][t])
        c_ref = res["centroid"][t]
        err["cen"].append(float(np.max(np.abs(cen[t] - c_ref))) / max(float(np.max(np.abs(c_ref))), ell))
    table = {k: ([float(np.quantile(v, 0.5)), float(np.quantile(v, 0.99)), float(np.max(v))] if v else None)
             for k, v in err.items()}
    return {"gate_tau": tau, "cells": len(ids), "certified": int(cert.sum()), "certified_mismatch": mism_c,
            "uncertified": int((~cert).sum()), "uncertified_mismatch": mism_u,
            "errors_p50_p99_max": table}


def cpu_baseline_and_errors(main, legs, seconds):
    """The oracle timed on the host on a sample of the headline workload
    (k-d tree candidates, no margins, every host thread); then the same cells
    with margins as the reference of the error tables of both forms, and a
    sample of the 20M workload likewise."""
    import numpy as np
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or (os.cpu_count() or 1)
    xyz, w, box = main["inputs"]
    n = len(xyz)
    rng = np.random.default_rng(12345)
    # calibrate on growing samples until one takes >= 1 s, then size the
    # measured sample for about `seconds` of work
    m0 = min(n, 64 * threads)
    while True:
        ids = np.sort(rng.choice(n, m0, replace=False))
        t0 = time.perf_counter()
        oracle.cells(xyz, w, box, ids=ids, threads=threads, margin=False)
        dt = time.perf_counter() - t0
        if dt >= 1.0 or m0 >= n:
            break
        m0 = min(n, m0 * 4)
    m = int(min(n, max(m0, m0 / max(dt, 1e-9) * seconds)))
    ids = np.sort(rng.choice(n, m, replace=False))
    t0 = time.perf_counter()
    oracle.cells(xyz, w, box, ids=ids, threads=threads, margin=False)
    dt = time.perf_counter() - t0
    base = {"value": m / dt, "unit": "cells/s", "cores": threads, "kind": "oracle",
            "sample": "%d random cells of the %d-site %s workload (includes the k-d tree build), FP64 oracle "
                      "with k-d tree candidates, no robustness margins, %.1f s" % (m, n, main["name"], dt)}
    errors = {}
    for leg in [main] + legs:
        if "diagrams" not in leg:
            continue
        lx, lw, lbox = leg["inputs"]
        k = 4000 if len(lx) <= 2_000_000 else 2000
        sids, res, _ = _oracle_sample(lx, lw, lbox, k, np.random.default_rng(7), threads)
        errors[leg["name"]] = {form: _error_table(dg, res, sids, 1e-5 if form == "fp32" else 1e-10)
                               for form, dg in leg["diagrams"].items()}
    return base, errors


# ------------------------------------------------------------------ main

def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only; --gpus %d is not supported" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2605_06408_amd as vd
    from paper_2605_06408_amd import workloads as wl

    log("generating %s" % args.config)
    xyz, w, box = wl.make(args.config, args.seed, args.n)
    if args.weight_ratio is not None:
        w = wl.ratio_weights(xyz, args.seed, args.weight_ratio)
    n = len(xyz)
    log("generated n=%d" % n)
    if args.copy_calibration:
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    kw = dict(precision=args.precision, leaf_size=args.leaf_size, culling=args.culling, traversal=args.traversal,
              warm_start=args.warm_start)
    rep, ctx, (tx, tw, bbox) = run_leg(args.config, xyz, w, box, kw, args.steps, args.warmup, "headline", True)
    ms = rep["ms_per_step"]
    k = rep["dominant_kernel"]
    roofline = {"bound": "alu", "achieved": k["achieved_Tops"], "peak": P_VALU_TOPS, "unit": "TFLOP/s",
                "frac": k["frac"], "traffic": measured_traffic(args.config), "kernel": k["kernel"],
                "kernel_ms": k["kernel_ms"], "w_alg_per_launch": k["w_alg"],
                "op_count": "lane operations of the FP32 vector units, FMA = 1: W_alg = 4 N_cls + 36 N_vnew + "
                            "30 N_node + 15 N_site + 16 N_fin; peak 256 CU x 64 lanes x 2.4 GHz"}
    out = {
        "metric": METRIC, "value": rep["value"], "unit": "cells/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": args.config, "n": n, "seed": args.seed, "box": bbox,
                   "weights": w is not None, "precision": "fp32" if args.precision == 1 else "mixed fp32/fp64",
                   "weight_ratio": args.weight_ratio,
                   "leaf_size": args.leaf_size or 32, "culling": args.culling, "traversal": args.traversal,
                   "warm_start": args.warm_start},
        "roofline": roofline,
        "step_roofline": rep["step_roofline"],
        "phases_ms": rep["phases_ms"],
        "counters": rep["counters"],
        "sizes": rep["sizes"],
    }
    main_leg = {"name": args.config, "inputs": (xyz, w, box)}
    legs = []
    if not args.no_extra:
        out["peaks_measured"] = vd.measure_peaks()
        log("peaks %s" % out["peaks_measured"])
        st = args.leg_steps or args.steps
        wu = min(args.warmup, 3)
        # mixed form on the headline workload, then keep one diagram per form
        log("mixed-precision leg (%s)" % args.config)
        mrep, mctx, _ = run_leg(args.config, xyz, w, box, dict(kw, precision=2), st, wu, "mixed")
        out["mixed"] = {k2: mrep[k2] for k2 in ("value", "ms_per_step", "kernel_ms_build", "step_roofline",
                                                "dominant_kernel", "fp64_side_test_frac")}
        out["mixed"]["cells_with_fp64"] = mrep["sizes"]["n_fp64"]
        out["mixed"]["uncertain"] = mrep["sizes"]["n_uncertain"]
        if args.precision == 1 and not args.no_cpu_baseline:
            main_leg["diagrams"] = {"fp32": ctx.build(tx, tw, bbox, **kw),
                                    "mixed": mctx.build(tx, tw, bbox, **dict(kw, precision=2))}
        del mctx
        # the symbolic perturbation of exact ties (mixed signs plus the checked
        # exact evaluation) on the same workload
        log("perturbed leg (%s)" % args.config)
        prep, _, _ = run_leg(args.config, xyz, w, box, dict(kw, perturb=1), st, wu, "perturbed")
        out["perturbed"] = {k2: prep[k2] for k2 in ("value", "ms_per_step", "kernel_ms_build")}
        out["perturbed"]["cells_perturbed"] = prep["sizes"]["n_perturbed"]
        out["legs"] = {}
        for name in ("surface_20m", "power_uniform_1m"):
            log("leg %s" % name)
            lx, lw, lbox = wl.make(name, args.seed)
            s2 = min(st, 10) if len(lx) > 2_000_000 else st
            lrep, lctx, (ltx, ltw, lbb) = run_leg(name, lx, lw, lbox, dict(kw, precision=1), s2, wu, name, True)
            mrep2, mctx2, _ = run_leg(name, lx, lw, lbox, dict(kw, precision=2), s2, wu, name + " mixed")
            lrep.pop("counters")
            lrep["mixed"] = {k2: mrep2[k2] for k2 in ("value", "ms_per_step", "kernel_ms_build",
                                                      "fp64_side_test_frac")}
            lrep["mixed"]["cells_with_fp64"] = mrep2["sizes"]["n_fp64"]
            lrep["mixed"]["uncertain"] = mrep2["sizes"]["n_uncertain"]
            out["legs"][name] = lrep
            if not args.no_cpu_baseline:
                leg = {"name": name, "inputs": (lx, lw, lbox),
                       "diagrams": {"fp32": lctx.build(ltx, ltw, lbb, precision=1),
                                    "mixed": mctx2.build(ltx, ltw, lbb, precision=2)}}
                legs.append(leg)
            del lctx, mctx2
        log("fwd+bwd leg (%s)" % args.bwd_config)
        out["fwd_bwd"] = fwd_bwd_leg(args.bwd_config, args.seed, dict(kw, profile=True), st, wu)
    if not args.no_cpu_baseline:
        log("cpu baseline and error tables")
        out["cpu_baseline"], errs = cpu_baseline_and_errors(main_leg, legs, args.cpu_seconds)
        if errs:
            out["error_tables"] = errs
        import platform
        cpu = ""
        try:
            with open("/proc/cpuinfo") as f:
                cpu = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), "")
        except OSError:
            pass
        out["cpu_baseline"]["cpu_model"] = cpu or platform.processor()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
