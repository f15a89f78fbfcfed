"""Throughput of the diagram construction on one MI355X.

One step = one full vd_build + vd_write (LBVH build, traversal and clipping,
prefix sums, CSR write-out of neighbours, facets, vertices, volumes and
centroids) over the whole site set, with the sites already resident in HBM.
Timing follows the paper's protocol (Sec. 5.2: warm-up runs, then the mean
of timed runs), bracketed by device synchronisation.

Prints one JSON line with the metric, the roofline of the dominant kernel
(the 64-vertex traversal+clip kernel, timed by HIP events on the library's
stream) and the CPU oracle timed on a bounded sample of the same workload.
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

# Nominal FP32 flops of one occurrence of each counted work unit (FMA = 2).
# They price the arithmetic the method needs for that unit, not the
# instructions this implementation happens to issue:
#   classify     a.y - b over 3 components and a compare            3 FMA + 1 = 7
#   new_vertex   three cross products (27), determinant (5), the
#                three numerator components (15), reciprocal + scale (4)     = 51
#   node_test    closest point (12), distance and weight bound (6),
#                octant radius (8), two square roots + compare (6)           = 32
#   site_test    difference (3), |a|^2 (5), b (2), octant radius (5),
#                rounding slack and squared compare (10)                     = 25
#   final_vertex three fan tetrahedra: cross (9), dot (5), moment (6) each   = 60
#   ball_test    point-to-box distance (12), vertex power (5), compare (3)  = 20
FLOPS_PER_UNIT = {"classify": 7, "new_vertex": 51, "node_test": 32, "site_test": 25, "final_vertex": 60,
                  "ball_test": 20}
PEAK_FP32_TFLOPS = 157.3   # MI355X FP32 vector peak (256 CUs x 2.4 GHz, packed FMA)
PEAK_HBM_GBS = 8000.0

# HBM traffic of the 64-vertex clip kernel per launch, from two rocprofv3 --pmc
# runs (FETCH_SIZE, WRITE_SIZE; KiB per dispatch) of bench.py on the named
# workload, each scaled by what the same counter reads for a plain 256 MiB
# device copy in the same run (FETCH_SIZE 131088.4 KiB -> x2.0, WRITE_SIZE
# 262144.0 KiB -> x1.0).  Valid only while the kernel source is unchanged.
TRAFFIC_MEASURED = {
    "sources_sha1": {"paper_2605_06408_amd/csrc/vd_clip.hip": "b002ce06ce6aedbf6e1e279cbc3d4818812120b1",
                     "paper_2605_06408_amd/csrc/vd_internal.h": "661a515ca8e5fede4dd2562752156d51cabc0bc5"},
    "workload": "clustered_1m", "fetch_kib": 28098.6, "write_kib": 896496.9, "fetch_scale": 2.0, "write_scale": 1.0,
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
    ap = argparse.ArgumentParser(description=__doc__)
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
    ap.add_argument("--weight-ratio", type=float, default=None,
                    help="replace the weights by w ~ N(0, (ratio * d_nn)^2), d_nn the median "
                         "nearest-neighbour distance (the paper's weight sweep)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the mixed-precision and fwd+bwd legs")
    ap.add_argument("--bwd-config", default="power_clustered_1m",
                    help="workload of the fwd+bwd leg (differentiable power diagram)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target CPU time of the oracle sample")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run one plain 256 MiB device copy (reference for HBM byte counters)")
    return ap.parse_args()


def cpu_baseline(xyz, w, box, seconds: float) -> dict:
    """The CPU oracle (FP64 brute-force clipper, all host threads) on a random
    sample of cells of the same workload; scaled to cells per second."""
    import numpy as np
    import oracle
    n = len(xyz)
    rng = np.random.default_rng(12345)
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or (os.cpu_count() or 1)
    # calibrate on growing samples until one takes >= 1 s, then size the
    # measured sample for about `seconds` of work
    m0 = min(n, 16 * threads)
    while True:
        ids = np.sort(rng.choice(n, m0, replace=False))
        t0 = time.perf_counter()
        oracle.cells(xyz, w, box, ids=ids, threads=threads)
        dt = time.perf_counter() - t0
        if dt >= 1.0 or m0 >= n:
            break
        m0 = min(n, m0 * 4)
    rate = m0 / max(dt, 1e-9)
    m = int(min(n, max(m0, rate * seconds)))
    ids = np.sort(rng.choice(n, m, replace=False))
    t0 = time.perf_counter()
    oracle.cells(xyz, w, box, ids=ids, threads=threads)
    dt = time.perf_counter() - t0
    return {"value": m / dt, "unit": "cells/s", "cores": threads, "kind": "oracle",
            "sample": "%d random cells of the same %d-site workload, FP64 oracle with robustness margins, %.1f s"
                      % (m, n, dt)}


def log(msg: str):
    print("[bench] " + msg, file=sys.stderr, flush=True)


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


def mixed_leg(ctx, tx, tw, bbox, kw, steps, warmup) -> dict:
    """The same workload with mixed FP32/FP64 predicates."""
    kw2 = dict(kw, precision=2)

    def step():
        ctx.write(ctx.build_sizes(tx, tw, bbox, **kw2))

    ms = timed(step, steps, warmup)
    sz = ctx.last_sizes
    return {"value": tx.shape[0] / (ms / 1000.0), "unit": "cells/s", "ms_per_step": ms,
            "precision": "mixed fp32/fp64", "cells_with_fp64": sz["n_fp64"], "uncertain": sz["n_uncertain"]}


def fwd_bwd_leg(config: str, seed: int, kw, steps, warmup) -> dict:
    import numpy as np
    """One training step of the differentiable power diagram: forward
    (build + volumes/centroids/vertices), the loss
    L = sum_i (V_i - |B|/n)^2 + |c_i - p_i|^2 and its hand-written backward to
    positions and weights."""
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
    return {"workload": config, "n": n, "value": n / (ms / 1000.0), "unit": "cells/s", "ms_per_step": ms,
            "fwd_ms": ms_fwd, "fwd_value": n / (ms_fwd / 1000.0), "bwd_kernel_ms": tm.get("backward"),
            "empty_cells": ctx.last_sizes["n_empty"], "dtype": "f32 in, f64 per-cell arithmetic"}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only; --gpus %d is not supported" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
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
    dev = torch.device("cuda", 0)
    tx = torch.from_numpy(xyz).to(dev)
    tw = None if w is None else torch.from_numpy(w).to(dev)
    bbox = [float(v) for v in box]
    ctx = vd.Context(0)
    kw = dict(precision=args.precision, leaf_size=args.leaf_size, culling=args.culling, traversal=args.traversal)

    def step(profile=False, counters=False):
        sz = ctx.build_sizes(tx, tw, bbox, profile=profile, counters=counters, **kw)
        return ctx.write(sz)

    # work counters from one untimed build (counting adds scalar work)
    step(counters=True)
    torch.cuda.synchronize()
    ctr = ctx.counters()
    log("counted build done")
    for _ in range(args.warmup):
        d = step(profile=True)
    torch.cuda.synchronize()
    clip_ms, phases = [], {k: 0.0 for k in vd.PHASES}
    t0 = time.perf_counter()
    for k in range(args.steps):
        d = step(profile=True)
        tm = ctx.timings()
        log("step %d: %.1f ms build" % (k, tm["build"]))
        clip_ms.append(tm["clip"])
        for k in phases:
            phases[k] += tm[k] / args.steps
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1000.0 / args.steps
    sizes = d.sizes

    # the roofline prices the 64-vertex kernel alone, with its own counters
    flops = sum(ctr["tier0"][k] * FLOPS_PER_UNIT[k] for k in FLOPS_PER_UNIT)
    clip_s = float(np.mean(clip_ms)) / 1000.0
    achieved = flops / clip_s / 1e12
    traffic = measured_traffic(args.config)
    roofline = {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / PEAK_FP32_TFLOPS, "traffic": traffic,
                "kernel": "k_clip<1,4,false> (64-vertex pass)", "kernel_ms": clip_s * 1000.0,
                "flops_per_launch": flops}

    out = {
        "metric": METRIC, "value": n / (ms / 1000.0), "unit": "cells/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": args.config, "n": n, "seed": args.seed, "box": bbox,
                   "weights": w is not None, "precision": "fp32" if args.precision == 1 else "mixed fp32/fp64",
                   "weight_ratio": args.weight_ratio,
                   "leaf_size": args.leaf_size or 32, "culling": args.culling, "traversal": args.traversal},
        "roofline": roofline,
        "phases_ms": phases,
        "counters": ctr,
        "sizes": sizes,
    }
    if not args.no_extra:
        log("mixed-precision leg")
        out["mixed"] = mixed_leg(ctx, tx, tw, bbox, kw, args.steps, args.warmup)
        log("fwd+bwd leg (%s)" % args.bwd_config)
        out["fwd_bwd"] = fwd_bwd_leg(args.bwd_config, args.seed, dict(kw, profile=True), args.steps, args.warmup)
    if not args.no_cpu_baseline:
        log("cpu baseline")
        out["cpu_baseline"] = cpu_baseline(xyz, w, box, args.cpu_seconds)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
