"""Seeded synthetic site sets shaped like the paper's workloads.

This module only draws random numbers; it holds none of the diagram
arithmetic, so both the GPU path's tests and the CPU oracle may use it.
Every generator draws in FP64 with ``numpy.random.default_rng(seed)`` (PCG64)
and casts to FP32 at the end.  Each returns ``(xyz f32[n,3], w f32[n] or
None, box f64[6])`` with box = [xmin, ymin, zmin, xmax, ymax, zmax].

Benchmark workloads (synthetic stand-ins for the distributions the paper
stresses -- uniform, strongly clustered, surface-like and weighted; its
Radiant Foam checkpoints do not ship here):

  uniform            n sites U[0,1]^3, Voronoi, box [0,1]^3
  clustered          10% U[0,1]^3 background + 90% over 64 isotropic Gaussian
                     clusters (centres U[0,1]^3, sigma = 10^U(-4,-1)), each
                     point redrawn until it falls inside [0,1]^3 (truncation)
  power_uniform      U[0,1]^3 with w = r^2, r = s exp(0.75 z), z ~ N(0,1),
                     s = 0.5 n^(-1/3)
  surface            95% on 250 spheres + 250 rectangles (centres U[0,1]^3,
                     size 10^U(log10 0.01, log10 0.3), rectangle sides
                     L x L U(0.25,1), random orientation, points in proportion
                     to area) with N(0, 1e-3^2) normal offset, plus 5% uniform
                     far field in [-4.5, 5.5]^3 (the 10x box); box = that box
  power_clustered    clustered positions (same seed) with the power_uniform
                     weight law at s = 0.005

The paper's own synthetic sets (Sec. 5.1), all in Omega = [-10, 10]^3, box
Omega:

  paper_uniform      p ~ U(Omega)
  paper_clusters     K cluster centres U(Omega), points split evenly over the
                     clusters, N(c, 0.1^2 I), clamped to Omega (K = 5 or 10)
  paper_gradient     density linear in x: x = a + (b - a) sqrt(u), u ~ U(0,1),
                     y, z ~ U(a, b), [a, b] = [-10, 10]
  paper_*_w          the same positions with w ~ N(0, (d_nn^2 / 3)^2), d_nn the
                     median nearest-neighbour distance of the set
"""
from __future__ import annotations

import numpy as np

UNIT_BOX = np.array([0.0, 0.0, 0.0, 1.0, 1.0, 1.0])
BIG_BOX = np.array([-4.5, -4.5, -4.5, 5.5, 5.5, 5.5])


def uniform(n: int, seed: int = 0):
    rng = np.random.default_rng(seed)
    xyz = rng.random((n, 3)).astype(np.float32)
    return xyz, None, UNIT_BOX.copy()


def _truncated_gaussian(rng, centre, sigma, count):
    out = np.empty((count, 3))
    filled = 0
    while filled < count:
        need = count - filled
        pts = rng.normal(centre, sigma, size=(need, 3))
        ok = np.all((pts >= 0.0) & (pts <= 1.0), axis=1)
        pts = pts[ok]
        out[filled:filled + len(pts)] = pts
        filled += len(pts)
    return out


def clustered_positions(n: int, seed: int = 0, n_clusters: int = 64, background: float = 0.1):
    rng = np.random.default_rng(seed)
    n_bg = int(round(background * n))
    n_cl = n - n_bg
    bg = rng.random((n_bg, 3))
    centres = rng.random((n_clusters, 3))
    sigmas = 10.0 ** rng.uniform(-4.0, -1.0, size=n_clusters)
    base, extra = divmod(n_cl, n_clusters)
    parts = [bg]
    for k in range(n_clusters):
        cnt = base + (1 if k < extra else 0)
        parts.append(_truncated_gaussian(rng, centres[k], sigmas[k], cnt))
    xyz = np.concatenate(parts).astype(np.float32)
    # FP32 rounding may land a point exactly on 1.0 but never outside [0,1]
    return xyz


def clustered(n: int, seed: int = 0):
    return clustered_positions(n, seed), None, UNIT_BOX.copy()


def _lognormal_weights(rng, n: int, s: float):
    z = rng.normal(0.0, 1.0, size=n)
    r = s * np.exp(0.75 * z)
    return (r * r).astype(np.float32)


def power_uniform(n: int, seed: int = 0):
    rng = np.random.default_rng(seed)
    xyz = rng.random((n, 3)).astype(np.float32)
    s = 0.5 * n ** (-1.0 / 3.0)
    return xyz, _lognormal_weights(rng, n, s), UNIT_BOX.copy()


def power_clustered(n: int, seed: int = 0, s: float = 0.005):
    xyz = clustered_positions(n, seed)
    rng = np.random.default_rng(seed + 1_000_003)
    return xyz, _lognormal_weights(rng, n, s), UNIT_BOX.copy()


def _random_rotation(rng):
    q, r = np.linalg.qr(rng.normal(size=(3, 3)))
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def surface(n: int, seed: int = 0, n_shapes: int = 500, far: float = 0.05, offset: float = 1e-3):
    rng = np.random.default_rng(seed)
    n_far = int(round(far * n))
    n_surf = n - n_far
    n_sph = n_shapes // 2
    centres = rng.random((n_shapes, 3))
    size = 10.0 ** rng.uniform(np.log10(0.01), np.log10(0.3), size=n_shapes)
    aspect = rng.uniform(0.25, 1.0, size=n_shapes)
    area = np.where(np.arange(n_shapes) < n_sph, 4.0 * np.pi * size ** 2, size * size * aspect)
    counts = rng.multinomial(n_surf, area / area.sum())
    parts = []
    for k in range(n_shapes):
        c = counts[k]
        if c == 0:
            continue
        if k < n_sph:
            d = rng.normal(size=(c, 3))
            d /= np.linalg.norm(d, axis=1, keepdims=True)
            pts = centres[k] + size[k] * d + rng.normal(0.0, offset, size=(c, 1)) * d
        else:
            rot = _random_rotation(rng)
            u = rng.uniform(-0.5, 0.5, size=c) * size[k]
            v = rng.uniform(-0.5, 0.5, size=c) * size[k] * aspect[k]
            t = rng.normal(0.0, offset, size=c)
            pts = centres[k] + u[:, None] * rot[:, 0] + v[:, None] * rot[:, 1] + t[:, None] * rot[:, 2]
        parts.append(pts)
    parts.append(BIG_BOX[:3] + rng.random((n_far, 3)) * (BIG_BOX[3:] - BIG_BOX[:3]))
    xyz = np.concatenate(parts)
    xyz = xyz[rng.permutation(len(xyz))].astype(np.float32)
    return xyz, None, BIG_BOX.copy()


PAPER_BOX = np.array([-10.0, -10.0, -10.0, 10.0, 10.0, 10.0])


def paper_uniform(n: int, seed: int = 0):
    rng = np.random.default_rng(seed)
    xyz = (-10.0 + 20.0 * rng.random((n, 3))).astype(np.float32)
    return xyz, None, PAPER_BOX.copy()


def paper_clusters(n: int, seed: int = 0, k: int = 10, sigma: float = 0.1):
    rng = np.random.default_rng(seed)
    centres = -10.0 + 20.0 * rng.random((k, 3))
    base, extra = divmod(n, k)
    parts = [rng.normal(centres[j], sigma, size=(base + (1 if j < extra else 0), 3)) for j in range(k)]
    xyz = np.clip(np.concatenate(parts), -10.0, 10.0).astype(np.float32)
    return xyz, None, PAPER_BOX.copy()


def paper_gradient(n: int, seed: int = 0):
    rng = np.random.default_rng(seed)
    a, b = -10.0, 10.0
    x = a + (b - a) * np.sqrt(rng.random(n))
    yz = a + (b - a) * rng.random((n, 2))
    xyz = np.column_stack([x, yz]).astype(np.float32)
    return xyz, None, PAPER_BOX.copy()


def median_nn_distance(xyz) -> float:
    from scipy.spatial import cKDTree
    p = np.asarray(xyz, np.float64)
    d, _ = cKDTree(p).query(p, k=2, workers=-1)
    return float(np.median(d[:, 1]))


def paper_weights(xyz, seed: int = 0):
    """w ~ N(0, (d_nn^2 / 3)^2) with d_nn the median nearest-neighbour
    distance of the (FP32) sites."""
    dnn = median_nn_distance(xyz)
    rng = np.random.default_rng(seed + 2_000_003)
    return rng.normal(0.0, dnn * dnn / 3.0, size=len(xyz)).astype(np.float32)


def ratio_weights(xyz, seed: int, ratio: float):
    """The paper's weight sweep (Sec. 5.2): w ~ N(0, sd^2) with sd the
    median nearest-neighbour distance times `ratio` (taken as stated; ratio 0
    gives w = 0, the Voronoi diagram)."""
    sd = ratio * median_nn_distance(xyz) if ratio else 0.0
    rng = np.random.default_rng(seed + 3_000_017)
    return rng.normal(0.0, sd, size=len(xyz)).astype(np.float32) if sd else np.zeros(len(xyz), np.float32)


def _weighted(gen):
    def fn(n: int, seed: int = 0):
        xyz, _, box = gen(n, seed)
        return xyz, paper_weights(xyz, seed), box
    return fn


def _clusters(k: int):
    return lambda n, seed=0: paper_clusters(n, seed, k)


# The five benchmark configurations at their full sizes, then the paper's
# own synthetic sets at 1M and 15M sites.
CONFIGS = {
    "uniform_10k": (uniform, 10_000),
    "clustered_1m": (clustered, 1_000_000),
    "power_uniform_1m": (power_uniform, 1_000_000),
    "surface_20m": (surface, 20_000_000),
    "power_clustered_1m": (power_clustered, 1_000_000),
}
for _n, _tag in ((1_000_000, "1m"), (15_000_000, "15m")):
    for _name, _gen in (("paper_uniform", paper_uniform), ("paper_gradient", paper_gradient),
                        ("paper_clusters5", _clusters(5)), ("paper_clusters10", _clusters(10))):
        CONFIGS["%s_%s" % (_name, _tag)] = (_gen, _n)
        CONFIGS["%s_w_%s" % (_name, _tag)] = (_weighted(_gen), _n)


def make(name: str, seed: int = 0, n: int | None = None):
    fn, n_full = CONFIGS[name]
    return fn(n_full if n is None else n, seed)
