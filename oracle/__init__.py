"""CPU oracle for 3D Voronoi / power cells -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product path (the HIP library and
its Python binding) never imports it and shares no code with it.

``cells()`` wraps ``liboracle.so`` (``vd_oracle.cpp``: FP64 clipping of the
cell definition, paper Sec. 3 Eq. 1 and Sec. 4.1, with candidates in
increasing plane distance from brute force or a k-d tree).
``brute`` holds an exact-rational vertex enumeration used to pin the C++
oracle on tiny inputs.  ``tetrahedra()`` reads the dual (regular / Delaunay)
tetrahedra off the cells.

Output layout (canonical, per requested cell, CSR over the requested cells):
  nbr_off/nbr          neighbour site ids, ascending
  vert_off/vert        vertex positions (FP64, global coordinates)
  vert_code            the 3 plane codes of each vertex, ascending; a code is a
                       site id (>= 0) or a box face -1..-6 =
                       x_min, x_max, y_min, y_max, z_min, z_max
                       (vertices of a cell are sorted by that triple)
  facet_off/facet_code facets of each cell, ascending code
  fv_off/fv            each facet's vertices (cell-local indices), CCW seen
                       from outside, starting at the smallest index
  vol, centroid        FP64
  flags                1 empty, 2 degenerate (not in general position),
                       4 coincident sites involved
  margin               robustness margin (0 for degenerate cells, capped 1e-3)
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "vd_oracle.cpp")

FLAG_EMPTY = 1
FLAG_DEGENERATE = 2
FLAG_COINCIDENT = 4

_lib = None


def build(force: bool = True) -> str:
    """Compile liboracle.so with g++ (OpenMP)."""
    if force or not os.path.exists(_LIB_PATH):
        cmd = ["g++", "-O2", "-std=c++17", "-fopenmp", "-fPIC", "-shared", "-o", _LIB_PATH, _SRC]
        subprocess.run(cmd, check=True)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        lib.orc_run.restype = P
        lib.orc_run.argtypes = [P, P, ctypes.c_int64, P, P, ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.c_int]
        lib.orc_run64.restype = P
        lib.orc_run64.argtypes = [P, P, ctypes.c_int64, P, P, ctypes.c_int64, ctypes.c_int, ctypes.c_int,
                                  ctypes.c_int]
        lib.orc_session_open.restype = P
        lib.orc_session_open.argtypes = [P, P, ctypes.c_int64, P, ctypes.c_int, ctypes.c_int]
        lib.orc_session_cells.restype = P
        lib.orc_session_cells.argtypes = [P, P, ctypes.c_int64, ctypes.c_int, ctypes.c_int64, P]
        lib.orc_session_close.restype = None
        lib.orc_session_close.argtypes = [P]
        lib.orc_sizes.restype = None
        lib.orc_sizes.argtypes = [P, P]
        lib.orc_fetch.restype = None
        lib.orc_fetch.argtypes = [P] * 14
        lib.orc_free.restype = None
        lib.orc_free.argtypes = [P]
        _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def default_box(xyz: np.ndarray) -> np.ndarray:
    """AABB of the sites (FP32 values widened to FP64)."""
    x = np.asarray(xyz, dtype=np.float32)
    return np.concatenate([x.min(axis=0), x.max(axis=0)]).astype(np.float64)


CANDIDATES = {"auto": 0, "brute": 1, "kdtree": 2}


def cells(xyz, w=None, box=None, ids=None, margin: bool = True, threads: int = 0, fp64: bool = False,
          candidates: str = "auto") -> dict:
    """Compute the cells ``ids`` (default: all) of the power diagram of
    (xyz, w) clipped to ``box`` = [xmin, ymin, zmin, xmax, ymax, zmax].

    By default sites, weights and box are FP32 values (as the library takes
    them).  ``fp64=True`` takes all three as FP64 values instead (finite
    differences perturb inputs below FP32 resolution).  ``candidates``:
    "brute" (every site), "kdtree" (best-first k-d tree walk) or "auto"
    (brute force up to 20000 sites); both give bit-identical results."""
    lib = _load()
    dt = np.float64 if fp64 else np.float32
    xyz = np.ascontiguousarray(xyz, dtype=dt)
    n = xyz.shape[0]
    if w is not None:
        w = np.ascontiguousarray(w, dtype=dt)
        assert w.shape == (n,)
    if box is None:
        box = np.concatenate([xyz.min(axis=0), xyz.max(axis=0)]).astype(np.float64)
    else:
        # the clip box is an input like the sites: use its value in their precision
        box = np.asarray(box, dtype=dt).astype(np.float64)
    if ids is not None:
        ids = np.ascontiguousarray(ids, dtype=np.int64)
        m = ids.shape[0]
    else:
        m = n
    run = lib.orc_run64 if fp64 else lib.orc_run
    h = run(_ptr(xyz), _ptr(w), n, _ptr(box), _ptr(ids), m, int(margin), int(threads), CANDIDATES[candidates])
    return _fetch(h, m, n, ids)


def _fetch(h, m, n, ids):
    """Copy a result handle into numpy arrays and free it."""
    lib = _load()
    if not h:
        raise ValueError("oracle rejected its input")
    try:
        tot = np.zeros(4, dtype=np.int64)
        lib.orc_sizes(h, _ptr(tot))
        out = dict(
            nbr_off=np.zeros(m + 1, np.int64), nbr=np.zeros(tot[0], np.int64),
            vert_off=np.zeros(m + 1, np.int64), vert=np.zeros((tot[1], 3), np.float64),
            vert_code=np.zeros((tot[1], 3), np.int64),
            facet_off=np.zeros(m + 1, np.int64), facet_code=np.zeros(tot[2], np.int64),
            fv_off=np.zeros(tot[2] + 1, np.int64), fv=np.zeros(tot[3], np.int64),
            vol=np.zeros(m, np.float64), centroid=np.zeros((m, 3), np.float64),
            flags=np.zeros(m, np.int32), margin=np.zeros(m, np.float64),
        )
        keys = ["nbr_off", "nbr", "vert_off", "vert", "vert_code", "facet_off", "facet_code",
                "fv_off", "fv", "vol", "centroid", "flags", "margin"]
        lib.orc_fetch(h, *[_ptr(out[k]) for k in keys])
    finally:
        lib.orc_free(h)
    out["ids"] = np.arange(n, dtype=np.int64) if ids is None else ids
    return out


class Session:
    """The oracle over one FP64 input kept across calls (with its k-d tree),
    for finite differences: ``cells(ids, moved=(k, xyz_k, w_k))`` computes
    cells with site k moved (and puts it back).  Results as ``cells()``."""

    def __init__(self, xyz, w=None, box=None, threads: int = 0, candidates: str = "auto"):
        lib = _load()
        self.xyz = np.ascontiguousarray(xyz, dtype=np.float64)
        self.n = self.xyz.shape[0]
        self.w = None if w is None else np.ascontiguousarray(w, dtype=np.float64)
        if box is None:
            box = np.concatenate([self.xyz.min(axis=0), self.xyz.max(axis=0)])
        self.box = np.asarray(box, dtype=np.float64)
        self.h = lib.orc_session_open(_ptr(self.xyz), _ptr(self.w), self.n, _ptr(self.box), int(threads),
                                      CANDIDATES[candidates])
        if not self.h:
            raise ValueError("oracle rejected its input")

    def cells(self, ids, margin: bool = False, moved=None) -> dict:
        ids = np.ascontiguousarray(ids, dtype=np.int64)
        k, mv = -1, None
        if moved is not None:
            k = int(moved[0])
            mv = np.zeros(4, np.float64)
            mv[:3] = moved[1]
            mv[3] = 0.0 if moved[2] is None else float(moved[2])
        h = _load().orc_session_cells(self.h, _ptr(ids), len(ids), int(margin), k, _ptr(mv))
        return _fetch(h, len(ids), self.n, ids)

    def close(self):
        if getattr(self, "h", None):
            _load().orc_session_close(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def tetrahedra(res: dict) -> np.ndarray:
    """Dual tetrahedra listed by the requested cells of a ``cells()`` result
    (paper Sec. 3: the power diagram's dual is the regular triangulation; with
    equal weights the Delaunay tetrahedralisation).  A vertex of cell i whose
    three planes are all site planes j < k < l with j > i is the power centre
    of tetrahedron (i, j, k, l); box-face vertices have no dual tetrahedron.
    Rows [T, 4] int64, sorted."""
    rows = []
    for t, i in enumerate(res["ids"]):
        codes = res["vert_code"][res["vert_off"][t]:res["vert_off"][t + 1]]
        for c in codes:
            if c[0] > i:
                rows.append((int(i), int(c[0]), int(c[1]), int(c[2])))
    out = np.array(sorted(rows), dtype=np.int64)
    return out.reshape(-1, 4)


def cell_view(res: dict, t: int) -> dict:
    """The t-th requested cell of a ``cells()`` result as plain arrays."""
    v0, v1 = res["vert_off"][t], res["vert_off"][t + 1]
    f0, f1 = res["facet_off"][t], res["facet_off"][t + 1]
    facets = []
    for f in range(f0, f1):
        a, b = res["fv_off"][f], res["fv_off"][f + 1]
        facets.append((int(res["facet_code"][f]), res["fv"][a:b].copy()))
    return dict(
        nbr=res["nbr"][res["nbr_off"][t]:res["nbr_off"][t + 1]].copy(),
        vert=res["vert"][v0:v1].copy(), vert_code=res["vert_code"][v0:v1].copy(),
        facets=facets, vol=float(res["vol"][t]), centroid=res["centroid"][t].copy(),
        flags=int(res["flags"][t]), margin=float(res["margin"][t]),
    )
