"""MI355X-native 3D Voronoi and power diagrams (HIP, gfx950).

Thin Python binding of the C ABI in ``include/vd.h`` (``libvd.so``): argument
marshalling only.  PyTorch provides device memory and the current stream;
every step of the construction runs in the library's HIP kernels.  If the
library has not been built the calls raise -- there is no fallback path.

    import torch, paper_2605_06408_amd as vd
    d = vd.build(xyz_cuda_f32_nx3, w=None, bbox=[0, 0, 0, 1, 1, 1])
    d.nbr_off, d.nbr, d.vol, d.centroid, ...
"""
from __future__ import annotations

import ctypes
import os
import threading
from collections import namedtuple

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libvd.so")

FLAG_EMPTY = 1
FLAG_FP64 = 2
FLAG_LARGE = 4
FLAG_UNCERTAIN = 8
FLAG_FAILED = 16
FLAG_PERTURBED = 32

PRECISION_FP32 = 1
PRECISION_MIXED = 2
CULLING_DIRECTIONAL = 1
CULLING_ISOTROPIC = 2
CULLING_BALLS = 3
TRAVERSAL_BEST_FIRST = 1
TRAVERSAL_DEPTH_FIRST = 2

MAX_SITES = 1 << 25
TIERS = 4  # capacity tiers: 64, 128, 1024, 16384 vertices per cell

PHASES = ("lbvh", "clip", "clip_large", "scan", "build", "write", "clip_tier1", "backward")
COUNTERS = ("classify", "new_vertex", "node_test", "site_test", "final_vertex", "clip", "clip_effective", "leaf",
            "ball_test", "fp64_test", "cycles_traverse", "cycles_leaf", "cycles_clip", "cycles_final")

STATUS = {0: "VD_OK", 1: "VD_ERR_INVALID_ARG", 2: "VD_ERR_HIP", 3: "VD_ERR_OOM", 4: "VD_ERR_STATE",
          5: "VD_ERR_CAPACITY"}


class VDError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s: %s" % (STATUS.get(status, status), msg))
        self.status = status


class Options(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("leaf_size", ctypes.c_int32), ("culling", ctypes.c_int32),
                ("traversal", ctypes.c_int32), ("profile", ctypes.c_int32), ("counters", ctypes.c_int32),
                ("warm_start", ctypes.c_int32), ("perturb", ctypes.c_int32)]


class Sizes(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in ("n", "n_nbr", "n_facet", "n_vert", "n_fv", "n_empty", "n_large",
                                               "n_uncertain", "n_failed", "n_fp64", "n_huge",
                                               "n_resumed", "n_perturbed")]

    def as_dict(self) -> dict:
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


OUTPUT_FIELDS = ("nbr_off", "nbr", "facet_off", "facet_nbr", "fv_off", "fv", "vert_off", "vert", "vert_planes",
                 "vol", "centroid", "flags")


class Outputs(ctypes.Structure):
    _fields_ = [(k, ctypes.c_void_p) for k in OUTPUT_FIELDS]


Diagram = namedtuple("Diagram", OUTPUT_FIELDS + ("sizes",))

_lib = None
_lib_lock = threading.Lock()


def library_path() -> str:
    return LIB_PATH


def load_library():
    """Load libvd.so; raises if it is missing (build it with ``build_library``)."""
    global _lib
    with _lib_lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError("libvd.so is not built (%s); run paper_2605_06408_amd.build_library()" % LIB_PATH)
            lib = ctypes.CDLL(LIB_PATH)
            P = ctypes.c_void_p
            lib.vd_create.restype = ctypes.c_int
            lib.vd_create.argtypes = [ctypes.c_int, ctypes.POINTER(P)]
            lib.vd_destroy.restype = None
            lib.vd_destroy.argtypes = [P]
            lib.vd_build.restype = ctypes.c_int
            lib.vd_build.argtypes = [P, P, P, ctypes.c_int64, P, ctypes.POINTER(Options), P, ctypes.POINTER(Sizes)]
            lib.vd_write.restype = ctypes.c_int
            lib.vd_write.argtypes = [P, ctypes.POINTER(Outputs), P]
            lib.vd_get_sizes.restype = ctypes.c_int
            lib.vd_get_sizes.argtypes = [P, ctypes.POINTER(Sizes)]
            lib.vd_last_error.restype = ctypes.c_char_p
            lib.vd_last_error.argtypes = []
            lib.vd_version.restype = ctypes.c_char_p
            lib.vd_version.argtypes = []
            lib.vd_get_timings.restype = ctypes.c_int
            lib.vd_get_timings.argtypes = [P, ctypes.POINTER(ctypes.c_float), ctypes.c_int32]
            lib.vd_get_counters.restype = ctypes.c_int
            lib.vd_get_counters.argtypes = [P, ctypes.POINTER(ctypes.c_uint64), ctypes.c_int32]
            lib.vd_backward.restype = ctypes.c_int
            lib.vd_backward.argtypes = [P, P, P, P, P, P, P]
            lib.vd_backward_noalloc.restype = ctypes.c_int
            lib.vd_backward_noalloc.argtypes = [P, P, P, P, P, P, P]
            lib.vd_inspect_bvh.restype = ctypes.c_int
            lib.vd_inspect_bvh.argtypes = [P, P, P, P, P, P, ctypes.POINTER(ctypes.c_uint32), P]
            lib.vd_measure_peaks.restype = ctypes.c_int
            lib.vd_measure_peaks.argtypes = [ctypes.c_int, P, ctypes.POINTER(ctypes.c_double),
                                             ctypes.POINTER(ctypes.c_double)]
            lib.vd_tetrahedra.restype = ctypes.c_int
            lib.vd_tetrahedra.argtypes = [P, P, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64), P]
            _lib = lib
    return _lib


def build_library(verbose: bool = False) -> str:
    from . import buildlib
    return buildlib.build(verbose=verbose)


def _check(status: int, what: str):
    if status != 0:
        raise VDError(status, "%s: %s" % (what, load_library().vd_last_error().decode()))


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


class Context:
    """Owns a libvd context (device scratch reused across builds)."""

    def __init__(self, device=None):
        import torch
        self.lib = load_library()
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else torch.device(device).index or 0)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(self.lib.vd_create(self.device.index, ctypes.byref(h)), "vd_create")
        self.handle = h
        self.generation = 0  # counts builds: a backward needs the build it follows

    def close(self):
        if getattr(self, "handle", None):
            self.lib.vd_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def build_sizes(self, xyz, w=None, bbox=None, precision=PRECISION_FP32, leaf_size=0,
                    culling=CULLING_BALLS, traversal=TRAVERSAL_BEST_FIRST, allow_failed=False,
                    profile=False, counters=False, warm_start=0, perturb=0) -> Sizes:
        """Run vd_build only (the diagram stays in the context)."""
        import torch
        if not (xyz.is_cuda and xyz.dtype == torch.float32 and xyz.dim() == 2 and xyz.shape[1] == 3):
            raise ValueError("xyz must be a CUDA float32 tensor of shape [n, 3]")
        xyz = xyz.contiguous()
        n = xyz.shape[0]
        if w is not None:
            if not (w.is_cuda and w.dtype == torch.float32 and w.shape == (n,)):
                raise ValueError("w must be a CUDA float32 tensor of shape [n]")
            w = w.contiguous()
        hb = None
        if bbox is not None:
            vals = [float(v) for v in bbox]
            if len(vals) != 6:
                raise ValueError("bbox must have 6 entries")
            hb = (ctypes.c_float * 6)(*vals)
        opt = Options(precision, leaf_size, culling, traversal, int(profile), int(counters), int(warm_start),
                      int(perturb))
        sz = Sizes()
        stream = torch.cuda.current_stream(self.device).cuda_stream
        with torch.cuda.device(self.device):
            st = self.lib.vd_build(self.handle, _ptr(xyz), _ptr(w), n, hb, ctypes.byref(opt),
                                   ctypes.c_void_p(stream), ctypes.byref(sz))
        self.generation += 1
        self.n = n
        self.last_sizes = sz.as_dict()
        if st == 5 and allow_failed:
            return sz
        _check(st, "vd_build")
        self._keep = (xyz, w)
        return sz

    def write(self, sz: Sizes) -> Diagram:
        """Allocate output tensors (torch caching allocator) and fill them."""
        import torch
        dev = self.device
        i64, i32, f32 = torch.int64, torch.int32, torch.float32
        n = sz.n
        t = dict(
            nbr_off=torch.empty(n + 1, dtype=i64, device=dev), nbr=torch.empty(sz.n_nbr, dtype=i32, device=dev),
            facet_off=torch.empty(n + 1, dtype=i64, device=dev),
            facet_nbr=torch.empty(sz.n_facet, dtype=i32, device=dev),
            fv_off=torch.empty(sz.n_facet + 1, dtype=i64, device=dev), fv=torch.empty(sz.n_fv, dtype=i32, device=dev),
            vert_off=torch.empty(n + 1, dtype=i64, device=dev), vert=torch.empty((sz.n_vert, 3), dtype=f32, device=dev),
            vert_planes=torch.empty((sz.n_vert, 3), dtype=i32, device=dev), vol=torch.empty(n, dtype=f32, device=dev),
            centroid=torch.empty((n, 3), dtype=f32, device=dev), flags=torch.empty(n, dtype=torch.uint8, device=dev),
        )
        out = Outputs(*[_ptr(t[k]) for k in OUTPUT_FIELDS])
        stream = torch.cuda.current_stream(dev).cuda_stream
        with torch.cuda.device(dev):
            _check(self.lib.vd_write(self.handle, ctypes.byref(out), ctypes.c_void_p(stream)), "vd_write")
        return Diagram(**t, sizes=sz.as_dict())

    def timings(self) -> dict:
        """Per-phase milliseconds of the last profiled build (and write)."""
        ms = (ctypes.c_float * len(PHASES))()
        _check(self.lib.vd_get_timings(self.handle, ms, len(PHASES)), "vd_get_timings")
        return dict(zip(PHASES, [float(x) for x in ms]))

    def counters(self) -> dict:
        """Work counters of the last build made with counters=True: a dict per
        capacity tier ("tier0" .. "tier3": 64, 128, 1024, 16384 vertices) and
        their sum ("total")."""
        k = len(COUNTERS)
        v = (ctypes.c_uint64 * (TIERS * k))()
        _check(self.lib.vd_get_counters(self.handle, v, TIERS * k), "vd_get_counters")
        vals = [int(x) for x in v]
        out = {"tier%d" % t: dict(zip(COUNTERS, vals[t * k:(t + 1) * k])) for t in range(TIERS)}
        out["total"] = {c: sum(out["tier%d" % t][c] for t in range(TIERS)) for c in COUNTERS}
        return out

    def build(self, xyz, w=None, bbox=None, **kw) -> Diagram:
        sz = self.build_sizes(xyz, w, bbox, **kw)
        return self.write(sz)

    def tetrahedra(self):
        """vd_tetrahedra over the last build: the dual (regular / Delaunay)
        tetrahedra whose power centre lies inside the box, int32 [T, 4], each
        row ascending and rows grouped by their first site."""
        import torch
        dev = self.device
        stream = torch.cuda.current_stream(dev).cuda_stream
        cnt = ctypes.c_int64(0)
        with torch.cuda.device(dev):
            _check(self.lib.vd_tetrahedra(self.handle, None, 0, ctypes.byref(cnt), ctypes.c_void_p(stream)),
                   "vd_tetrahedra")
            tets = torch.empty((cnt.value, 4), dtype=torch.int32, device=dev)
            _check(self.lib.vd_tetrahedra(self.handle, _ptr(tets), cnt.value, ctypes.byref(cnt),
                                          ctypes.c_void_p(stream)), "vd_tetrahedra")
        return tets

    def inspect_bvh(self) -> dict:
        """vd_inspect_bvh over the last build: Morton codes (caller's order),
        sorted codes, Morton order, node records [n-1, 2] of
        (lo xyz, wmax, hi xyz, ref) as int32/float32 views, leaf records and
        the root reference."""
        import torch
        dev = self.device
        n = self.n
        t = dict(morton=torch.empty(n, dtype=torch.int64, device=dev),
                 sorted_keys=torch.empty(n, dtype=torch.int64, device=dev),
                 order=torch.empty(n, dtype=torch.int32, device=dev),
                 nodes=torch.zeros((max(n - 1, 1), 2, 8), dtype=torch.int32, device=dev),
                 leaf_of=torch.zeros(n, dtype=torch.int32, device=dev))
        root = ctypes.c_uint32(0)
        stream = torch.cuda.current_stream(dev).cuda_stream
        with torch.cuda.device(dev):
            _check(self.lib.vd_inspect_bvh(self.handle, _ptr(t["morton"]), _ptr(t["sorted_keys"]), _ptr(t["order"]),
                                           _ptr(t["nodes"]), _ptr(t["leaf_of"]), ctypes.byref(root),
                                           ctypes.c_void_p(stream)), "vd_inspect_bvh")
        torch.cuda.synchronize(dev)
        out = {k: v.cpu().numpy() for k, v in t.items()}
        out["root"] = root.value
        return out

    def backward(self, g_vol=None, g_cen=None, g_vert=None, want_w=True, noalloc=False):
        """vd_backward over the last build: gradients of
        sum g_vol V + g_cen . c + g_vert . x with respect to the sites (and
        weights).  Returns (g_xyz [n, 3], g_w [n] or None).  noalloc=True
        calls vd_backward_noalloc (the library's fixed device scratch; the
        output tensors still come from torch)."""
        import torch
        dev = self.device
        n = self.n

        def arg(t, shape):
            if t is None:
                return None
            if not (t.is_cuda and t.dtype == torch.float32 and tuple(t.shape) == shape):
                raise ValueError("gradient must be a CUDA float32 tensor of shape %s" % (shape,))
            return t.contiguous()

        gv = arg(g_vol, (n,))
        gc = arg(g_cen, (n, 3))
        gx = None if g_vert is None else arg(g_vert, (self.last_sizes["n_vert"], 3))
        g_xyz = torch.empty((n, 3), dtype=torch.float32, device=dev)
        g_w = torch.empty(n, dtype=torch.float32, device=dev) if want_w else None
        stream = torch.cuda.current_stream(dev).cuda_stream
        with torch.cuda.device(dev):
            fn = self.lib.vd_backward_noalloc if noalloc else self.lib.vd_backward
            _check(fn(self.handle, _ptr(gv), _ptr(gc), _ptr(gx), _ptr(g_xyz), _ptr(g_w), ctypes.c_void_p(stream)),
                   "vd_backward_noalloc" if noalloc else "vd_backward")
        self._keep_grad = (gv, gc, gx)
        return g_xyz, g_w


def _power_diagram_fn():
    import torch

    class PowerDiagramFn(torch.autograd.Function):
        """Differentiable diagram: (xyz, w) -> every output field of vd_write;
        volumes, centroids and vertices carry gradients (vd_backward), the
        integer topology does not.  The forward's cell records stay in the
        context as the checkpoint, so the backward must come before the next
        build on that context."""

        @staticmethod
        def forward(ctx, xyz, w, bbox, context, options):
            sz = context.build_sizes(xyz.detach(), None if w is None else w.detach(), bbox, **options)
            d = context.write(sz)
            ctx.context = context
            ctx.generation = context.generation
            ctx.has_w = w is not None
            ctx.n_vert = sz.n_vert
            ctx.set_materialize_grads(False)
            outs = tuple(getattr(d, k) for k in OUTPUT_FIELDS)
            ctx.mark_non_differentiable(*[t for k, t in zip(OUTPUT_FIELDS, outs)
                                          if k not in ("vol", "centroid", "vert")])
            ctx.sizes = d.sizes
            return outs

        @staticmethod
        def backward(ctx, *grads):
            g = dict(zip(OUTPUT_FIELDS, grads))
            if ctx.context.generation != ctx.generation:
                raise RuntimeError("the context was used for another build after this forward; give each "
                                   "differentiable diagram its own Context until its backward has run")
            if g["vol"] is None and g["centroid"] is None and g["vert"] is None:
                return None, None, None, None, None
            g_xyz, g_w = ctx.context.backward(g["vol"], g["centroid"], g["vert"], want_w=ctx.has_w)
            return g_xyz, g_w, None, None, None

    return PowerDiagramFn


_fn_cache = {}


def power_diagram(xyz, w=None, bbox=None, context: Context | None = None, **options) -> Diagram:
    """Differentiable build: like ``build`` but ``vol``, ``centroid`` and
    ``vert`` carry gradients to ``xyz`` and ``w`` (hand-written backward,
    combinatorics held fixed).  Uses a fresh Context unless one is given."""
    if "fn" not in _fn_cache:
        _fn_cache["fn"] = _power_diagram_fn()
    ctx = context if context is not None else Context(xyz.device)
    outs = _fn_cache["fn"].apply(xyz, w, bbox, ctx, options)
    d = dict(zip(OUTPUT_FIELDS, outs))
    d["sizes"] = ctx.last_sizes
    return Diagram(**d)


def measure_peaks(device=None) -> dict:
    """vd_measure_peaks: achievable HBM copy bandwidth (GB/s) and FP32 FMA
    rate (10^12 lane operations per second) of the device."""
    import torch
    dev = torch.device("cuda", torch.cuda.current_device() if device is None else torch.device(device).index or 0)
    lib = load_library()
    cg, ft = ctypes.c_double(0.0), ctypes.c_double(0.0)
    stream = torch.cuda.current_stream(dev).cuda_stream
    with torch.cuda.device(dev):
        _check(lib.vd_measure_peaks(dev.index, ctypes.c_void_p(stream), ctypes.byref(cg), ctypes.byref(ft)),
               "vd_measure_peaks")
    return {"copy_GBs": cg.value, "fma_Tops": ft.value}


_contexts: dict = {}


def context(device=None) -> Context:
    import torch
    idx = torch.cuda.current_device() if device is None else (torch.device(device).index or 0)
    if idx not in _contexts:
        _contexts[idx] = Context(idx)
    return _contexts[idx]


def build(xyz, w=None, bbox=None, **kw) -> Diagram:
    """Power (w given) or Voronoi diagram of the sites ``xyz`` clipped to ``bbox``
    (default: the sites' bounding box).  See ``include/vd.h`` for the layout."""
    return context(xyz.device).build(xyz, w, bbox, **kw)
