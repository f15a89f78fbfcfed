"""vd_backward_noalloc (the backward whose scratch is the library's fixed
device array, for callers that cannot allocate) against vd_backward on the
same build: two calls in a row, the second on a smaller diagram (and with
the sites' own box, so the box-face scratch is used too), then a diagram too
large for the fixed scratch, which must be refused with a clear error.

Both entry points run the same kernels; only the order of the FP64 atomic
adds of facets not listed back by their neighbour may differ, so the
gradients must agree to FP32 rounding of the same FP64 sums (relative 1e-6
of the site's gradient plus the mean gradient size)."""
import numpy as np
import pytest
import torch

import paper_2605_06408_amd as vd
from paper_2605_06408_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _grads(ctx, seed, n_vert, with_vert):
    g = torch.Generator().manual_seed(seed)
    n = ctx.n
    gv = torch.randn(n, generator=g).float().cuda()
    gc = torch.randn(n, 3, generator=g).float().cuda()
    gx = torch.randn(n_vert, 3, generator=g).float().cuda() if with_vert else None
    return gv, gc, gx


def _compare(a, b):
    a = a.double().cpu().numpy()
    b = b.double().cpu().numpy()
    scale = np.abs(b).reshape(len(b), -1).max(axis=1) + np.abs(b).mean()
    err = np.abs(a - b).reshape(len(b), -1).max(axis=1) / scale
    assert np.isfinite(a).all()
    assert float(err.max()) <= 1e-6, float(err.max())


@pytest.mark.parametrize("case", [0])
def test_noalloc_backward_matches_vd_backward(case):
    ctx = vd.Context(0)
    try:
        # first call: 3000 weighted sites in a given box, with a vertex gradient
        xyz, w, box = wl.power_uniform(3000, 0)
        w = (w * 0.05).astype(np.float32)
        sz = ctx.build_sizes(torch.from_numpy(xyz).cuda(), torch.from_numpy(w).cuda(), [float(v) for v in box])
        gv, gc, gx = _grads(ctx, 1, sz.n_vert, True)
        ref_x, ref_w = ctx.backward(gv, gc, gx)
        got_x, got_w = ctx.backward(gv, gc, gx, noalloc=True)
        torch.cuda.synchronize()
        print("call 1: n=%d facets=%d" % (sz.n, sz.n_facet))
        _compare(got_x, ref_x)
        _compare(got_w, ref_w)

        # second call, smaller: 700 Voronoi sites, box = the sites' own (its
        # faces carry gradient to the extreme sites), no vertex gradient
        xyz2, _, _ = wl.uniform(700, 3)
        sz2 = ctx.build_sizes(torch.from_numpy(xyz2).cuda(), None, None)
        gv2, gc2, _ = _grads(ctx, 2, sz2.n_vert, False)
        ref_x2, ref_w2 = ctx.backward(gv2, gc2, None)
        got_x2, got_w2 = ctx.backward(gv2, gc2, None, noalloc=True)
        torch.cuda.synchronize()
        print("call 2: n=%d facets=%d" % (sz2.n, sz2.n_facet))
        _compare(got_x2, ref_x2)
        _compare(got_w2, ref_w2)
        # the extreme sites do receive the box-face terms
        assert float(got_x2.abs().max()) > 0.0
    finally:
        ctx.close()


def test_noalloc_backward_refuses_a_diagram_beyond_its_scratch():
    ctx = vd.Context(0)
    try:
        # 32 B per facet alone exceed 64 MiB beyond about 2.1M facets
        xyz, _, box = wl.uniform(200000, 4)
        sz = ctx.build_sizes(torch.from_numpy(xyz).cuda(), None, [float(v) for v in box])
        assert 32 * sz.n_facet > 64 << 20
        gv = torch.ones(sz.n, dtype=torch.float32, device="cuda")
        with pytest.raises(vd.VDError) as e:
            ctx.backward(gv, None, None, noalloc=True)
        assert e.value.status == 1 and "scratch" in str(e.value)
        # the refused call left nothing behind: a small diagram still works
        xyz2, _, box2 = wl.uniform(500, 5)
        ctx.build_sizes(torch.from_numpy(xyz2).cuda(), None, [float(v) for v in box2])
        gv2 = torch.ones(500, dtype=torch.float32, device="cuda")
        a, _ = ctx.backward(gv2, None, None)
        b, _ = ctx.backward(gv2, None, None, noalloc=True)
        torch.cuda.synchronize()
        _compare(b, a)
    finally:
        ctx.close()
