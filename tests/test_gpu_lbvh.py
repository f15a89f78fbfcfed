"""Unit tests of the bounding-volume hierarchy the library builds (Sec. 4.3:
a binary BVH over the sites whose nodes also hold the largest weight below
them), read through vd_inspect_bvh:

  * the radix sort: the sorted Morton codes and the order equal a stable
    torch.sort of the codes;
  * the tree: a walk from the root reaches every internal node once and every
    site in exactly one leaf; leaves hold at most leaf_size sites in
    consecutive Morton positions; every node covers a contiguous range;
  * bounds: each child record's box is exactly the min/max of its sites and
    its max weight exactly their largest weight (a box that is too tight or a
    wrong max weight would only show as a rare parity miss);
  * leaf records: each site's record is the leaf that holds it."""
import numpy as np
import pytest

from paper_2605_06408_amd import workloads as wl

pytestmark = pytest.mark.gpu

LEAF_BIT = 0x80000000


def _build(xyz, w, box, leaf_size):
    import torch
    import paper_2605_06408_amd as vd
    ctx = vd.Context(0)
    ctx.build_sizes(torch.from_numpy(xyz).cuda(), None if w is None else torch.from_numpy(w).cuda(),
                    [float(v) for v in box], leaf_size=leaf_size)
    return ctx.inspect_bvh()


def _walk(b, n):
    """Ranges of every child record by an explicit-stack walk from the root;
    returns [(node, side, first, last)] for all child records and the list of
    leaf ranges in visiting order."""
    nodes = b["nodes"]
    refs = nodes[:, :, 7].view(np.uint32)
    visits = np.zeros(len(nodes), np.int64)
    leaves = []
    records = []
    rng = {}

    def leaf_range(ref):
        first = ref & 0x1FFFFFF
        return first, first + ((ref >> 25) & 63)

    # post-order: ranges of internal nodes from their children
    stack = [(0, False)]
    while stack:
        node, expanded = stack.pop()
        if not expanded:
            visits[node] += 1
            stack.append((node, True))
            for s in (1, 0):
                r = int(refs[node, s])
                if not r & LEAF_BIT:
                    stack.append((r, False))
            continue
        span = []
        for s in (0, 1):
            r = int(refs[node, s])
            if r & LEAF_BIT:
                f, l = leaf_range(r)
                leaves.append((f, l))
            else:
                f, l = rng[r]
            records.append((node, s, f, l))
            span.append((f, l))
        # the two children are adjacent Morton ranges
        (f0, l0), (f1, l1) = span
        assert l0 + 1 == f1, (node, span)
        rng[node] = (f0, l1)
    return visits, leaves, records, rng


@pytest.mark.parametrize("name,n,leaf_size", [("uniform", 100_000, 32), ("clustered", 200_000, 32),
                                              ("clustered", 30_000, 1), ("power_uniform", 100_000, 7),
                                              ("power_clustered", 120_000, 64)])
def test_bvh(name, n, leaf_size):
    import torch
    xyz, w, box = getattr(wl, name)(n, 4)
    b = _build(xyz, w, box, leaf_size)
    # radix sort against torch.sort (stable: equal codes keep input order)
    mort = torch.from_numpy(b["morton"])
    vals, idx = torch.sort(mort, stable=True)
    assert np.array_equal(b["sorted_keys"], vals.numpy())
    assert np.array_equal(b["order"].astype(np.int64), idx.numpy())
    assert np.all(b["morton"] >= 0) and b["morton"].max() < (1 << 63)
    # tree
    assert not b["root"] & LEAF_BIT
    visits, leaves, records, rng = _walk(b, n)
    assert np.all(visits[visits > 0] == 1)
    cover = np.zeros(n, np.int64)
    for f, l in leaves:
        assert l - f + 1 <= leaf_size
        cover[f:l + 1] += 1
    assert np.all(cover == 1)
    assert rng[0] == (0, n - 1)
    # bounds and max weights, exactly
    order = b["order"].astype(np.int64)
    sp = xyz[order]
    sw = np.zeros(n, np.float32) if w is None else w[order]
    nodes = b["nodes"]
    fl = nodes.view(np.float32)
    for node, s, f, l in records:
        lo, hi = sp[f:l + 1].min(0), sp[f:l + 1].max(0)
        assert np.array_equal(fl[node, s, 0:3], lo), (node, s)
        assert np.array_equal(fl[node, s, 4:7], hi), (node, s)
        assert fl[node, s, 3] == sw[f:l + 1].max(), (node, s)
    # leaf records
    lo = b["leaf_of"].view(np.uint32).astype(np.int64)
    ref = nodes[:, :, 7].view(np.uint32)[lo >> 1, lo & 1].astype(np.int64)
    assert np.all(ref & LEAF_BIT)
    first = ref & 0x1FFFFFF
    last = first + ((ref >> 25) & 63)
    k = np.arange(n)
    assert np.all((first <= k) & (k <= last))


def test_root_is_a_leaf_for_small_inputs():
    xyz, w, box = wl.uniform(20, 1)
    b = _build(xyz, None, box, 32)
    assert b["root"] & LEAF_BIT and (b["root"] & 0x1FFFFFF) == 0 and ((b["root"] >> 25) & 63) + 1 == 20
