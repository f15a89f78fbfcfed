"""Extension (1), precision: the plain FP32 form against the mixed FP32/FP64
form, each against the FP64 oracle, and the rate at which the mixed form
re-evaluates vertex side tests in FP64.

The plain FP32 form must be exact on cells certified at TAU_FP32 = 1e-5 and
the mixed form on cells certified at TAU_MIXED = 1e-10 (its doubtful signs are
decided in FP64, so only configurations within FP64 reach of a degeneracy
remain undecided).  The report states, per form, the mismatch rate of the
cells below its gate (configurations its arithmetic cannot decide, Sec.
"Precision" of the supplement) and the p50 / p99 / max geometry errors."""
import numpy as np
import pytest

from paper_2605_06408_amd import workloads as wl

from .parity import TAU_FP32, TAU_MIXED, compare, error_table, gpu_build, to_numpy

pytestmark = pytest.mark.gpu


def _report(oracle_mod, name, n_sample, seed):
    import torch
    xyz, w, box = wl.make(name, 0)
    n = len(xyz)
    rng = np.random.default_rng(seed)
    rows = {}
    flagged = set()
    for prec in (1, 2):
        d = gpu_build(xyz, w, box, precision=prec)
        flags = d.flags.cpu().numpy()
        flagged |= set(np.nonzero(flags & 2)[0][:300].tolist())
        rows[prec] = d
    ids = np.array(sorted(set(rng.choice(n, n_sample, replace=False).tolist()) | flagged), np.int64)
    o = oracle_mod.cells(xyz, w, box, ids=ids)
    out = {}
    for prec, d in rows.items():
        g = to_numpy(d, ids)
        rep = compare(g, o, tau=TAU_FP32 if prec == 1 else TAU_MIXED)
        out[prec] = rep
        print("%s precision=%d (gate %g): cells %d certified %d uncertified %d (mismatch %d) certified failures "
              "%d/%d; whole build: fp64 cells %d uncertain %d; errors p50/p99/max %s"
              % (name, prec, rep["tau"], rep["cells"], rep["certified"], rep["uncertified"],
                 rep["uncertified_mismatch"], len(rep["topo_fail"]), len(rep["geo_fail"]), d.sizes["n_fp64"],
                 d.sizes["n_uncertain"], error_table(rep)))
    del rows
    torch.cuda.empty_cache()
    return out


@pytest.mark.parametrize("name,n_sample", [("surface_20m", 1500), ("power_uniform_1m", 3000)])
def test_fp32_and_mixed_against_oracle(oracle_mod, name, n_sample):
    out = _report(oracle_mod, name, n_sample, 5)
    for prec in (1, 2):
        rep = out[prec]
        assert not rep["topo_fail"] and not rep["geo_fail"], rep
        assert rep["max_vert_err"] <= 1e-5 and rep["max_vol_err"] <= 1e-5 and rep["max_cen_err"] <= 1e-5
    # below its gate each form may differ from the oracle, but rarely
    for prec in (1, 2):
        rep = out[prec]
        assert rep["uncertified_mismatch"] <= max(3, 0.5 * rep["uncertified"]), rep["uncertified_mismatch"]
    # the mixed form's gate covers at least the FP32 form's cells
    assert out[2]["certified"] >= out[1]["certified"]


@pytest.mark.parametrize("name", ["power_uniform_1m", "surface_20m"])
def test_fp64_hit_rate(name):
    """Share of vertex side tests the mixed form re-evaluates in FP64."""
    import torch
    import paper_2605_06408_amd as vd
    xyz, w, box = wl.make(name, 0)
    ctx = vd.Context(0)
    x = torch.from_numpy(xyz).cuda()
    ww = None if w is None else torch.from_numpy(w).cuda()
    sz = ctx.build_sizes(x, ww, [float(v) for v in box], precision=2, counters=True)
    c = ctx.counters()["total"]
    rate = c["fp64_test"] / max(c["classify"], 1)
    print("%s mixed: %d of %d side tests in FP64 (%.3e), %d cells used FP64, %d uncertain"
          % (name, c["fp64_test"], c["classify"], rate, sz.n_fp64, sz.n_uncertain))
    assert rate < 1e-2
    assert sz.n_failed == 0
