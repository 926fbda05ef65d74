"""GPU parity of setup reuse (mgr_update_values): after new values on the same
pattern the GPU hierarchy must equal the oracle's reused hierarchy (C/F splits,
patterns and values bit-exact), and apply / solve must match it."""
import ctypes

import numpy as np
import pytest

import workloads as W
from _systems import elem_err, SMALL, gpu_solver, oracle_mgr, perturbed_values, rel, say

pytestmark = pytest.mark.gpu


def _same_csr(g, o, what):
    nr, nc, rp, ci, v = g
    assert (nr, nc) == (o.nr, o.nc), what
    assert np.array_equal(rp, o.rp) and np.array_equal(ci, o.ci), what
    assert np.array_equal(v, o.v), (what, np.abs(v - o.v).max() if len(v) else 0)


def _same_hierarchy(gs, om, levels):
    assert gs.info() == om.info()
    oi = om.info()
    for l in range(len(oi["mgr_levels"])):
        assert np.array_equal(gs.export(0, l, 0), om.export(0, l, 0))
        for what in (1, 2, 5):
            _same_csr(gs.export(0, l, what), om.export(0, l, what), f"MGR{l}/{what}")
    for k in range(len(oi["amg_levels"])):
        if k + 1 < len(oi["amg_levels"]):
            assert np.array_equal(gs.export(1, k, 0), om.export(1, k, 0))
            _same_csr(gs.export(1, k, 2), om.export(1, k, 2), f"AMG{k} P")
        _same_csr(gs.export(1, k, 1), om.export(1, k, 1), f"AMG{k} A")
    for l, lv in enumerate(levels):
        if lv.get("frelax") != "amg":
            continue
        k = 0
        while True:
            try:
                o = om.export(2, k, 1, sub=l)
            except KeyError:
                break
            _same_csr(gs.export(2, k, 1, sub=l), o, f"F-AMG{k} A")
            k += 1
        assert k >= 2


@pytest.mark.parametrize("name", ["tpfa_16^3", "mimetic_20^3", "comp4_20x18x12", "frac_12^3"])
def test_update_values_matches_oracle_reuse(name):
    s = SMALL[name]()
    say(f"[reuse] {name}")
    gs = gpu_solver(s)
    om = oracle_mgr(s)
    vals2 = perturbed_values(s, seed=7)
    s2 = dict(s, vals=vals2)
    gs.update_values(vals2)
    om2 = om.update(vals2)
    assert om2.status == 0
    _same_hierarchy(gs, om2, s["levels"])
    v = np.random.default_rng(3).standard_normal(s["n"])
    assert elem_err(gs.apply(v).cpu().numpy(), om2.apply(v), s["field"]) <= 1e-10
    assert elem_err(gs.apply(v, transpose=True).cpu().numpy(), om2.apply(v, trans=True), s["field"]) <= 1e-10
    X, [ig] = gs.solve(s2["rhs"])
    xo, io = om2.solve(s2["rhs"])
    say(f"[reuse] {name}: iterations gpu {ig.iterations} oracle {io.iterations}, x err {rel(X.cpu().numpy(), xo):.2e}")
    assert ig.status == 0 and abs(ig.iterations - io.iterations) <= 1 and elem_err(X.cpu().numpy(), xo, s["field"]) <= 1e-8
    # the FP32 apply is formed from the new values too
    gs.set_opts(precision=32)
    X32, [i32] = gs.solve(s2["rhs"])
    A2 = W.csr_of(s2)
    assert i32.status == 0
    assert np.linalg.norm(s2["rhs"] - A2 @ X32.cpu().numpy()) <= 1e-8 * np.linalg.norm(s2["rhs"])
    # a second update in a row
    vals3 = perturbed_values(s, seed=8)
    gs.update_values(vals3)
    om3 = om2.update(vals3)
    _same_hierarchy(gs, om3, s["levels"])


def test_update_keeping_frelaxation_amg_whole():
    s = SMALL["frac_18^3"]()
    say("[reuse] fracturing, F-relaxation AMG kept whole")
    gs = gpu_solver(s)
    om = oracle_mgr(s)
    vals2 = perturbed_values(s, seed=9, rows_field=3)
    gs.update_values(vals2, keep_frelax_amg=True)
    om2 = om.update(vals2, keep_frelax_amg=True)
    _same_hierarchy(gs, om2, s["levels"])
    v = np.random.default_rng(4).standard_normal(s["n"])
    assert elem_err(gs.apply(v).cpu().numpy(), om2.apply(v), s["field"]) <= 1e-10
    s2 = dict(s, vals=vals2)
    X, [ig] = gs.solve(s2["rhs"])
    xo, io = om2.solve(s2["rhs"])
    assert ig.status == 0 and abs(ig.iterations - io.iterations) <= 1 and elem_err(X.cpu().numpy(), xo, s["field"]) <= 1e-8


def test_update_errors():
    import torch
    import paper_2101_11649_amd as P
    L = P.lib()
    h = ctypes.c_void_p()
    assert L.mgr_create(ctypes.byref(h), None, None, P._ALLOC_FN(), P._FREE_FN(), None) == 0
    buf = torch.zeros(4, dtype=torch.float64, device="cuda")
    say("[reuse] update before setup")
    assert L.mgr_update_values(h, ctypes.c_void_p(buf.data_ptr()), 0) == -1
    L.mgr_destroy(h)
    s = SMALL["tpfa_7x6x5"]()
    gs = gpu_solver(s)
    v = torch.tensor(s["vals"], device="cuda")
    say("[reuse] null values, unknown flags")
    assert L.mgr_update_values(gs._h, None, 0) == -1
    assert L.mgr_update_values(gs._h, ctypes.c_void_p(v.data_ptr()), 4) == -1
    # the handle is still usable after a rejected call
    gs.update_values(v)
    X, [info] = gs.solve(s["rhs"])
    assert info.status == 0
