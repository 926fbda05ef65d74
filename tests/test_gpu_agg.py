"""GPU parity of aggressive coarsening with multi-pass interpolation (the first
level of the mechanics AMG, Sec. 4.1) against the oracle: every level's C/F
split and every P and A_k bit-identical (coarse AMG and F-relaxation AMG),
forward and transposed applies entry-wise within 1e-10, solutions within 1e-8
with iteration counts within one."""
import numpy as np
import pytest

import workloads as W
from _systems import SMALL, elem_err, gpu_solver, oracle_mgr, say

pytestmark = pytest.mark.gpu


def _same_csr(g, o, what):
    nr, nc, rp, ci, v = g
    assert (nr, nc) == (o.nr, o.nc), what
    assert np.array_equal(rp, o.rp) and np.array_equal(ci, o.ci), what
    assert np.array_equal(v, o.v), what


def _compare_amg(gs, om, kind, sub):
    k = 0
    while True:
        try:
            oa = om.export(kind, k, 1, sub=sub)
        except KeyError:
            break
        _same_csr(gs.export(kind, k, 1, sub=sub), oa, f"AMG({kind}) level {k} A")
        try:
            ocf = om.export(kind, k, 0, sub=sub)
        except KeyError:
            break
        assert np.array_equal(gs.export(kind, k, 0, sub=sub), ocf), f"AMG({kind}) level {k} C/F"
        _same_csr(gs.export(kind, k, 2, sub=sub), om.export(kind, k, 2, sub=sub), f"AMG({kind}) level {k} P")
        k += 1
    return k


def _agg_levels(s, frelax_agg):
    return [dict(l, amg_agg_levels=frelax_agg) if l.get("frelax") == "amg" else l for l in s["levels"]]


CASES = [
    # MGR_U: aggressive first level of the unknown-based displacement AMG (F-relaxation)
    ("frac_12^3", dict(levels=1)),
    ("frac_18^3", dict(levels=1)),
    # MGR_P: aggressive first level of the coarse unknown-based displacement AMG
    ("frac_p_12^3", dict(coarse=1)),
    ("frac_p_18^3", dict(coarse=1)),
    # scalar coarse AMGs, two aggressive levels on the TPFA pressure system
    ("mimetic_20^3", dict(coarse=1)),
    ("tpfa_16^3", dict(coarse=2)),
]


@pytest.mark.parametrize("name,agg", CASES)
def test_aggressive_coarsening_parity(name, agg):
    s = SMALL[name]()
    lv = _agg_levels(s, agg.get("levels", 0))
    kw = dict(agg_levels=agg.get("coarse", 0))
    om = oracle_mgr(s, levels=lv, **kw)
    gs = gpu_solver(s, levels=lv, **kw)
    gi, oi = gs.info(), om.info()
    say(f"[agg] {name} {agg}: gpu {gi} oracle {oi}")
    assert gi == oi
    nk = _compare_amg(gs, om, 1, -1)
    for l, lvo in enumerate(lv):
        if lvo.get("frelax") == "amg":
            nk += _compare_amg(gs, om, 2, l)
    assert nk >= 1
    rng = np.random.default_rng(21)
    for tr in (False, True):
        v = rng.standard_normal(s["n"])
        e = elem_err(gs.apply(v, transpose=tr).cpu().numpy(), om.apply(v, trans=tr), s["field"])
        say(f"[agg] {name} apply trans={tr}: entry-wise err {e:.2e}")
        assert e <= 1e-10
    xo, io = om.solve(s["rhs"])
    X, [ig] = gs.solve(s["rhs"])
    x = X.cpu().numpy()
    A = W.csr_of(s)
    res = np.linalg.norm(s["rhs"] - A @ x) / np.linalg.norm(s["rhs"])
    say(f"[agg] {name}: iterations gpu {ig.iterations} oracle {io.iterations}; true res {res:.2e}")
    assert ig.status == 0 and abs(ig.iterations - io.iterations) <= 1 and res <= 1e-8
    assert elem_err(x, xo, s["field"]) <= 1e-8
    gs.close()


def test_aggressive_coarsening_with_setup_reuse():
    s = SMALL["frac_12^3"]()
    lv = _agg_levels(s, 1)
    om = oracle_mgr(s, levels=lv)
    gs = gpu_solver(s, levels=lv)
    rng = np.random.default_rng(5)
    vals2 = s["vals"] * (1.0 + 0.02 * rng.standard_normal(s["vals"].size))
    om2 = om.update(vals2)
    gs.update_values(vals2)
    assert _compare_amg(gs, om2, 2, 0) >= 1
    v = rng.standard_normal(s["n"])
    assert elem_err(gs.apply(v).cpu().numpy(), om2.apply(v), s["field"]) <= 1e-10
    gs.close()
