"""GPU parity of the displacement AMG built on the separate-component
approximation (Sec. 4.4; amg_unknown_based = 2) against the oracle: the
filtered level-0 operator and every level's C/F split, P and A_k of the
F-relaxation AMG bit-identical, forward and transposed applies entry-wise
within 1e-10, solutions within 1e-8 with iteration counts within one, with
plain and aggressive first levels, L1-Jacobi and hybrid Gauss-Seidel, and
after a setup reuse (new values on the same pattern)."""
import numpy as np
import pytest

import workloads as W
from _systems import SMALL, elem_err, gpu_solver, oracle_mgr, say
from test_gpu_agg import _compare_amg

pytestmark = pytest.mark.gpu


def _sdc_levels(s, agg):
    return [dict(l, amg_unknown_based=2, amg_agg_levels=agg) if l.get("frelax") == "amg" else l for l in s["levels"]]


CASES = [("frac_12^3", 0, {}), ("frac_12^3", 1, dict(smoother="hybrid-gs", chunk=32, nu_pre=1, nu_post=1)),
         ("frac_18^3", 1, dict(smoother="hybrid-gs", chunk=32, nu_pre=1, nu_post=1)), ("frac_18^3", 0, {})]


@pytest.mark.parametrize("name,agg,kw", CASES)
def test_separate_component_amg_parity(name, agg, kw):
    s = SMALL[name]()
    lv = _sdc_levels(s, agg)
    om = oracle_mgr(s, levels=lv, **kw)
    gs = gpu_solver(s, levels=lv, **kw)
    assert gs.info() == om.info()
    nk = _compare_amg(gs, om, 2, 0)
    assert nk >= 2
    a0 = gs.export(2, 0, 1, sub=0)
    assert len(a0[3]) < gs.export(0, 0, 4)[2][-1]      # the filter dropped entries
    rng = np.random.default_rng(31)
    for tr in (False, True):
        v = rng.standard_normal(s["n"])
        e = elem_err(gs.apply(v, transpose=tr).cpu().numpy(), om.apply(v, trans=tr), s["field"])
        say(f"[sdc] {name} agg {agg} {kw.get('smoother', 'l1-jacobi')} apply trans={tr}: entry-wise err {e:.2e}")
        assert e <= 1e-10
    xo, io = om.solve(s["rhs"])
    X, [ig] = gs.solve(s["rhs"])
    x = X.cpu().numpy()
    A = W.csr_of(s)
    res = np.linalg.norm(s["rhs"] - A @ x) / np.linalg.norm(s["rhs"])
    say(f"[sdc] {name}: iterations gpu {ig.iterations} oracle {io.iterations}; true res {res:.2e}")
    assert ig.status == 0 and abs(ig.iterations - io.iterations) <= 1 and res <= 1e-8
    assert elem_err(x, xo, s["field"]) <= 1e-8
    gs.close()


def test_separate_component_amg_setup_reuse():
    s = SMALL["frac_12^3"]()
    lv = _sdc_levels(s, 1)
    om = oracle_mgr(s, levels=lv)
    gs = gpu_solver(s, levels=lv)
    rng = np.random.default_rng(6)
    vals2 = s["vals"] * (1.0 + 0.02 * rng.standard_normal(s["vals"].size))
    om2 = om.update(vals2)
    gs.update_values(vals2)
    assert _compare_amg(gs, om2, 2, 0) >= 2
    v = rng.standard_normal(s["n"])
    assert elem_err(gs.apply(v).cpu().numpy(), om2.apply(v), s["field"]) <= 1e-10
    gs.close()


def test_separate_component_option_range():
    import paper_2101_11649_amd as P
    s = SMALL["frac_12^3"]()
    lv = [dict(l, amg_unknown_based=3) if l.get("frelax") == "amg" else l for l in s["levels"]]
    with pytest.raises(P.MgrError) as e:
        gpu_solver(s, levels=lv)
    assert e.value.code == -1
