"""GPU parity of the AMG with extended+i (distance-two) interpolation against
the oracle with the same option: C/F splits and interpolation patterns at every
level bit-exact, values bitwise equal (both sum in the same order), apply and
transposed apply within 1e-10, solutions within 1e-8 with iteration counts
within one.  Systems: scalar coarse AMG (two-field TPFA, mimetic MGR_P and
MGR_Pi, compositional) and the unknown-based F-relaxation AMG of the
fracturing system (labels)."""
import numpy as np
import pytest

import workloads as W
from _systems import elem_err, SMALL, gpu_solver, oracle_mgr, rel, say

pytestmark = pytest.mark.gpu

NAMES = ["tpfa_16^3", "mimetic_20^3", "mimetic_tpfa_pi_26x21x17", "comp_20x18x10", "frac_12^3"]


def _same_csr(g, o, what):
    assert np.array_equal(g[2], o.rp) and np.array_equal(g[3], o.ci), f"{what}: pattern"
    err = np.abs(g[4] - o.v).max() / max(np.abs(o.v).max(), 1e-300) if len(o.v) else 0.0
    assert err <= 1e-10, f"{what}: values {err:.2e}"
    return np.array_equal(g[4], o.v)


@pytest.mark.parametrize("name", NAMES)
def test_ext_interp_hierarchy_apply_solve(name):
    s = SMALL[name]()
    say(f"[ext+i] {name} n={s['n']}")
    om = oracle_mgr(s, interp="ext+i")
    gs = gpu_solver(s, interp="ext+i")
    gi, oi = gs.info(), om.info()
    say(f"[ext+i] {name}: gpu {gi} oracle {oi}")
    assert gi == oi
    bitwise = []
    for k in range(len(oi["amg_levels"])):
        if k + 1 < len(oi["amg_levels"]):
            assert np.array_equal(gs.export(1, k, 0), om.export(1, k, 0)), f"AMG level {k} C/F"
            bitwise.append(_same_csr(gs.export(1, k, 2), om.export(1, k, 2), f"AMG{k} P"))
        bitwise.append(_same_csr(gs.export(1, k, 1), om.export(1, k, 1), f"AMG{k} A"))
    for l, lv in enumerate(s["levels"]):
        if lv.get("frelax") != "amg":
            continue
        k = 0
        while True:
            try:
                ocf = om.export(2, k, 0, sub=l)
            except KeyError:
                break
            assert np.array_equal(gs.export(2, k, 0, sub=l), ocf), f"F-relaxation AMG level {k} C/F"
            bitwise.append(_same_csr(gs.export(2, k, 2, sub=l), om.export(2, k, 2, sub=l), f"F-AMG{k} P"))
            bitwise.append(_same_csr(gs.export(2, k, 1, sub=l), om.export(2, k, 1, sub=l), f"F-AMG{k} A"))
            k += 1
        assert k >= 2
    say(f"[ext+i] {name}: values bitwise equal in {sum(bitwise)}/{len(bitwise)} operators")
    assert all(bitwise)
    # the option took effect: the first interpolation differs from direct interpolation's
    od = oracle_mgr(s)
    kind, sub = (2, 0) if any(lv.get("frelax") == "amg" for lv in s["levels"]) else (1, -1)
    pe = om.export(kind, 0, 2, sub=sub) if sub >= 0 else om.export(kind, 0, 2)
    pd = od.export(kind, 0, 2, sub=sub) if sub >= 0 else od.export(kind, 0, 2)
    assert len(pe.ci) > len(pd.ci)
    rng = np.random.default_rng(5)
    for tr in (False, True):
        v = rng.standard_normal(s["n"])
        e = elem_err(gs.apply(v, transpose=tr).cpu().numpy(), om.apply(v, trans=tr), s["field"])
        say(f"[ext+i] {name} apply trans={tr}: entry-wise err {e:.2e}")
        assert e <= 1e-10
    xo, io = om.solve(s["rhs"])
    X, [ig] = gs.solve(s["rhs"])
    x = X.cpu().numpy()
    tr = np.linalg.norm(s["rhs"] - W.csr_of(s) @ x) / np.linalg.norm(s["rhs"])
    say(f"[ext+i] {name}: iters gpu {ig.iterations} oracle {io.iterations}; true res {tr:.2e}; "
        f"x err {rel(x, xo):.2e}")
    assert ig.status == 0 and io.status == 0
    assert abs(ig.iterations - io.iterations) <= 1
    assert tr <= 1e-8 and elem_err(x, xo, s["field"]) <= 1e-8
    # FP32 apply with the same hierarchy
    gs.set_opts(precision=32)
    X32, [i32] = gs.solve(s["rhs"])
    tr32 = np.linalg.norm(s["rhs"] - W.csr_of(s) @ X32.cpu().numpy()) / np.linalg.norm(s["rhs"])
    say(f"[ext+i] {name}: fp32 apply iters {i32.iterations}, true res {tr32:.2e}")
    assert i32.status == 0 and tr32 <= 1e-8
    gs.close()


def test_ext_interp_full_size_mimetic():
    # the 64^3 mimetic system: hierarchy and solution against the oracle
    s = W.hybrid_mimetic(64, 64, 64, seed=1)
    gs = gpu_solver(s, interp="ext+i")
    X, [ig] = gs.solve(s["rhs"])
    om = oracle_mgr(s, interp="ext+i")
    gi, oi = gs.info(), om.info()
    say(f"[ext+i] mimetic 64^3: gpu {gi}")
    assert gi == oi
    for k in range(len(oi["amg_levels"]) - 1):
        assert np.array_equal(gs.export(1, k, 0), om.export(1, k, 0)), f"AMG level {k} C/F"
        _same_csr(gs.export(1, k, 2), om.export(1, k, 2), f"AMG{k} P")
    xo, io = om.solve(s["rhs"])
    x = X.cpu().numpy()
    say(f"[ext+i] mimetic 64^3: iters gpu {ig.iterations} oracle {io.iterations}; x err {rel(x, xo):.2e}")
    assert ig.status == 0 and abs(ig.iterations - io.iterations) <= 1 and elem_err(x, xo, s["field"]) <= 1e-8
    gs.close()
