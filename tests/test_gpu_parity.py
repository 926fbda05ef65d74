"""GPU parity: the HIP library (through its C-ABI) against the FP64 oracle on the
same seeded inputs.  Bar: C/F splits and sparsity patterns bit-exact; FP64
values within 1e-10 relative; solutions within 1e-8 relative of the oracle's."""
import numpy as np
import pytest

import workloads as W
from _systems import elem_err, SMALL, gpu_solver, oracle_mgr, rel, say

pytestmark = pytest.mark.gpu

NAMES = list(SMALL)


@pytest.fixture(scope="module")
def built():
    cache = {}

    def get(name, **kw):
        key = (name, tuple(sorted(kw.items())))
        if key not in cache:
            s = SMALL[name]()
            say(f"[setup] {name} n={s['n']} kw={kw}")
            cache[key] = (s, oracle_mgr(s), gpu_solver(s, **kw))
        return cache[key]
    return get


@pytest.mark.parametrize("name", NAMES)
def test_matvec(built, name):
    s, om, gs = built(name)
    rng = np.random.default_rng(1)
    x = rng.standard_normal(s["n"])
    for tr in (False, True):
        y = gs.matvec(x, transpose=tr).cpu().numpy()
        assert elem_err(y, om.matvec(x, trans=tr), s["field"]) <= 1e-14


def _compare_csr(g, o, what):
    nr, nc, rp, ci, v = g
    assert (nr, nc) == (o.nr, o.nc), what
    assert np.array_equal(rp, o.rp), what + " row pointers"
    assert np.array_equal(ci, o.ci), what + " columns"
    scale = np.abs(o.v).max() if len(o.v) else 1.0
    err = np.abs(v - o.v).max() / scale if len(o.v) else 0.0
    assert err <= 1e-10, (what, err)
    return bool(np.array_equal(v, o.v))


@pytest.mark.parametrize("name", NAMES)
def test_hierarchy_bit_exact(built, name):
    s, om, gs = built(name)
    gi, oi = gs.info(), om.info()
    say(f"{name}: gpu {gi} oracle {oi}")
    assert gi == oi
    bitwise = []
    for l in range(len(oi["mgr_levels"])):
        assert np.array_equal(gs.export(0, l, 0), om.export(0, l, 0))
        for what, nm in ((1, "A_c"), (2, "P_F"), (4, "A_FF"), (5, "M")):
            bitwise.append(_compare_csr(gs.export(0, l, what), om.export(0, l, what), f"MGR{l} {nm}"))
    for k in range(len(oi["amg_levels"])):
        if k + 1 < len(oi["amg_levels"]):
            assert np.array_equal(gs.export(1, k, 0), om.export(1, k, 0)), f"AMG level {k} C/F"
            bitwise.append(_compare_csr(gs.export(1, k, 2), om.export(1, k, 2), f"AMG{k} P"))
        bitwise.append(_compare_csr(gs.export(1, k, 1), om.export(1, k, 1), f"AMG{k} A"))
    # AMG hierarchies used as F-relaxation (MGR_FRELAX_AMG levels)
    for l, lv in enumerate(s["levels"]):
        if lv.get("frelax") != "amg":
            continue
        k = 0
        while True:
            try:
                o = om.export(2, k, 1, sub=l)
            except KeyError:
                break
            bitwise.append(_compare_csr(gs.export(2, k, 1, sub=l), o, f"F-AMG{k} A"))
            try:
                ocf = om.export(2, k, 0, sub=l)
            except KeyError:
                break
            assert np.array_equal(gs.export(2, k, 0, sub=l), ocf), f"F-relaxation AMG level {k} C/F"
            bitwise.append(_compare_csr(gs.export(2, k, 2, sub=l), om.export(2, k, 2, sub=l), f"F-AMG{k} P"))
            k += 1
        assert k >= 1
    say(f"{name}: values bitwise equal in {sum(bitwise)}/{len(bitwise)} operators")
    assert all(bitwise)


@pytest.mark.parametrize("name", NAMES)
def test_apply(built, name):
    s, om, gs = built(name)
    rng = np.random.default_rng(2)
    for tr in (False, True):
        v = rng.standard_normal(s["n"])
        z = gs.apply(v, transpose=tr).cpu().numpy()
        zo = om.apply(v, trans=tr)
        e = elem_err(z, zo, s["field"])
        say(f"{name} apply trans={tr}: entry-wise err {e:.2e} (2-norm {rel(z, zo):.2e})")
        assert e <= 1e-10


@pytest.mark.parametrize("name", NAMES)
def test_solve(built, name):
    s, om, gs = built(name)
    xo, io = om.solve(s["rhs"])
    X, [ig] = gs.solve(s["rhs"])
    x = X.cpu().numpy()
    A = W.csr_of(s)
    tr = np.linalg.norm(s["rhs"] - A @ x) / np.linalg.norm(s["rhs"])
    say(f"{name}: iters gpu {ig.iterations} oracle {io.iterations}; true res {tr:.2e}; "
        f"x err {rel(x, xo):.2e}")
    assert ig.status == 0 and io.status == 0
    assert abs(ig.iterations - io.iterations) <= 1
    assert tr <= 1e-8
    assert elem_err(x, xo, s["field"]) <= 1e-8


@pytest.mark.parametrize("name", ["tpfa_16^3", "mimetic_20^3", "comp_20x18x10", "comp4_20x18x12"])
def test_solve_fp32_apply(built, name):
    s, om, gs = built(name, precision=32)
    xo, io = om.solve(s["rhs"])
    X, [ig] = gs.solve(s["rhs"])
    x = X.cpu().numpy()
    A = W.csr_of(s)
    tr = np.linalg.norm(s["rhs"] - A @ x) / np.linalg.norm(s["rhs"])
    say(f"{name} fp32 apply: iters {ig.iterations} (fp64 oracle {io.iterations}); true res {tr:.2e}; "
        f"x err vs oracle {rel(x, xo):.2e}")
    assert ig.status == 0 and tr <= 1e-8
    # z = M^{-1} v in FP32 storage/accumulation: within single-precision rounding of the FP64 oracle
    v = np.random.default_rng(3).standard_normal(s["n"])
    z32, zo = gs.apply(v).cpu().numpy(), om.apply(v)
    e32 = elem_err(z32, zo, s["field"])
    say(f"{name} fp32 apply vs fp64 oracle: entry-wise err {e32:.2e} (2-norm {rel(z32, zo):.2e})")
    assert rel(z32, zo) <= 1e-4 and e32 <= 1e-3


VARIANTS = {
    "jacobi_restriction": dict(restrict="jacobi"),
    "two_sweeps_omega": dict(sweeps=2, omega=0.8),
    "amg_frelax": dict(frelax="amg"),
    "ilu0_frelax": dict(frelax="ilu0"),
    "ilu0_two_sweeps_jacobi_r": dict(frelax="ilu0", sweeps=2, restrict="jacobi"),
}


@pytest.mark.parametrize("variant", list(VARIANTS))
def test_level_variants(variant):
    s = W.two_field_tpfa(9, 8, 7, seed=21)
    lv = [dict(s["levels"][0], **VARIANTS[variant])]
    say(f"[variant] {variant}")
    om = oracle_mgr(s, levels=lv, max_coarse=40)
    gs = gpu_solver(s, levels=lv, max_coarse=40)
    v = np.random.default_rng(4).standard_normal(s["n"])
    assert elem_err(gs.apply(v).cpu().numpy(), om.apply(v), s["field"]) <= 1e-10
    if VARIANTS[variant].get("sweeps", 1) == 1:
        assert elem_err(gs.apply(v, transpose=True).cpu().numpy(), om.apply(v, trans=True), s["field"]) <= 1e-10
    X, [ig] = gs.solve(s["rhs"])
    xo, io = om.solve(s["rhs"])
    assert abs(ig.iterations - io.iterations) <= 1 and elem_err(X.cpu().numpy(), xo, s["field"]) <= 1e-8


def test_pure_amg_no_mgr_level():
    s = W.hybrid_mimetic(8, 8, 8, seed=9, consistent=False, upwind=False)
    say("[pure AMG]")
    om = oracle_mgr(s, levels=[])
    gs = gpu_solver(s, levels=[])
    v = np.random.default_rng(5).standard_normal(s["n"])
    assert elem_err(gs.apply(v).cpu().numpy(), om.apply(v), s["field"]) <= 1e-10


def test_error_codes():
    import paper_2101_11649_amd as P
    s = W.two_field_tpfa(4, 4, 4, seed=1)
    bad = dict(s)
    bad["field"] = s["field"].copy()
    bad["field"][3] = 40
    say("[errors] bad label")
    with pytest.raises(P.MgrError) as e:
        gpu_solver(bad)
    assert e.value.code == -5
    say("[errors] empty F set")
    with pytest.raises(P.MgrError) as e:
        gpu_solver(s, levels=[dict(s["levels"][0], fmask=1 << 5)])
    assert e.value.code == -5
    z = dict(s)
    z["vals"] = s["vals"].copy().reshape(-1, 2, 2)
    # zero the saturation diagonal of block row 0 (its diagonal block is the first of the row)
    z["vals"][s["rp"][0] + list(s["ci"][s["rp"][0]:s["rp"][1]]).index(0), 1, 1] = 0.0
    z["vals"] = z["vals"].reshape(-1)
    say("[errors] zero F pivot")
    with pytest.raises(P.MgrError) as e:
        gpu_solver(z)
    assert e.value.code == -3


def test_zero_rhs_and_maxiter():
    s = W.two_field_tpfa(5, 5, 5, seed=2)
    gs = gpu_solver(s, maxiter=3)
    say("[edge] zero rhs / maxiter")
    X, [i0] = gs.solve(np.zeros(s["n"]))
    assert i0.status == 0 and i0.iterations == 0 and not X.cpu().numpy().any()
    X, [i1] = gs.solve(s["rhs"])
    assert i1.status == 1 and i1.iterations == 3


def test_multi_rhs_solve_and_gradient():
    import torch
    import paper_2101_11649_amd as P
    s = W.hybrid_mimetic(5, 4, 4, seed=13, nrhs=3)
    say("[adjoint] 3 rhs")
    om = oracle_mgr(s)
    gs = gpu_solver(s, rtol=1e-12)
    B = s["rhs"]
    X, infos = gs.solve(B)
    C = s["loss_weights"]
    Lam, _ = gs.solve(C, transpose=True)
    X, Lam = X.cpu().numpy(), Lam.cpu().numpy()
    for k in range(3):
        xo, _ = om.solve(B[k], rtol=1e-12)
        lo, _ = om.solve(C[k], trans=True, rtol=1e-12)
        assert elem_err(X[k], xo, s["field"]) <= 1e-9 and elem_err(Lam[k], lo, s["field"]) <= 1e-9
    import oracle as O
    g = gs.grad_values(Lam, X).cpu().numpy()
    go = O.grad_values(1, s["rp"], s["ci"], Lam, X)
    assert elem_err(g, go) <= 1e-13
    # through torch.autograd
    vals = torch.tensor(s["vals"], device="cuda", requires_grad=True)
    Bt = torch.tensor(B, device="cuda", requires_grad=True)
    struct = dict(b=1, rp=s["rp"], ci=s["ci"], field=s["field"], levels=s["levels"], opts=dict(rtol=1e-12))
    Xt = P.MGRSolve.apply(vals, Bt, struct)
    loss = (Xt * torch.tensor(C, device="cuda")).sum()
    loss.backward()
    assert elem_err(vals.grad.cpu().numpy(), go) <= 1e-8
    assert elem_err(Bt.grad.cpu().numpy(), Lam, s["field"]) <= 1e-8


def test_ilu0_on_compositional_components():
    # ILU(0) F-relaxation of the three component densities (the paper recommends
    # incomplete factorizations for such transport blocks)
    s = W.compositional_wells(12, 10, 8, seed=9)
    lv = [dict(s["levels"][0], frelax="ilu0"), s["levels"][1]]
    say("[ilu0] compositional 12x10x8")
    om = oracle_mgr(s, levels=lv)
    gs = gpu_solver(s, levels=lv)
    v = np.random.default_rng(8).standard_normal(s["n"])
    assert elem_err(gs.apply(v).cpu().numpy(), om.apply(v), s["field"]) <= 1e-10
    assert elem_err(gs.apply(v, transpose=True).cpu().numpy(), om.apply(v, trans=True), s["field"]) <= 1e-10
    X, [ig] = gs.solve(s["rhs"])
    xo, io = om.solve(s["rhs"])
    say(f"[ilu0] iterations gpu {ig.iterations} oracle {io.iterations}")
    assert abs(ig.iterations - io.iterations) <= 1 and elem_err(X.cpu().numpy(), xo, s["field"]) <= 1e-8
    gs.set_opts(precision=32)
    X32, [i32] = gs.solve(s["rhs"])
    assert i32.status == 0 and elem_err(X32.cpu().numpy(), xo, s["field"]) <= 1e-7


@pytest.mark.parametrize("name,restart", [("tpfa_7x6x5", 7), ("mimetic_9x7x6", 5), ("comp_8x8x6", 3),
                                          ("frac_12^3", 10)])
def test_solve_with_restarts(name, restart):
    """Short restart cycles: every cycle ends on a completed Hessenberg column
    and the next one restarts from the true residual; iteration counts and
    solutions as the oracle's FGMRES(restart)."""
    s = SMALL[name]()
    om = oracle_mgr(s)
    gs = gpu_solver(s, restart=restart, rtol=1e-10)
    xo, io = om.solve(s["rhs"], restart=restart, rtol=1e-10)
    X, [ig] = gs.solve(s["rhs"])
    x = X.cpu().numpy()
    A = W.csr_of(s)
    tr = np.linalg.norm(s["rhs"] - A @ x) / np.linalg.norm(s["rhs"])
    say(f"{name} restart {restart}: iters gpu {ig.iterations} ({ig.restarts} restarts) oracle {io.iterations} "
        f"({io.restarts}); true res {tr:.2e}; x err {rel(x, xo):.2e}")
    assert ig.status == 0 and io.status == 0 and ig.restarts >= 1
    assert abs(ig.iterations - io.iterations) <= 1
    assert tr <= 1e-10
    assert elem_err(x, xo, s["field"]) <= 1e-8
    gs.close()
