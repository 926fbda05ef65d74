"""GPU parity of the hybrid L1 Gauss-Seidel AMG smoother (Sec. 4.1) against the
oracle on the same seeded systems and chunk sizes: hierarchies unchanged
(bit-exact), forward and transposed applies entry-wise within 1e-10,
solutions within 1e-8 with iteration counts within one; FP32 apply; chunks of
one row against L1-Jacobi; option errors."""
import numpy as np
import pytest

import workloads as W
from _systems import SMALL, elem_err, gpu_solver, oracle_mgr, rel, say

pytestmark = pytest.mark.gpu

CASES = [("tpfa_16^3", 32), ("mimetic_20^3", 32), ("comp_20x18x10", 7), ("comp4_20x18x12", 32),
         ("frac_12^3", 32), ("frac_18^3", 128), ("frac_p_12^3", 5)]


@pytest.mark.parametrize("name,chunk", CASES)
def test_hybrid_gs_parity(name, chunk):
    s = SMALL[name]()
    kw = dict(smoother="hybrid-gs", chunk=chunk)
    om = oracle_mgr(s, **kw)
    gs = gpu_solver(s, **kw)
    say(f"[hgs] {name} chunk {chunk}: n = {s['n']}")
    assert gs.info() == om.info()
    rng = np.random.default_rng(11)
    for tr in (False, True):
        v = rng.standard_normal(s["n"])
        z, zo = gs.apply(v, transpose=tr).cpu().numpy(), om.apply(v, trans=tr)
        e = elem_err(z, zo, s["field"])
        say(f"[hgs] {name} apply trans={tr}: entry-wise err {e:.2e}")
        assert e <= 1e-10
    xo, io = om.solve(s["rhs"])
    X, [ig] = gs.solve(s["rhs"])
    x = X.cpu().numpy()
    A = W.csr_of(s)
    res = np.linalg.norm(s["rhs"] - A @ x) / np.linalg.norm(s["rhs"])
    say(f"[hgs] {name}: iterations gpu {ig.iterations} oracle {io.iterations}; true res {res:.2e}")
    assert ig.status == 0 and abs(ig.iterations - io.iterations) <= 1 and res <= 1e-8
    assert elem_err(x, xo, s["field"]) <= 1e-8
    gs.close()


def test_hybrid_gs_fp32_apply():
    s = SMALL["frac_18^3"]()
    om = oracle_mgr(s, smoother="hybrid-gs", chunk=32)
    gs = gpu_solver(s, smoother="hybrid-gs", chunk=32, precision=32)
    v = np.random.default_rng(3).standard_normal(s["n"])
    z32, zo = gs.apply(v).cpu().numpy(), om.apply(v)
    say(f"[hgs] fp32 apply vs fp64 oracle: 2-norm {rel(z32, zo):.2e}, entry-wise {elem_err(z32, zo, s['field']):.2e}")
    assert rel(z32, zo) <= 1e-4 and elem_err(z32, zo, s["field"]) <= 1e-3
    X, [ig] = gs.solve(s["rhs"])
    xo, io = om.solve(s["rhs"])
    assert ig.status == 0 and elem_err(X.cpu().numpy(), xo, s["field"]) <= 1e-7
    gs.close()


def test_hybrid_gs_chunk_one_is_l1_jacobi():
    s = SMALL["mimetic_9x7x6"]()
    gj = gpu_solver(s)
    gg = gpu_solver(s, smoother="hybrid-gs", chunk=1)
    v = np.random.default_rng(4).standard_normal(s["n"])
    for tr in (False, True):
        a, b = gg.apply(v, transpose=tr).cpu().numpy(), gj.apply(v, transpose=tr).cpu().numpy()
        assert elem_err(a, b, s["field"]) <= 1e-12
    gj.close(); gg.close()


def test_hybrid_gs_option_errors():
    import paper_2101_11649_amd as P
    s = SMALL["tpfa_7x6x5"]()
    for chunk in (0, 129):
        with pytest.raises(P.MgrError) as e:
            gpu_solver(s, smoother="hybrid-gs", chunk=chunk)
        assert e.value.code == -1


def _expected_tables(nr, rp, ci, v, chunk, backward):
    """Slot tables of the in-chunk entries of a CSR operator, written out row by
    row on the host: slot k of position t of chunk c at (t W + k) nchp + c."""
    nch = -(-nr // chunk)
    nchp = -(-nch // 64) * 64
    rows = []
    for i in range(nr):
        c0 = i - i % chunk
        c1 = min(nr, c0 + chunk)
        e = [(j - c0, x) for j, x in zip(ci[rp[i]:rp[i + 1]], v[rp[i]:rp[i + 1]])
             if (i < j < c1 if backward else c0 <= j < i)]
        rows.append(e)
    w = max((len(e) for e in rows), default=0)
    col = np.zeros(chunk * w * nchp, np.int64)
    val = np.zeros(chunk * w * nchp)
    for t in range(chunk):
        for c in range(nchp):
            i = c * chunk + t
            e = rows[i] if i < nr else []
            for k in range(w):
                o = (t * w + k) * nchp + c
                col[o], val[o] = e[k] if k < len(e) else (t, 0.0)
    return chunk * nchp, w, col, val


@pytest.mark.parametrize("name,chunk", [("comp_20x18x10", 7), ("frac_12^3", 32), ("mimetic_9x7x6", 128)])
def test_hybrid_gs_slot_tables(name, chunk):
    """The sweep's slot tables hold exactly each row's in-chunk entries (bit-equal
    values, columns relative to the chunk), then zero padding, for every level of
    every AMG hierarchy, with ragged last chunks."""
    s = SMALL[name]()
    gs = gpu_solver(s, smoother="hybrid-gs", chunk=chunk)
    hier = [(1, -1, len(gs.info()["amg_levels"]))]
    for sub in range(len(gs.info()["mgr_levels"])):
        k = 0
        while gs.export_sizes(2, k, 1, sub) is not None:
            k += 1
        if k:
            hier.append((2, sub, k))
    checked = 0
    for kind, sub, nl in hier:
        for k in range(nl - 1):
            nr, _, rp, ci, v = gs.export(kind, k, 1, sub)
            for what, bw in ((7, False), (8, True)):
                per, w, col, val = _expected_tables(nr, rp, ci, v, chunk, bw)
                got = gs.export(kind, k, what, sub)
                assert (got[0], got[1]) == (per, w), (kind, sub, k, what)
                assert np.array_equal(got[3], col) and np.array_equal(got[4], val), (kind, sub, k, what)
                checked += 1
    say(f"[hgs] {name} chunk {chunk}: {checked} slot tables equal to the host's")
    assert checked >= 4
    gs.close()
