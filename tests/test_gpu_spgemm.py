"""GPU: Galerkin products whose symbolic pass overflows its hash tables.

The coarse operator A_c = A_CC - A_CF D_FF^-1 A_FC of this system has one row
(C-point 0) with 577 distinct columns: it reaches 24 F-points, each coupled to
24 other C-points of its own.  The row-length bound (24 x 25 = 600) lets the
symbolic pass use hash tables of 512 slots, which that row overflows, so the
product is counted again by the merging kernels.  A second system overflows
the first, 64-slot count of the fused A_C = A_CC + A_CF P_F product (counted
again in tables sized for its bound).  The hierarchies must still match the
oracle's bit for bit and the solves must agree."""
import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W
from _systems import elem_err, gpu_solver, oracle_mgr, rel, say

pytestmark = pytest.mark.gpu


def _star_system(nc=5000, nf=600, fan=24, seed=3):
    rng = np.random.default_rng(seed)
    n = nc + nf
    rows, cols, vals = [], [], []

    def add(i, j, v):
        rows.append(i); cols.append(j); vals.append(v)

    for i in range(nc):
        add(i, i, 10.0 + rng.random())
        if i + 1 < nc:
            add(i, i + 1, -1.0); add(i + 1, i, -1.0)
    for k in range(nf):
        f = nc + k
        add(f, f, 10.0 + rng.random())
        if k < fan:
            nbrs = [0] + [1 + fan * k + t for t in range(fan)]
        else:
            nbrs = [(7 * k) % nc, (7 * k + 1) % nc]
        for c in nbrs:
            v = -0.1 * (0.5 + rng.random())
            add(f, c, v); add(c, f, v)
    A = sp.coo_matrix((vals, (rows, cols)), shape=(n, n)).tocsr()
    A.sum_duplicates()
    A.sort_indices()
    field = np.concatenate([np.zeros(nc, np.int32), np.ones(nf, np.int32)])
    return W._system(1, A.indptr, A.indices, A.data, field, rng.standard_normal(n),
                     [W.level(1 << 1, "jacobi")], "star_5000_600")


def test_hash_count_overflow_recount():
    s = _star_system()
    om = oracle_mgr(s)
    gs = gpu_solver(s)
    nr, nc, rp, ci, v = gs.export(0, 0, 1)
    o = om.export(0, 0, 1)
    lens = np.diff(rp)
    say(f"star: coarse operator {nr} rows, longest {lens.max()} (row {lens.argmax()})")
    assert lens.max() == 577 and lens.argmax() == 0
    assert np.array_equal(rp, o.rp) and np.array_equal(ci, o.ci)
    assert np.abs(v - o.v).max() <= 1e-10 * np.abs(o.v).max()
    assert gs.info() == om.info()
    xo, io = om.solve(s["rhs"])
    X, [ig] = gs.solve(s["rhs"])
    x = X.cpu().numpy()
    say(f"star: iters gpu {ig.iterations} oracle {io.iterations}, x err {rel(x, xo):.2e}")
    assert ig.status == 0 and abs(ig.iterations - io.iterations) <= 1 and elem_err(x, xo, s["field"]) <= 1e-8
    gs.close()


def _fan_system(nc=2000, nf=400, fan=12, seed=4):
    """A_c = A_CC + A_CF P_F as one fused hashed product (row bound 12 x 13 + 3
    = 159 <= 256) whose first symbolic pass, in tables of 64 slots, overflows on
    row 0 (C-point 0 reaches 12 F-points, each coupled to 12 other C-points):
    the product is counted again in tables sized for the bound."""
    rng = np.random.default_rng(seed)
    n = nc + nf
    rows, cols, vals = [], [], []

    def add(i, j, v):
        rows.append(i); cols.append(j); vals.append(v)

    for i in range(nc):
        add(i, i, 10.0 + rng.random())
        if i + 1 < nc:
            add(i, i + 1, -1.0); add(i + 1, i, -1.0)
    for k in range(nf):
        f = nc + k
        add(f, f, 10.0 + rng.random())
        if k < fan:
            nbrs = [0] + [1 + fan * k + t for t in range(fan)]
        else:
            nbrs = [(7 * k) % nc, (7 * k + 1) % nc]
        for c in nbrs:
            v = -0.1 * (0.5 + rng.random())
            add(f, c, v); add(c, f, v)
    A = sp.coo_matrix((vals, (rows, cols)), shape=(n, n)).tocsr()
    A.sum_duplicates()
    A.sort_indices()
    field = np.concatenate([np.zeros(nc, np.int32), np.ones(nf, np.int32)])
    return W._system(1, A.indptr, A.indices, A.data, field, rng.standard_normal(n),
                     [W.level(1 << 1, "jacobi")], "fan_2000_400")


def test_fused_coarse_product_count_overflow():
    s = _fan_system()
    om = oracle_mgr(s)
    gs = gpu_solver(s)
    nr, nc, rp, ci, v = gs.export(0, 0, 1)
    o = om.export(0, 0, 1)
    lens = np.diff(rp)
    say(f"fan: coarse operator {nr} rows, longest {lens.max()} (row {lens.argmax()})")
    assert lens.max() > 64 and lens.argmax() == 0
    assert np.array_equal(rp, o.rp) and np.array_equal(ci, o.ci) and np.array_equal(v, o.v)
    assert gs.info() == om.info()
    xo, io = om.solve(s["rhs"])
    X, [ig] = gs.solve(s["rhs"])
    x = X.cpu().numpy()
    say(f"fan: iters gpu {ig.iterations} oracle {io.iterations}, x err {rel(x, xo):.2e}")
    assert ig.status == 0 and abs(ig.iterations - io.iterations) <= 1 and elem_err(x, xo, s["field"]) <= 1e-8
    gs.close()
