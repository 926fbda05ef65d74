"""Pins for the oracle's aggressive coarsening and multi-pass interpolation (the
first level of the mechanics AMG, Sec. 4.1; Stueben 2001), each against
something other than the oracle's own loops:

* the aggressive split is the greedy maximal independent set, in decreasing
  (weight, index) order, of the distance-two strong graph on the first PMIS
  C-points, built here by brute force (Luby's selection on a symmetric graph);
  final C-points are never within two strong connections of each other;
* multi-pass interpolation on hand-worked 1-D examples (two and three
  passes);
* it equals direct interpolation when every F-point has a strong C-neighbour;
* it preserves constants for a zero-row-sum M-matrix (every row of P sums to
  one);
* an AMG level coarsened aggressively exports exactly that split and P, and
  its coarse operator is the Galerkin product."""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O
from test_oracle_pins import lap2d
from test_oracle_pins_relax import amg_only, hierarchy


def strong_graph(a, strong):
    n = a.shape[0]
    nbr = [set() for _ in range(n)]
    for i in range(n):
        for p in range(a.indptr[i], a.indptr[i + 1]):
            if strong[p]:
                nbr[i].add(int(a.indices[p]))
    return nbr


def expected_aggressive(a, strong, seed, level):
    cf1, _ = O.pmis(a, strong, seed, level)
    S = strong_graph(a, strong)
    c1 = [i for i in range(a.shape[0]) if cf1[i] == 1]
    pos = {i: k for k, i in enumerate(c1)}
    T = []
    for i in c1:
        reach = set(S[i])
        for k in S[i]:
            reach |= S[k]
        T.append(sorted(pos[j] for j in reach if j in pos and j != i))
    n1 = len(c1)
    lam = np.zeros(n1)
    for row in T:
        for j in row:
            lam[j] += 1
    w = lam + np.array([O.pmis_uniform(seed, level + 64, k) for k in range(n1)])
    adj = [set(row) for row in T]
    for k, row in enumerate(T):
        for j in row:
            adj[j].add(k)
    c2 = np.full(n1, -1)
    for k in sorted(range(n1), key=lambda k: (w[k], k), reverse=True):
        if adj[k] and all(c2[j] != 1 for j in adj[k]):
            c2[k] = 1
    cf = np.full(a.shape[0], -1)
    for k, i in enumerate(c1):
        if c2[k] == 1:
            cf[i] = 1
    return cf, cf1, S


def lap3d(m):
    e = np.ones(m)
    t = sp.diags([-e[:-1], 2 * e, -e[:-1]], [-1, 0, 1])
    i = sp.identity(m)
    return (sp.kron(sp.kron(t, i), i) + sp.kron(sp.kron(i, t), i) + sp.kron(sp.kron(i, i), t)).tocsr()


@pytest.mark.parametrize("seed", [3, 4])
@pytest.mark.parametrize("mat", ["lap2d", "lap3d"])
def test_aggressive_split_is_greedy_mis_of_the_distance_two_graph(mat, seed):
    a = lap2d(13) if mat == "lap2d" else lap3d(7)
    a = sp.csr_matrix(a)
    a.sort_indices()
    strong = O.strength(a, 0.25)
    cf = O.aggressive_split(a, strong, seed, 0)
    exp, cf1, S = expected_aggressive(a, strong, seed, 0)
    assert np.array_equal(cf, exp)
    c = np.flatnonzero(cf == 1)
    assert 0 < len(c) < np.count_nonzero(cf1 == 1)
    assert np.all(cf1[c] == 1)
    cs = set(c.tolist())
    for i in c:
        two = set(S[i])
        for k in S[i]:
            two |= S[k]
        assert not (two - {i}) & cs


def tridiag(n):
    e = np.ones(n)
    a = sp.diags([-e[:-1], 2 * e, -e[:-1]], [-1, 0, 1]).tocsr()
    a.sort_indices()
    return a


def test_multipass_two_passes_by_hand():
    # C = {0, 4, 8}: points 1, 3, 5, 7 get direct interpolation (one C-neighbour:
    # alpha = -2 / -1 = 2, w = -(2 * -1) / 2 = 1); points 2 and 6 have only
    # F-neighbours, both interpolated in pass 1: alpha = 1, w = 1/2 each
    a = tridiag(9)
    strong = O.strength(a, 0.25)
    cf = np.array([1, -1, -1, -1, 1, -1, -1, -1, 1])
    P, st = O.multipass_interp(a, strong, cf)
    assert st == 0
    expect = np.zeros((9, 3))
    expect[[0, 1], 0] = 1
    expect[[3, 4, 5], 1] = 1
    expect[[7, 8], 2] = 1
    expect[2, [0, 1]] = 0.5
    expect[6, [1, 2]] = 0.5
    assert np.array_equal(P.to_scipy().toarray(), expect)


def test_multipass_three_passes_by_hand():
    # C = {0, 6}: pass 1 reaches 1 and 5; pass 2 reaches 2 (only neighbour 1 is
    # interpolated: alpha = 2, w = 1) and 4; pass 3 reaches 3 (neighbours 2 and 4)
    a = tridiag(7)
    strong = O.strength(a, 0.25)
    cf = np.array([1, -1, -1, -1, -1, -1, 1])
    P, st = O.multipass_interp(a, strong, cf)
    assert st == 0
    expect = np.zeros((7, 2))
    expect[[0, 1, 2], 0] = 1
    expect[[4, 5, 6], 1] = 1
    expect[3] = [0.5, 0.5]
    assert np.array_equal(P.to_scipy().toarray(), expect)


def test_multipass_equals_direct_when_every_f_point_has_a_strong_c_neighbour():
    a = lap2d(11) + 0.2 * sp.kron(sp.identity(11), sp.diags([-np.ones(10)], [1]))
    a = sp.csr_matrix(a)
    a.sort_indices()
    strong = O.strength(a, 0.25)
    cf, _ = O.pmis(a, strong, 7)
    Pd, _ = O.direct_interp(a, strong, cf)
    Pm, _ = O.multipass_interp(a, strong, cf)
    assert np.array_equal(Pd.rp, Pm.rp) and np.array_equal(Pd.ci, Pm.ci) and np.array_equal(Pd.v, Pm.v)


def test_multipass_preserves_constants_on_a_zero_row_sum_matrix():
    m = 12
    e = np.ones(m)
    t = sp.diags([-e[:-1], 2 * e, -e[:-1]], [-1, 0, 1]).tolil()
    t[0, m - 1] = t[m - 1, 0] = -1            # periodic: zero row sums
    t = t.tocsr()
    a = (sp.kron(t, sp.identity(m)) + sp.kron(sp.identity(m), t)).tocsr()
    a.sort_indices()
    strong = O.strength(a, 0.25)
    cf = O.aggressive_split(a, strong, 5, 0)
    P, st = O.multipass_interp(a, strong, cf)
    assert st == 0
    rows = P.to_scipy() @ np.ones(P.nc)
    np.testing.assert_allclose(rows, 1.0, rtol=0, atol=1e-14)


def test_aggressive_level_in_the_amg_hierarchy():
    nx = 16
    a = lap2d(nx) + 0.05 * sp.identity(nx * nx)
    m, s = amg_only(a, max_coarse=10, agg_levels=1)
    m0, _ = amg_only(a, max_coarse=10)
    a = sp.csr_matrix(a)
    a.sort_indices()
    strong = O.strength(a, 0.25)
    cf = O.aggressive_split(a, strong, 12345, 0)
    assert np.array_equal(m.export(1, 0, 0), cf)
    P, _ = O.multipass_interp(a, strong, cf)
    Pe = m.export(1, 0, 2)
    assert np.array_equal(Pe.rp, P.rp) and np.array_equal(Pe.ci, P.ci) and np.array_equal(Pe.v, P.v)
    As, Ps = hierarchy(m)
    np.testing.assert_allclose(As[1], Ps[0].T @ As[0] @ Ps[0], rtol=1e-12, atol=1e-13)
    # only the first level is aggressive: far fewer coarse points there than with PMIS
    assert m.info()["amg_levels"][1][0] < 0.6 * m0.info()["amg_levels"][1][0]
