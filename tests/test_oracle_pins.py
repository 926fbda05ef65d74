"""Pins for the FP64 oracle, each against something other than the oracle itself:
dense linear algebra, scipy products, closed forms from the paper (exact
inverse of MGR with ideal transfer operators, Schur-complement identities),
textbook facts (Luby MIS = greedy MIS for fixed priorities, constant
preservation of direct interpolation), the adjoint identity and finite
differences.  All run on the CPU."""
import os

import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O
import workloads as W
from oracle import LevelOpts
from _systems import perturbed_values as _perturbed

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rand_sparse(n, m, density, rng, diag=None):
    a = sp.random(n, m, density=density, random_state=rng, format="csr")
    a.data = rng.standard_normal(a.nnz)
    if diag is not None:
        a = a + sp.diags(np.full(n, diag))
    a = a.tocsr()
    a.sort_indices()
    return a


def lap1d(n):
    return sp.diags([-np.ones(n - 1), 2 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1]).tocsr()


def lap2d(nx):
    t = lap1d(nx)
    i = sp.identity(nx)
    return (sp.kron(t, i) + sp.kron(i, t)).tocsr()


# --------------------------------------------------------------------------- SpGEMM / add / transpose
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_spgemm_matches_dense_and_symbolic_pattern(seed):
    rng = np.random.default_rng(seed)
    a = rand_sparse(37, 23, 0.15, rng)
    b = rand_sparse(23, 41, 0.2, rng)
    c = O.spgemm(a, b)
    dense = a.toarray() @ b.toarray()
    np.testing.assert_allclose(c.to_scipy().toarray(), dense, rtol=1e-14, atol=1e-14)
    # symbolic pattern = boolean product (explicit zeros kept), columns sorted
    pat = (a.astype(bool).astype(int) @ b.astype(bool).astype(int)).toarray() > 0
    got = np.zeros_like(pat)
    for i in range(c.nr):
        cols = c.ci[c.rp[i]:c.rp[i + 1]]
        assert np.all(np.diff(cols) > 0)
        got[i, cols] = True
    assert np.array_equal(pat, got)


def test_spgemm_accumulation_order_is_gustavson():
    # (1e16 + 1) - 1e16 differs from 1e16 + (1 - 1e16): the order is fixed by the
    # left factor's column order (k ascending).
    a = sp.csr_matrix(np.array([[1.0, 1.0, 1.0]]))
    b = sp.csr_matrix(np.array([[1e16], [1.0], [-1e16]]))
    c = O.spgemm(a, b)
    assert c.v[0] == ((0.0 + 1e16) + 1.0) + -1e16


def test_add_and_transpose():
    rng = np.random.default_rng(5)
    a = rand_sparse(30, 20, 0.2, rng)
    b = rand_sparse(30, 20, 0.2, rng)
    np.testing.assert_array_equal(O.csr_add(a, b).to_scipy().toarray(), (a + b).toarray())
    t = O.transpose(a)
    np.testing.assert_array_equal(t.to_scipy().toarray(), a.T.toarray())


# --------------------------------------------------------------------------- dense kernels
def test_lu_solve_matches_numpy():
    rng = np.random.default_rng(3)
    m = rng.standard_normal((40, 40)) + 5 * np.eye(40)
    b = rng.standard_normal(40)
    x, st = O.lu_solve(m, b)
    assert st == 0
    np.testing.assert_allclose(x, np.linalg.solve(m, b), rtol=1e-12)
    xt, _ = O.lu_solve(m, b, trans=True)
    np.testing.assert_allclose(xt, np.linalg.solve(m.T, b), rtol=1e-12)


def test_lu_zero_pivot_detected():
    _, st = O.lu_solve(np.zeros((3, 3)), np.ones(3))
    assert st == -3


@pytest.mark.parametrize("bs", [1, 2, 3, 4])
def test_small_inverse(bs):
    rng = np.random.default_rng(bs)
    blk = rng.standard_normal((bs, bs)) + 3 * np.eye(bs)
    inv, st = O.small_inverse(blk)
    assert st == 0
    np.testing.assert_allclose(inv, np.linalg.inv(blk), rtol=1e-13, atol=1e-14)


# --------------------------------------------------------------------------- strength / PMIS
def test_strength_definition_by_hand():
    a = sp.csr_matrix(np.array([[4.0, -1.0, -0.2, 0.3], [-1.0, 4.0, -2.0, 0.0],
                                [0.0, 0.0, 1.0, 0.0], [-3.0, -0.5, 0.0, 5.0]]))
    a.sort_indices()
    s = O.strength(a, 0.25)
    # row 0: max(-a) = 1 -> strong iff -a >= 0.25: col1 yes, col2 no (0.2), col3 no
    # row 1: max = 2 -> threshold 0.5: col0 yes (1), col2 yes (2), col3 (0) no
    # row 2: no off-diagonals -> empty
    # row 3: max = 3 -> threshold .75: col0 yes, col1 no (0.5)
    expect = {(0, 1), (1, 0), (1, 2), (3, 0)}
    got = set()
    for i in range(4):
        for p in range(a.indptr[i], a.indptr[i + 1]):
            if s[p]:
                got.add((i, a.indices[p]))
    assert got == expect


def _greedy_mis(a, strong, w):
    """Sequential greedy MIS visiting points by decreasing (w, index): for a
    symmetric strength graph this equals Luby/PMIS with the same priorities."""
    n = a.shape[0]
    nbr = [set() for _ in range(n)]
    for i in range(n):
        for p in range(a.indptr[i], a.indptr[i + 1]):
            if strong[p]:
                nbr[i].add(a.indices[p])
                nbr[a.indices[p]].add(i)
    order = sorted(range(n), key=lambda i: (w[i], i), reverse=True)
    cf = np.full(n, -1)
    for i in order:
        if not nbr[i]:
            continue
        if all(cf[j] != 1 for j in nbr[i]):
            cf[i] = 1
    return cf


@pytest.mark.parametrize("seed", [11, 12, 13])
def test_pmis_equals_greedy_mis_on_symmetric_graphs(seed):
    a = lap2d(8)
    a.sort_indices()
    strong = O.strength(a, 0.25)
    cf, rounds = O.pmis(a, strong, seed)
    lam = np.bincount(a.indices[strong.astype(bool)], minlength=a.shape[0])
    w = lam + np.array([O.pmis_uniform(seed, 0, i) for i in range(a.shape[0])])
    assert np.array_equal(cf, _greedy_mis(a, strong, w))
    # maximal independent set: no two C neighbours, every F has a C neighbour
    for i in range(a.shape[0]):
        cols = a.indices[a.indptr[i]:a.indptr[i + 1]][strong[a.indptr[i]:a.indptr[i + 1]].astype(bool)]
        if cf[i] == 1:
            assert not np.any(cf[cols] == 1)
        else:
            assert np.any(cf[cols] == 1)
    assert rounds >= 1


def test_pmis_uniform_is_splitmix64():
    # splitmix64 reference value: first output for seed 0 is 0xE220A8397B1DCDAF
    # (Vigna's published test vector); k = (level << 32) + i + 1 with i = 0.
    u = O.pmis_uniform(0, 0, 0)
    assert u == (0xE220A8397B1DCDAF >> 11) * 2.0 ** -53


def test_pmis_nonsymmetric_invariants():
    rng = np.random.default_rng(4)
    a = rand_sparse(200, 200, 0.03, rng)
    a = (a - sp.diags(a.diagonal()) + sp.diags(np.full(200, 10.0))).tocsr()
    a.sort_indices()
    strong = O.strength(a, 0.25)
    cf, _ = O.pmis(a, strong, 99)
    lam = np.bincount(a.indices[strong.astype(bool)], minlength=200)
    assert set(np.unique(cf)) <= {-1, 1}
    for i in range(200):
        sl = slice(a.indptr[i], a.indptr[i + 1])
        s_i = a.indices[sl][strong[sl].astype(bool)]
        if lam[i] == 0:
            assert cf[i] == -1            # nobody depends on i -> F from the start
        elif cf[i] == -1:
            assert np.any(cf[s_i] == 1)   # made F by a C point it depends on


# --------------------------------------------------------------------------- direct interpolation
def _read_golden_interp():
    lines = [l.strip() for l in open(os.path.join(GOLDEN, "direct_interp_1d.txt")) if not l.startswith("#")]
    i = lines.index("matrix")
    rows = []
    j = i + 1
    while lines[j] != "cf":
        rows.append(lines[j]); j += 1
    cf = np.array([int(t) for t in lines[j + 1].split()])
    k = j + 2
    assert lines[k].startswith("expected_P")
    prow = lines[k + 1:k + 1 + len(rows)]
    n = len(rows)
    a = np.zeros((n, n))
    for r in rows:
        ri, rest = r.split(":", 1)
        for tok in rest.split():
            c, v = tok.split(":")
            a[int(ri), int(c)] = float(v)
    nc = int((cf == 1).sum())
    p = np.zeros((n, nc))
    for r in prow:
        ri, rest = r.split(":", 1)
        for tok in rest.split():
            c, v = tok.split(":")
            p[int(ri), int(c)] = float(v)
    return sp.csr_matrix(a), cf, p


def test_direct_interp_golden():
    a, cf, p_expect = _read_golden_interp()
    a.sort_indices()
    strong = O.strength(a, 0.25)
    p, st = O.direct_interp(a, strong, cf)
    assert st == 0
    np.testing.assert_allclose(p.to_scipy().toarray(), p_expect, rtol=1e-15)


def test_direct_interp_preserves_constants_on_zero_row_sum():
    n = 64
    a = lap1d(n).tolil()
    a[0, 0] = 1.0
    a[n - 1, n - 1] = 1.0           # Neumann ends: every row sums to zero
    a = a.tocsr(); a.sort_indices()
    strong = O.strength(a, 0.25)
    cf, _ = O.pmis(a, strong, 7)
    p, st = O.direct_interp(a, strong, cf)
    assert st == 0
    ps = p.to_scipy()
    s = ps @ np.ones(ps.shape[1])
    has = np.diff(p.rp) > 0
    np.testing.assert_allclose(s[has], 1.0, rtol=1e-14)
    for i in np.where(cf == 1)[0]:   # C rows are unit rows
        assert p.rp[i + 1] - p.rp[i] == 1 and p.v[p.rp[i]] == 1.0


# --------------------------------------------------------------------------- extended+i interpolation
def test_ext_interp_is_linear_interpolation_across_two_f_points():
    # 1-D Laplacian with the split C F F C F F C: every F-point has one strong
    # C-neighbour and one strong F-neighbour, whose other C-neighbour joins the
    # interpolatory set; extended+i then reproduces linear interpolation
    # (weights 2/3 and 1/3), which direct interpolation cannot (one C-point)
    n = 7
    a = lap1d(n)
    a.sort_indices()
    cf = np.array([1, -1, -1, 1, -1, -1, 1], np.int32)
    strong = O.strength(a, 0.25)
    p, st = O.ext_interp(a, strong, cf)
    assert st == 0
    expect = np.zeros((n, 3))
    expect[[0, 3, 6], [0, 1, 2]] = 1.0
    expect[1, :2] = [2 / 3, 1 / 3]
    expect[2, :2] = [1 / 3, 2 / 3]
    expect[4, 1:] = [2 / 3, 1 / 3]
    expect[5, 1:] = [1 / 3, 2 / 3]
    np.testing.assert_allclose(p.to_scipy().toarray(), expect, rtol=1e-15, atol=0)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_ext_interp_preserves_constants_on_zero_row_sum(seed):
    # graph Laplacian (random positive weights on a 2-D grid with diagonals):
    # with zero row sums the weights of every F-row add up to one
    rng = np.random.default_rng(seed)
    nx = 12
    idx = np.arange(nx * nx).reshape(nx, nx)
    pairs = [(idx[:, :-1], idx[:, 1:]), (idx[:-1, :], idx[1:, :]), (idx[:-1, :-1], idx[1:, 1:])]
    r = np.concatenate([u.ravel() for u, _ in pairs]); c = np.concatenate([v.ravel() for _, v in pairs])
    w = rng.uniform(0.1, 2.0, len(r))
    W_ = sp.coo_matrix((np.r_[w, w], (np.r_[r, c], np.r_[c, r])), shape=(nx * nx,) * 2).tocsr()
    a = (sp.diags(np.asarray(W_.sum(axis=1)).ravel()) - W_).tocsr()
    a.sort_indices()
    strong = O.strength(a, 0.25)
    cf, _ = O.pmis(a, strong, 3)
    p, st = O.ext_interp(a, strong, cf)
    assert st == 0
    ps = p.to_scipy()
    has = np.diff(p.rp) > 0
    np.testing.assert_allclose((ps @ np.ones(ps.shape[1]))[has], 1.0, rtol=1e-13)
    # the interpolatory set reaches distance two: some F-row interpolates from
    # a C-point that is not its neighbour
    nb = a.copy(); nb.data[:] = 1.0
    cols = np.where(cf == 1)[0]
    reach = (ps.toarray() != 0) & (nb.toarray()[:, cols] == 0)
    assert reach[cf != 1].any()


def test_ext_interp_equals_direct_where_all_neighbours_are_strong_c():
    # F-rows whose every off-diagonal coupling is negative and strong to a
    # C-point have F_i^s empty and nothing to lump: both formulas give
    # -a_ij / a_ii, to the last bit
    rng = np.random.default_rng(4)
    n = 41
    off = -rng.uniform(0.5, 1.5, n - 1)
    a = sp.diags([off, 2.5 + rng.uniform(0, 1, n), off * rng.uniform(0.8, 1.2, n - 1)], [-1, 0, 1]).tocsr()
    a.sort_indices()
    cf = np.where(np.arange(n) % 2 == 0, 1, -1).astype(np.int32)
    strong = O.strength(a, 0.25)
    pe, st = O.ext_interp(a, strong, cf)
    pd, st2 = O.direct_interp(a, strong, cf)
    assert st == 0 and st2 == 0
    assert np.array_equal(pe.rp, pd.rp) and np.array_equal(pe.ci, pd.ci) and np.array_equal(pe.v, pd.v)


def test_ext_interp_with_labels_ignores_other_labels():
    # two 1-D Laplacians interleaved (label 0 on even rows, 1 on odd rows) with
    # weak cross-label couplings: with labels, the strength, the interpolatory
    # sets and every sum of extended+i ignore the other label, so each label's
    # weights are those of its own Laplacian on its own
    rng = np.random.default_rng(6)
    m = 20
    parts = [lap1d(m).tolil(), lap1d(m).tolil()]
    for q in parts:
        for i in range(m):
            q[i, i] = 2.0 + rng.uniform(0.0, 0.2)
    n = 2 * m
    a = sp.lil_matrix((n, n))
    for lab in (0, 1):
        q = parts[lab].tocoo()
        a[2 * q.row + lab, 2 * q.col + lab] = q.data
    for i in range(m):                       # cross-label couplings, either sign
        a[2 * i, 2 * i + 1] = rng.uniform(-0.3, 0.3)
        a[2 * i + 1, 2 * i] = rng.uniform(-0.3, 0.3)
    a = a.tocsr(); a.sort_indices()
    label = np.arange(n) % 2
    cf1 = np.array([1 if i % 3 == 0 or i == m - 1 else -1 for i in range(m)], np.int32)
    cf = np.repeat(cf1, 2)                   # the same split on both labels
    p, st = O.ext_interp(a, O.strength(a, 0.25, label), cf, label)
    assert st == 0
    pd = p.to_scipy().toarray()
    for lab in (0, 1):
        q = parts[lab].tocsr(); q.sort_indices()
        ps, st2 = O.ext_interp(q, O.strength(q, 0.25), cf1)
        assert st2 == 0
        rows = np.arange(lab, n, 2)
        ccols = np.cumsum(cf == 1) - 1       # coarse index of each C-point
        cols = ccols[rows[cf1 == 1]]
        np.testing.assert_array_equal(pd[np.ix_(rows, cols)], ps.to_scipy().toarray())
        other = np.setdiff1d(np.arange(pd.shape[1]), cols)
        assert not pd[np.ix_(rows, other)].any()


def test_ext_interp_two_grid_and_fgmres_on_laplacians():
    # AMG with extended+i on the 2-D Laplacian behind a trivial MGR level:
    # FGMRES reaches 1e-10 quickly and agrees with a dense solve
    L = lap2d(24)
    A = sp.block_diag([sp.identity(3) * 2.0, L]).tocsr()
    A.sort_indices()
    n = A.shape[0]
    field = np.array([1] * 3 + [0] * (n - 3), np.int32)
    s = dict(b=1, rp=A.indptr.astype(np.int32), ci=A.indices.astype(np.int32), vals=A.data.copy(),
             field=field, n=n)
    lv = [dict(fmask=1 << 1, frelax="jacobi", sweeps=1, omega=1.0, restrict="injection",
               amg_unknown_based=False)]
    b = np.random.default_rng(2).standard_normal(n)
    its = {}
    for interp in ("direct", "ext+i"):
        m = build(s, levels=lv, max_coarse=16, interp=interp)
        x, info = m.solve(b, rtol=1e-10)
        assert info.status == 0
        np.testing.assert_allclose(x, np.linalg.solve(A.toarray(), b), rtol=1e-8, atol=1e-9)
        its[interp] = info.iterations
    assert its["ext+i"] <= its["direct"]


# --------------------------------------------------------------------------- whole MGR: exactness pins
def small_mimetic(n=3, consistent=True, upwind=True, seed=5):
    return W.hybrid_mimetic(n, n, n, seed=seed, consistent=consistent, upwind=upwind)


def build(sys_, levels=None, **kw):
    lv = [LevelOpts(**l) for l in (levels or sys_["levels"])]
    m = O.MGR(sys_["b"], sys_["rp"], sys_["ci"], sys_["vals"], sys_["field"], lv, **kw)
    assert m.status == 0, m.status
    return m


@pytest.mark.parametrize("consistent", [True, False])
def test_exact_inverse_ideal_interp_diagonal_aff(consistent):
    # F = cells: A_FF diagonal, so Jacobi P is the ideal P of eq. (3), the Jacobi
    # F-relaxation is exact, and the coarse system (108 faces <= max_coarse) is
    # solved exactly by LU: MGR is then A^{-1} (block LDU of eq. (2)).
    s = small_mimetic(consistent=consistent)
    m = build(s)
    A = W.csr_of(s).toarray()
    rng = np.random.default_rng(0)
    for _ in range(3):
        v = rng.standard_normal(s["n"])
        z = m.apply(v)
        ref = np.linalg.solve(A, v)
        assert np.linalg.norm(z - ref) <= 1e-12 * np.linalg.norm(ref)
    x, info = m.solve(s["rhs"], rtol=1e-12)
    assert info.iterations == 1 and info.status == 0


def block_diag_ff_system(nb=12, bs=3, nc=40, seed=0):
    """Random system whose F-F block is block diagonal (bs x bs per block row)."""
    rng = np.random.default_rng(seed)
    b = bs + 1                     # block row = bs F-dofs + 1 C-dof
    nbr = nb
    n = nbr * b
    A = np.zeros((n, n))
    for I in range(nbr):
        blk = rng.standard_normal((b, b)) + 4 * np.eye(b)
        A[I * b:(I + 1) * b, I * b:(I + 1) * b] = blk
    # couplings only through the C-dof (index bs within each block) rows/cols
    for _ in range(3 * nbr):
        I, J = rng.integers(0, nbr, 2)
        if I == J:
            continue
        r = rng.integers(0, b)
        A[I * b + r, J * b + bs] += rng.standard_normal() * 0.3
        A[J * b + bs, I * b + rng.integers(0, b)] += rng.standard_normal() * 0.3
    Ab = sp.bsr_matrix(A, blocksize=(b, b))
    Ab.sort_indices()
    field = np.tile(np.array([1] * bs + [0]), nbr)
    return dict(b=b, rp=Ab.indptr.astype(np.int32), ci=Ab.indices.astype(np.int32),
                vals=Ab.data.reshape(-1).copy(), field=field.astype(np.int32), n=n, A=A)


def test_exact_inverse_block_jacobi_on_block_diagonal_aff():
    s = block_diag_ff_system()
    lv = [dict(fmask=1 << 1, frelax="block_jacobi", sweeps=1, omega=1.0, restrict="injection",
               amg_unknown_based=False)]
    m = build(s, levels=lv)
    v = np.random.default_rng(1).standard_normal(s["n"])
    z = m.apply(v)
    ref = np.linalg.solve(s["A"], v)
    assert np.linalg.norm(z - ref) <= 1e-12 * np.linalg.norm(ref)
    # the same with Jacobi restriction (any R works with ideal P and exact solves)
    lv[0]["restrict"] = "jacobi"
    m2 = build(s, levels=lv)
    z2 = m2.apply(v)
    assert np.linalg.norm(z2 - ref) <= 1e-12 * np.linalg.norm(ref)


def _dense_blocks(s, lvl=0, m=None):
    A = W.csr_of(s).toarray()
    isF = np.array([(s["levels"][lvl]["fmask"] >> f) & 1 for f in s["field"]], bool)
    F, C = np.where(isF)[0], np.where(~isF)[0]
    return A, F, C


def test_schur_identity_injection_jacobi_p():
    # eq. (4) with injection R: A_c = A_CC - A_CF D_FF^{-1} A_FC (text after eq. (9))
    s = W.two_field_tpfa(3, 3, 2, seed=3)
    m = build(s)
    A, F, C = _dense_blocks(s)
    D = np.diag(np.diag(A[np.ix_(F, F)]))
    expect = A[np.ix_(C, C)] - A[np.ix_(C, F)] @ np.linalg.inv(D) @ A[np.ix_(F, C)]
    ac = m.export(0, 0, 1).to_scipy().toarray()
    np.testing.assert_allclose(ac, expect, rtol=1e-13, atol=1e-13 * np.abs(expect).max())


def test_mgr_pi_on_tpfa_mimetic_is_the_exact_cell_schur_complement():
    # MGR_Pi of Sec. 3.1 (F = faces, C = cells): in the TPFA variant A_pipi is
    # diagonal, so Jacobi P is the ideal P of eq. (3), the coarse system is
    # S = A_pp - A_ppi A_pipi^-1 A_pip, and S couples a cell only with the cells
    # that share one of its faces (7 points)
    nx, ny, nz = 4, 3, 3
    s = W.hybrid_mimetic(nx, ny, nz, seed=6, consistent=False, reduction="pi")
    m = build(s)
    A, F, C = _dense_blocks(s)
    assert len(C) == nx * ny * nz and np.all(s["field"][C] == 0)
    AFF = A[np.ix_(F, F)]
    assert np.count_nonzero(AFF - np.diag(np.diag(AFF))) == 0
    expect = A[np.ix_(C, C)] - A[np.ix_(C, F)] @ np.linalg.inv(AFF) @ A[np.ix_(F, C)]
    ac = m.export(0, 0, 1).to_scipy()
    np.testing.assert_allclose(ac.toarray(), expect, rtol=1e-13, atol=1e-13 * np.abs(expect).max())
    # brute-force 7-point pattern of the cell grid (cells numbered x fastest)
    pattern = set()
    for c in range(nx * ny * nz):
        x, y, z = c % nx, (c // nx) % ny, c // (nx * ny)
        for dx, dy, dz in [(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)]:
            if 0 <= x + dx < nx and 0 <= y + dy < ny and 0 <= z + dz < nz:
                pattern.add((c, (x + dx) + nx * ((y + dy) + ny * (z + dz))))
    coo = ac.tocoo()
    assert set(zip(coo.row.tolist(), coo.col.tolist())) == pattern


@pytest.mark.parametrize("reduction", ["p", "pi"])
def test_mgr_p_and_mgr_pi_exact_on_tpfa_mimetic(reduction):
    # both reductions of Sec. 3.1 eliminate a diagonal block in the TPFA
    # variant; with the coarse grid solved by LU (108 faces or 27 cells, both
    # <= max_coarse) MGR is A^{-1} and FGMRES takes one iteration
    s = W.hybrid_mimetic(3, 3, 3, seed=7, consistent=False, reduction=reduction)
    m = build(s)
    A = W.csr_of(s).toarray()
    v = np.random.default_rng(8).standard_normal(s["n"])
    ref = np.linalg.solve(A, v)
    assert np.linalg.norm(m.apply(v) - ref) <= 1e-12 * np.linalg.norm(ref)
    x, info = m.solve(s["rhs"], rtol=1e-12)
    assert info.iterations == 1 and info.status == 0


def test_four_level_system_structure():
    # the generator's structure that the reduction order relies on (Sec. 3.2):
    # rho_2 rows couple only inside their cell, and every pressure-controlled
    # well leaves a zero on the diagonal of the well block
    s = W.compositional_4level(5, 4, 3, seed=2, wells_per_axis=2)
    A = W.csr_of(s).tocoo()
    cell = np.arange(s["n"]) // 3
    rho2 = (s["field"][A.row] == 2) & (A.data != 0.0)   # stored zeros of the 3x3 blocks aside
    assert np.all(cell[A.row[rho2]] == cell[A.col[rho2]])
    d = W.csr_of(s).diagonal()
    q_rows = np.where(s["field"] == 4)[0]
    assert np.sum(d[q_rows] == 0.0) == s["nwells"] // 2


def test_four_level_first_reduction_is_the_exact_schur_complement():
    # level 1 eliminates rho_2 (+ padding), whose block is diagonal: Jacobi P is
    # the ideal P of eq. (3) and A_c = A_CC - A_CF A_FF^{-1} A_FC exactly
    s = W.compositional_4level(5, 4, 3, seed=3, wells_per_axis=2)
    m = build(s)
    A, F, C = _dense_blocks(s)
    AFF = A[np.ix_(F, F)]
    assert np.count_nonzero(AFF - np.diag(np.diag(AFF))) == 0
    expect = A[np.ix_(C, C)] - A[np.ix_(C, F)] @ np.linalg.inv(AFF) @ A[np.ix_(F, C)]
    ac = m.export(0, 0, 1).to_scipy().toarray()
    np.testing.assert_allclose(ac, expect, rtol=1e-13, atol=1e-13 * np.abs(expect).max())


def test_four_level_exact_with_exact_coarse_solve():
    # only the first (exact) level, and a coarse grid small enough for the
    # pivoted LU (which must cope with the zero well diagonals): MGR = A^{-1}
    s = W.compositional_4level(4, 4, 2, seed=4, wells_per_axis=2)
    m = build(s, levels=s["levels"][:1], max_coarse=128)
    assert m.info()["amg_levels"] == [(s["n"] - 32 - 4, m.info()["amg_levels"][0][1])]
    A = W.csr_of(s).toarray()
    v = np.random.default_rng(7).standard_normal(s["n"])
    ref = np.linalg.solve(A, v)
    assert np.linalg.norm(m.apply(v) - ref) <= 1e-11 * np.linalg.norm(ref)


def test_four_level_fgmres_matches_direct_solve():
    import scipy.sparse.linalg as spla
    s = W.compositional_4level(10, 9, 8, seed=5, wells_per_axis=2)
    m = build(s)
    assert [l[0] for l in m.info()["mgr_levels"]] == [s["n"], s["n"] - 4 - 720, 728]
    x, info = m.solve(s["rhs"])
    xd = spla.spsolve(W.csr_of(s).tocsc(), s["rhs"])
    assert info.status == 0 and info.iterations <= 15
    assert np.linalg.norm(x - xd) <= 1e-7 * np.linalg.norm(xd)


def test_rap_equals_literal_triple_product_jacobi_r():
    # eq. (5) restriction: A_c = R A P with the full R = [-A_CF D^{-1}, I], P = [-D^{-1} A_FC; I]
    s = W.two_field_tpfa(3, 2, 2, seed=4)
    lv = [dict(s["levels"][0], restrict="jacobi")]
    m = build(s, levels=lv)
    A, F, C = _dense_blocks(s)
    n = A.shape[0]
    Dinv = np.diag(1.0 / np.diag(A[np.ix_(F, F)]))
    P = np.zeros((n, len(C))); P[C, np.arange(len(C))] = 1.0
    P[F, :] = -Dinv @ A[np.ix_(F, C)]
    R = np.zeros((len(C), n)); R[np.arange(len(C)), C] = 1.0
    R[:, F] = -A[np.ix_(C, F)] @ Dinv
    expect = R @ A @ P
    ac = m.export(0, 0, 1).to_scipy().toarray()
    np.testing.assert_allclose(ac, expect, rtol=1e-12, atol=1e-12 * np.abs(expect).max())


def test_one_level_closed_form_matches_block_ldu_approximation():
    # With Jacobi P, injection R, one Jacobi sweep from zero and an exact coarse
    # solve, Algorithm 1 gives z = [D^{-1}(v_F - A_FC e); e], e = S~^{-1}(v_C - A_CF D^{-1} v_F)
    s = W.two_field_tpfa(3, 3, 2, seed=8)
    m = build(s, max_coarse=128)
    A, F, C = _dense_blocks(s)
    D = np.diag(A[np.ix_(F, F)])
    S = A[np.ix_(C, C)] - A[np.ix_(C, F)] @ (A[np.ix_(F, C)] / D[:, None])
    v = np.random.default_rng(2).standard_normal(A.shape[0])
    e = np.linalg.solve(S, v[C] - A[np.ix_(C, F)] @ (v[F] / D))
    z = np.zeros_like(v)
    z[C] = e
    z[F] = (v[F] - A[np.ix_(F, C)] @ e) / D
    np.testing.assert_allclose(m.apply(v), z, rtol=1e-11, atol=1e-12 * np.abs(z).max())


# --------------------------------------------------------------------------- FGMRES
@pytest.mark.parametrize("gen", ["tpfa", "mimetic"])
def test_fgmres_solution_matches_dense_solve(gen):
    s = W.two_field_tpfa(6, 5, 4, seed=2) if gen == "tpfa" else W.hybrid_mimetic(5, 4, 4, seed=2)
    m = build(s, max_coarse=16)
    x, info = m.solve(s["rhs"], rtol=1e-12)
    assert info.status == 0
    ref = np.linalg.solve(W.csr_of(s).toarray(), s["rhs"])
    assert np.linalg.norm(x - ref) <= 1e-9 * np.linalg.norm(ref)
    assert info.rel_res_true <= 1e-12


def test_fgmres_restart_and_mgs_agree():
    s = W.two_field_tpfa(8, 8, 4, seed=6)
    m = build(s, max_coarse=16)
    x1, i1 = m.solve(s["rhs"], rtol=1e-10)
    x2, i2 = m.solve(s["rhs"], rtol=1e-10, mgs=True)
    x3, i3 = m.solve(s["rhs"], rtol=1e-10, restart=7)
    assert abs(i1.iterations - i2.iterations) <= 1
    assert i3.restarts >= 1 and i3.status == 0
    A = W.csr_of(s)
    for x in (x1, x2, x3):
        assert np.linalg.norm(s["rhs"] - A @ x) <= 1.01e-10 * np.linalg.norm(s["rhs"])


def test_fgmres_zero_rhs_and_maxiter():
    s = W.two_field_tpfa(4, 4, 4, seed=6)
    m = build(s)
    x, info = m.solve(np.zeros(s["n"]))
    assert info.status == 0 and info.iterations == 0 and not x.any()
    x, info = m.solve(s["rhs"], maxiter=2)
    assert info.status == 1 and info.iterations == 2


# --------------------------------------------------------------------------- transpose apply / adjoint
LEVEL_VARIANTS = [
    dict(frelax="jacobi", restrict="injection"),
    dict(frelax="jacobi", restrict="jacobi"),
    dict(frelax="jacobi", restrict="injection", omega=0.7),
    dict(frelax="ilu0", restrict="injection"),
    dict(frelax="amg", restrict="injection"),
]


@pytest.mark.parametrize("variant", range(len(LEVEL_VARIANTS)))
def test_transpose_apply_dot_product_identity(variant):
    s = W.two_field_tpfa(6, 6, 5, seed=9)
    lv = [dict(s["levels"][0], **LEVEL_VARIANTS[variant])]
    m = build(s, levels=lv, max_coarse=20)
    rng = np.random.default_rng(variant)
    u, v = rng.standard_normal(s["n"]), rng.standard_normal(s["n"])
    lhs = u @ m.apply(v)
    rhs = m.apply(u, trans=True) @ v
    assert abs(lhs - rhs) <= 1e-13 * (abs(lhs) + np.linalg.norm(u) * np.linalg.norm(v) * 1e-3)


def test_transpose_apply_matches_dense_transpose_of_operator():
    s = W.hybrid_mimetic(3, 3, 2, seed=3)
    m = build(s, max_coarse=8)
    n = s["n"]
    M = np.stack([m.apply(e) for e in np.eye(n)], axis=1)
    MT = np.stack([m.apply(e, trans=True) for e in np.eye(n)], axis=1)
    np.testing.assert_allclose(MT, M.T, rtol=1e-11, atol=1e-13 * np.abs(M).max())


def test_adjoint_identity_and_finite_differences():
    s = W.hybrid_mimetic(4, 3, 3, seed=7)
    m = build(s)
    rng = np.random.default_rng(17)
    c = rng.standard_normal(s["n"])
    x, i1 = m.solve(s["rhs"], rtol=1e-14, maxiter=400)
    lam, i2 = m.solve(c, trans=True, rtol=1e-14, maxiter=400)
    # <lambda, b> = <c, x> = c^T A^{-1} b
    assert abs(lam @ s["rhs"] - c @ x) <= 1e-11 * abs(c @ x)
    g = O.grad_values(1, s["rp"], s["ci"], lam, x)
    h = 1e-6
    for k in rng.choice(len(s["vals"]), 20, replace=False):
        vp = s["vals"].copy(); vp[k] += h
        vm = s["vals"].copy(); vm[k] -= h
        Ap = sp.csr_matrix((vp, s["ci"], s["rp"])); Am = sp.csr_matrix((vm, s["ci"], s["rp"]))
        fd = (c @ np.linalg.solve(Ap.toarray(), s["rhs"]) - c @ np.linalg.solve(Am.toarray(), s["rhs"])) / (2 * h)
        assert abs(g[k] - fd) <= 1e-6 * max(abs(fd), 1e-3 * np.abs(g).max())


def test_two_grid_amg_on_1d_laplacian_converges():
    # AMG alone (no MGR level would apply): wrap the Laplacian as a system whose
    # only MGR level eliminates a trivially decoupled diagonal field, so the
    # coarse AMG sees the Laplacian; V-cycle convergence factor well below 1.
    n = 257
    L = lap1d(n)
    A = sp.block_diag([sp.identity(3) * 2.0, L]).tocsr()
    A.sort_indices()
    field = np.array([1] * 3 + [0] * n, np.int32)
    s = dict(b=1, rp=A.indptr.astype(np.int32), ci=A.indices.astype(np.int32), vals=A.data.copy(),
             field=field, n=n + 3)
    lv = [dict(fmask=1 << 1, frelax="jacobi", sweeps=1, omega=1.0, restrict="injection",
               amg_unknown_based=False)]
    m = build(s, levels=lv, max_coarse=16)
    x, info = m.solve(np.random.default_rng(1).standard_normal(n + 3), rtol=1e-10)
    assert info.status == 0 and info.iterations < 40


# --------------------------------------------------------------------------- setup reuse (Sec. 3.3, Sec. 4.4)
def test_reuse_with_unchanged_values_is_the_same_hierarchy():
    s = W.two_field_tpfa(7, 6, 5, seed=11)
    m = build(s)
    m2 = m.update(s["vals"])
    assert m2.status == 0 and m2.info() == m.info()
    for k in range(len(m.info()["amg_levels"])):
        a, b = m.export(1, k, 1), m2.export(1, k, 1)
        assert np.array_equal(a.ci, b.ci) and np.array_equal(a.v, b.v)
    v = np.random.default_rng(2).standard_normal(s["n"])
    assert np.array_equal(m.apply(v), m2.apply(v))


def test_reuse_keeps_interpolation_and_forms_galerkin_products_anew():
    s = W.two_field_tpfa(9, 8, 7, seed=12)
    m = build(s)
    vals2 = _perturbed(s, seed=3)
    s2 = dict(s, vals=vals2)
    r = m.update(vals2)
    fresh = build(s2)
    assert r.status == 0
    # MGR levels do not depend on the AMG: equal to a fresh setup, bit for bit
    for what in (1, 2, 5):
        a, b = r.export(0, 0, what), fresh.export(0, 0, what)
        assert np.array_equal(a.ci, b.ci) and np.array_equal(a.v, b.v)
    nl = len(m.info()["amg_levels"])
    for k in range(nl - 1):
        assert np.array_equal(r.export(1, k, 0), m.export(1, k, 0))          # C/F split kept
        P = m.export(1, k, 2).to_scipy()
        assert np.array_equal(r.export(1, k, 2).to_scipy().toarray(), P.toarray())   # P kept
        Ak = r.export(1, k, 1).to_scipy()
        expect = (P.T @ (Ak @ P)).toarray()                                  # Galerkin product of the new values
        got = r.export(1, k + 1, 1).to_scipy().toarray()
        np.testing.assert_allclose(got, expect, rtol=1e-12, atol=1e-12 * np.abs(expect).max())
    x, info = r.solve(s2["rhs"])
    A2 = W.csr_of(s2)
    assert info.status == 0 and np.linalg.norm(s2["rhs"] - A2 @ x) <= 1e-8 * np.linalg.norm(s2["rhs"])


def test_reuse_keeping_the_frelaxation_amg_whole_equals_a_fresh_setup():
    # fracturing: only the fracture (pressure) rows change, so A_uu -- the F-block
    # relaxed by AMG -- is the same and its whole hierarchy can be kept (Sec. 3.3)
    s = W.fracturing(9, seed=5)
    opts = s["solver_opts"]
    m = build(s, **opts)
    vals2 = _perturbed(s, seed=4, rows_field=3)
    s2 = dict(s, vals=vals2)
    r = m.update(vals2, keep_frelax_amg=True)
    fresh = build(s2, **opts)
    assert r.status == 0 and r.info() == fresh.info()
    k = 0
    while True:
        try:
            a = fresh.export(2, k, 1, sub=0)
        except KeyError:
            break
        b = r.export(2, k, 1, sub=0)
        assert np.array_equal(a.ci, b.ci) and np.array_equal(a.v, b.v)
        k += 1
    assert k >= 2
    v = np.random.default_rng(5).standard_normal(s["n"])
    assert np.array_equal(r.apply(v), fresh.apply(v)) or \
        np.linalg.norm(r.apply(v) - fresh.apply(v)) <= 1e-12 * np.linalg.norm(fresh.apply(v))
