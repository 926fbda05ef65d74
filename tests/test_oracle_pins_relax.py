"""Pins for the oracle's relaxation parts, each against a closed form computed
with dense linear algebra (numpy), not against the oracle's own steps:

* ILU(0) (an F-solver option, Sec. 2, the guidance after Algorithm 1): the
  factors L (unit lower) and U live on the pattern of A and reproduce A on
  that pattern, (LU)_ij = a_ij, which fixes them uniquely; with no fill
  (tridiagonal A) the solve is exact; the transposed solve is (LU)^{-T}.
* F-relaxation with nu sweeps and weight omega (Algorithm 1's F-relaxation
  step, repeated): from z = 0 the F-part after nu sweeps is
  [I - (I - omega M A_FF)^nu] A_FF^{-1} v_F, and the whole one-level cycle
  with an exact coarse solve has the block form of eqs. (2)-(5).
* The AMG V(nu_pre, nu_post) cycle of the coarse solve (Sec. 4.1, with
  L1-Jacobi smoothing): its error propagation is
  E_k = S_k^{nu_post} (I - P_k B_{k+1} P_k^T A_k) S_k^{nu_pre},
  S_k = I - D_k^{-1} A_k, B_k = (I - E_k) A_k^{-1}, B_coarsest = A^{-1}; the
  cycle applied to v must equal B_0 v (and its transpose B_0^T v)."""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O
import workloads as W
from oracle import LevelOpts


def lap1d(n):
    return sp.diags([-np.ones(n - 1), 2 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1]).tocsr()


def lap2d(nx, ny=None):
    ny = ny or nx
    return (sp.kron(lap1d(ny), sp.identity(nx)) + sp.kron(sp.identity(ny), lap1d(nx))).tocsr()


def random_pattern_matrix(n, density, seed, sym_pattern=True):
    """Nonsymmetric values, diagonally dominant, on a random pattern with the diagonal."""
    rng = np.random.default_rng(seed)
    m = sp.random(n, n, density=density, random_state=rng, format="csr")
    if sym_pattern:
        m = m + m.T
    m = m.tocsr()
    m.data = rng.uniform(-1.0, 1.0, m.nnz)
    rs = np.asarray(abs(m).sum(axis=1)).ravel()
    m = (m + sp.diags(rs + rng.uniform(0.5, 1.5, n))).tocsr()
    m.sort_indices()
    return m


def lu_dense(a, lu, diag):
    """Dense unit-lower L and upper U from the factor values on a's pattern."""
    n = a.shape[0]
    L, U = np.eye(n), np.zeros((n, n))
    for i in range(n):
        for p in range(a.indptr[i], a.indptr[i + 1]):
            j = a.indices[p]
            if j < i:
                L[i, j] = lu[p]
            else:
                U[i, j] = lu[p]
    return L, U


# --------------------------------------------------------------------------- ILU(0)
@pytest.mark.parametrize("case", ["lap2d", "random_sym_pattern", "random_nonsym_pattern"])
def test_ilu0_reproduces_a_on_its_pattern(case):
    if case == "lap2d":
        a = lap2d(7, 6)
    else:
        a = random_pattern_matrix(60, 0.06, seed=3, sym_pattern=(case == "random_sym_pattern"))
    a.sort_indices()
    lu, diag, st = O.ilu0(a)
    assert st == 0
    L, U = lu_dense(a, lu, diag)
    LU = L @ U
    A = a.toarray()
    pat = A != 0
    np.fill_diagonal(pat, True)
    scale = np.abs(A).max()
    # the defining property: (LU)_ij = a_ij for every (i, j) in the pattern
    assert np.abs(LU - A)[pat].max() <= 1e-13 * scale
    # and the product does have fill outside it (so the check is not vacuous)
    assert np.abs(LU)[~pat].max() > 1e-3 * scale
    # the diagonal positions point at the diagonal entries
    for i in range(a.shape[0]):
        assert a.indices[diag[i]] == i


def test_ilu0_without_fill_is_the_exact_lu():
    a = random_pattern_matrix(40, 0.0, seed=5) + sp.diags([np.linspace(-1, 1, 39), np.linspace(0.5, -0.5, 39)],
                                                          [-1, 1])
    a = sp.csr_matrix(a)
    a.sort_indices()
    lu, diag, st = O.ilu0(a)
    assert st == 0
    A = a.toarray()
    r = np.random.default_rng(4).standard_normal(a.shape[0])
    for tr in (False, True):
        z = O.ilu0_solve(a, lu, diag, r, trans=tr)
        ref = np.linalg.solve(A.T if tr else A, r)
        assert np.linalg.norm(z - ref) <= 1e-13 * np.linalg.norm(ref)


def test_ilu0_solves_with_the_factors():
    a = lap2d(6, 5) + sp.diags(np.linspace(0.1, 0.3, 30))
    a = sp.csr_matrix(a)
    a.sort_indices()
    lu, diag, st = O.ilu0(a)
    L, U = lu_dense(a, lu, diag)
    r = np.random.default_rng(6).standard_normal(30)
    z = O.ilu0_solve(a, lu, diag, r)
    np.testing.assert_allclose(z, np.linalg.solve(L @ U, r), rtol=1e-13, atol=1e-14)
    zt = O.ilu0_solve(a, lu, diag, r, trans=True)
    np.testing.assert_allclose(zt, np.linalg.solve((L @ U).T, r), rtol=1e-13, atol=1e-14)


# --------------------------------------------------------------------------- F-relaxation closed forms
def build(sysd, levels, **kw):
    m = O.MGR(sysd["b"], sysd["rp"], sysd["ci"], sysd["vals"], sysd["field"], [LevelOpts(**l) for l in levels], **kw)
    assert m.status == 0, m.status
    return m


def one_level_closed_form(A, F, C, Mf, Mp, nu, omega, jacobi_r, v, Bc=None):
    """One MGR level of Algorithm 1 from z = 0, in block form: nu F-relaxation
    sweeps with M_FF^{-1} = Mf, P_F = -Mp A_FC, R_F = -A_CF Mp (Jacobi
    restriction) or 0 (injection), coarse solve Bc (None: exact)."""
    AFF, AFC, ACF, ACC = (A[np.ix_(F, F)], A[np.ix_(F, C)], A[np.ix_(C, F)], A[np.ix_(C, C)])
    nF = len(F)
    G = np.linalg.matrix_power(np.eye(nF) - omega * Mf @ AFF, nu)
    zF0 = (np.eye(nF) - G) @ np.linalg.solve(AFF, v[F])
    PF = -Mp @ AFC
    RF = -ACF @ Mp if jacobi_r else np.zeros((len(C), nF))
    Ac = ACC + ACF @ PF + RF @ AFC + RF @ AFF @ PF
    rc = (v[C] - ACF @ zF0) + RF @ (v[F] - AFF @ zF0)
    e = np.linalg.solve(Ac, rc) if Bc is None else Bc @ rc
    z = np.zeros_like(v)
    z[F] = zF0 + PF @ e
    z[C] = e
    return z


def block_inverse(AFF, groups):
    M = np.zeros_like(AFF)
    for g in groups:
        M[np.ix_(g, g)] = np.linalg.inv(AFF[np.ix_(g, g)])
    return M


@pytest.mark.parametrize("nu,omega,restrict", [(1, 1.0, "injection"), (3, 0.7, "injection"), (2, 1.2, "jacobi"),
                                               (4, 0.9, "jacobi")])
def test_jacobi_frelaxation_sweeps_closed_form(nu, omega, restrict):
    # two-field TPFA: A_FF (saturations) has off-diagonal upwind couplings, so
    # every sweep changes z_F; the 64 pressures are solved exactly by the coarse LU
    s = W.two_field_tpfa(4, 4, 4, seed=3)
    m = build(s, [dict(fmask=1 << 1, frelax="jacobi", sweeps=nu, omega=omega, restrict=restrict)])
    A = W.csr_of(s).toarray()
    F, C = np.where(s["field"] == 1)[0], np.where(s["field"] == 0)[0]
    assert m.info()["amg_levels"] == [(len(C), m.info()["amg_levels"][0][1])]   # coarse solve is exact
    Dinv = np.diag(1.0 / np.diag(A[np.ix_(F, F)]))
    rng = np.random.default_rng(nu)
    for _ in range(2):
        v = rng.standard_normal(s["n"])
        z = one_level_closed_form(A, F, C, Dinv, Dinv, nu, omega, restrict == "jacobi", v)
        np.testing.assert_allclose(m.apply(v), z, rtol=1e-11, atol=1e-12 * np.abs(z).max())


def test_jacobi_sweeps_on_a_diagonal_aff_equal_one_sweep():
    # F = cells of the mimetic system: A_FF diagonal, Jacobi exact, so every
    # sweep after the first leaves z unchanged at omega = 1; with omega != 1
    # the F-part is (1 - (1 - omega)^nu) A_FF^{-1} v_F
    s = W.hybrid_mimetic(3, 3, 3, seed=5)
    lv = dict(s["levels"][0])
    v = np.random.default_rng(2).standard_normal(s["n"])
    z1 = build(s, [dict(lv, sweeps=1)]).apply(v)
    z3 = build(s, [dict(lv, sweeps=3)]).apply(v)
    np.testing.assert_allclose(z3, z1, rtol=1e-13, atol=1e-14 * np.abs(z1).max())
    A = W.csr_of(s).toarray()
    F, C = np.where(s["field"] == 0)[0], np.where(s["field"] == 1)[0]
    Dinv = np.diag(1.0 / np.diag(A[np.ix_(F, F)]))
    zw = build(s, [dict(lv, sweeps=3, omega=0.6)]).apply(v)
    ref = one_level_closed_form(A, F, C, Dinv, Dinv, 3, 0.6, False, v)
    np.testing.assert_allclose(zw, ref, rtol=1e-11, atol=1e-12 * np.abs(ref).max())


@pytest.mark.parametrize("nu,omega,restrict", [(1, 1.0, "injection"), (2, 0.8, "jacobi"), (3, 1.1, "injection")])
def test_block_jacobi_frelaxation_sweeps_closed_form(nu, omega, restrict):
    # compositional system, one level: F = the three components (and the well
    # padding), grouped per cell; the coarse pressures + well are solved exactly
    s = W.compositional_wells(3, 3, 2, seed=4, wells_per_axis=1)
    fm = (1 << 1) | (1 << 2) | (1 << 3) | (1 << 5)
    m = build(s, [dict(fmask=fm, frelax="block_jacobi", sweeps=nu, omega=omega, restrict=restrict)])
    A = W.csr_of(s).toarray()
    isF = np.array([(fm >> f) & 1 for f in s["field"]], bool)
    F, C = np.where(isF)[0], np.where(~isF)[0]
    assert len(C) <= 128
    blk = F // s["b"]
    groups = [np.where(blk == b)[0] for b in np.unique(blk)]
    assert max(len(g) for g in groups) == 3
    Mb = block_inverse(A[np.ix_(F, F)], groups)
    v = np.random.default_rng(7).standard_normal(s["n"])
    z = one_level_closed_form(A, F, C, Mb, Mb, nu, omega, restrict == "jacobi", v)
    np.testing.assert_allclose(m.apply(v), z, rtol=1e-11, atol=1e-12 * np.abs(z).max())


def chain_f_system(nF=24, nC=10, seed=0):
    """CSR system whose F-F block is tridiagonal (F-points on a chain), so
    ILU(0) of A_FF is its exact LU; labels: F = 1, C = 0."""
    rng = np.random.default_rng(seed)
    n = nF + nC
    A = np.zeros((n, n))
    F, C = np.arange(nF), np.arange(nF, n)
    for k in range(nF):
        A[k, k] = 4.0 + rng.uniform()
        if k > 0:
            A[k, k - 1] = -1.0 + 0.3 * rng.uniform()
        if k + 1 < nF:
            A[k, k + 1] = -1.0 - 0.3 * rng.uniform()
    for i in C:
        A[i, i] = 5.0 + rng.uniform()
    for _ in range(3 * nC):
        i, j = rng.choice(C), rng.choice(C)
        if i != j:
            A[i, j] = -0.4 * rng.uniform()
    for _ in range(2 * nF):
        k, i = rng.choice(F), rng.choice(C)
        A[k, i] = -0.5 * rng.uniform()
        A[i, rng.choice(F)] = -0.5 * rng.uniform()
    a = sp.csr_matrix(A)
    a.sort_indices()
    field = np.array([1] * nF + [0] * nC, np.int32)
    return dict(b=1, rp=a.indptr.astype(np.int32), ci=a.indices.astype(np.int32), vals=a.data.copy(), field=field,
                n=n), A, F, C


@pytest.mark.parametrize("nu,omega,restrict", [(1, 1.0, "injection"), (2, 0.7, "jacobi")])
def test_ilu0_frelaxation_on_a_tridiagonal_aff_is_exact(nu, omega, restrict):
    # ILU(0) of a tridiagonal A_FF has no fill: M = A_FF^{-1}, so the F-part
    # after nu sweeps is (1 - (1 - omega)^nu) A_FF^{-1} v_F; interpolation and
    # restriction keep Jacobi's D^{-1} (eq. (4), (5))
    s, A, F, C = chain_f_system()
    m = build(s, [dict(fmask=1 << 1, frelax="ilu0", sweeps=nu, omega=omega, restrict=restrict)])
    Dinv = np.diag(1.0 / np.diag(A[np.ix_(F, F)]))
    Mf = np.linalg.inv(A[np.ix_(F, F)])
    v = np.random.default_rng(8).standard_normal(s["n"])
    z = one_level_closed_form(A, F, C, Mf, Dinv, nu, omega, restrict == "jacobi", v)
    np.testing.assert_allclose(m.apply(v), z, rtol=1e-11, atol=1e-12 * np.abs(z).max())


def test_ilu0_frelaxation_with_fill_uses_the_ilu_factors():
    # A_FF = a 2-D Laplacian block (fill outside the pattern): M = (LU)^{-1}
    # with the factors pinned by test_ilu0_reproduces_a_on_its_pattern
    nx = 5
    AFF = (lap2d(nx) + sp.identity(nx * nx) * 0.5).toarray()
    nF, nC = nx * nx, 8
    rng = np.random.default_rng(2)
    n = nF + nC
    A = np.zeros((n, n))
    A[:nF, :nF] = AFF
    A[nF:, nF:] = np.diag(3.0 + rng.uniform(size=nC))
    for _ in range(20):
        A[rng.integers(nF), nF + rng.integers(nC)] = -0.3
        A[nF + rng.integers(nC), rng.integers(nF)] = -0.3
    a = sp.csr_matrix(A)
    a.sort_indices()
    s = dict(b=1, rp=a.indptr.astype(np.int32), ci=a.indices.astype(np.int32), vals=a.data.copy(),
             field=np.array([1] * nF + [0] * nC, np.int32), n=n)
    F, C = np.arange(nF), np.arange(nF, n)
    m = build(s, [dict(fmask=1 << 1, frelax="ilu0", sweeps=2, omega=0.9, restrict="injection")])
    aff = sp.csr_matrix(AFF)
    aff.sort_indices()
    lu, diag, st = O.ilu0(aff)
    L, U = lu_dense(aff, lu, diag)
    Mf = np.linalg.inv(L @ U)
    assert np.abs(Mf - np.linalg.inv(AFF)).max() > 1e-4     # ILU(0) is not exact here
    Dinv = np.diag(1.0 / np.diag(AFF))
    v = rng.standard_normal(n)
    z = one_level_closed_form(A, F, C, Mf, Dinv, 2, 0.9, False, v)
    np.testing.assert_allclose(m.apply(v), z, rtol=1e-11, atol=1e-12 * np.abs(z).max())


# --------------------------------------------------------------------------- AMG V-cycle closed form
def l1_diag(A):
    off = np.abs(A).sum(axis=1) - np.abs(np.diag(A))
    return np.diag(A) + off


def vcycle_operator(As, Ps, nu_pre, nu_post):
    """B_0 of the V(nu_pre, nu_post) cycle from its error propagation, coarsest
    level solved exactly."""
    B = np.linalg.inv(As[-1])
    for k in range(len(As) - 2, -1, -1):
        A, P = As[k], Ps[k]
        n = A.shape[0]
        S = np.eye(n) - A / l1_diag(A)[:, None]
        E = (np.linalg.matrix_power(S, nu_post) @ (np.eye(n) - P @ B @ P.T @ A) @
             np.linalg.matrix_power(S, nu_pre))
        B = (np.eye(n) - E) @ np.linalg.inv(A)
    return B


def amg_only(a, **kw):
    a = sp.csr_matrix(a)
    a.sort_indices()
    s = dict(b=1, rp=a.indptr.astype(np.int32), ci=a.indices.astype(np.int32), vals=a.data.copy(),
             field=np.zeros(a.shape[0], np.int32), n=a.shape[0])
    return build(s, [], **kw), s


def hierarchy(m):
    info = m.info()["amg_levels"]
    As = [m.export(1, k, 1).to_scipy().toarray() for k in range(len(info))]
    Ps = [m.export(1, k, 2).to_scipy().toarray() for k in range(len(info) - 1)]
    return As, Ps


@pytest.mark.parametrize("nu_pre,nu_post", [(1, 1), (2, 1), (0, 2), (2, 3)])
def test_amg_vcycle_equals_its_error_propagation_closed_form(nu_pre, nu_post):
    # a nonsymmetric, anisotropic 2-D operator: three or more levels with max_coarse 20
    nx = 14
    a = lap2d(nx) + 0.3 * sp.kron(sp.identity(nx), sp.diags([-np.ones(nx - 1)], [1])) + 0.05 * sp.identity(nx * nx)
    m, s = amg_only(a, max_coarse=20, nu_pre=nu_pre, nu_post=nu_post)
    As, Ps = hierarchy(m)
    assert len(As) >= 3
    # Galerkin coarse operators (Sec. 2's R A P with R = P^T)
    for k in range(len(Ps)):
        np.testing.assert_allclose(As[k + 1], Ps[k].T @ As[k] @ Ps[k], rtol=1e-12, atol=1e-13 * np.abs(As[k]).max())
    B = vcycle_operator(As, Ps, nu_pre, nu_post)
    rng = np.random.default_rng(nu_pre * 10 + nu_post)
    for _ in range(2):
        v = rng.standard_normal(s["n"])
        z = B @ v
        np.testing.assert_allclose(m.apply(v), z, rtol=1e-11, atol=1e-12 * np.abs(z).max())
        # the transposed cycle is the transposed operator
        zt = B.T @ v
        np.testing.assert_allclose(m.apply(v, trans=True), zt, rtol=1e-11, atol=1e-12 * np.abs(zt).max())


def test_amg_vcycle_closed_form_unknown_based():
    # two decoupled-label 1-D Laplacians interleaved with a weak cross coupling:
    # strength and interpolation stay within a label, Galerkin keeps the cross terms
    n = 60
    A = np.zeros((2 * n, 2 * n))
    L1 = lap1d(n).toarray() + 0.1 * np.eye(n)
    L2 = 2.0 * lap1d(n).toarray() + 0.2 * np.eye(n)
    A[0::2, 0::2] = L1
    A[1::2, 1::2] = L2
    for i in range(n):
        A[2 * i, 2 * i + 1] = -0.05
        A[2 * i + 1, 2 * i] = -0.02
    a = sp.csr_matrix(A)
    a.sort_indices()
    field = np.tile([0, 1], n).astype(np.int32)
    s = dict(b=1, rp=a.indptr.astype(np.int32), ci=a.indices.astype(np.int32), vals=a.data.copy(), field=field,
             n=2 * n)
    m = build(s, [], max_coarse=12, coarse_unknown_based=True)
    As, Ps = hierarchy(m)
    assert len(As) >= 3
    # interpolation never mixes labels
    P0 = Ps[0]
    cf = m.export(1, 0, 0)
    clab = field[cf == 1]
    for i in range(2 * n):
        for j in np.nonzero(P0[i])[0]:
            assert clab[j] == field[i]
    B = vcycle_operator(As, Ps, 1, 1)
    v = np.random.default_rng(3).standard_normal(2 * n)
    np.testing.assert_allclose(m.apply(v), B @ v, rtol=1e-11, atol=1e-12 * np.abs(B @ v).max())


def test_amg_frelaxation_cycle_inside_mgr_closed_form():
    # MGR level whose F-relaxation is one AMG V-cycle on A_FF (Sec. 3.3): the
    # F-part is B_FF v_F with B_FF the cycle operator of the F-relaxation AMG,
    # and the coarse pressures get the coarse AMG's cycle operator
    s = W.two_field_tpfa(6, 6, 5, seed=9)
    m = build(s, [dict(fmask=1 << 1, frelax="amg", sweeps=1, omega=1.0, restrict="injection")], max_coarse=20)
    A = W.csr_of(s).toarray()
    F, C = np.where(s["field"] == 1)[0], np.where(s["field"] == 0)[0]
    # the F-relaxation hierarchy (kind 2, sub = level 0)
    As, Ps = [], []
    k = 0
    while True:
        try:
            As.append(m.export(2, k, 1, sub=0).to_scipy().toarray())
        except KeyError:
            break
        try:
            Ps.append(m.export(2, k, 2, sub=0).to_scipy().toarray())
        except KeyError:
            break
        k += 1
    assert len(As) >= 2 and len(Ps) == len(As) - 1
    Bff = vcycle_operator(As, Ps, 1, 1)
    Bc = vcycle_operator(*hierarchy(m), 1, 1)
    Dinv = np.diag(1.0 / np.diag(A[np.ix_(F, F)]))
    v = np.random.default_rng(5).standard_normal(s["n"])
    z = one_level_closed_form(A, F, C, Bff, Dinv, 1, 1.0, False, v, Bc=Bc)
    np.testing.assert_allclose(m.apply(v), z, rtol=1e-10, atol=1e-12 * np.abs(z).max())
