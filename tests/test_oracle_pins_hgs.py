"""Pins for the oracle's hybrid L1 Gauss-Seidel AMG smoother (Sec. 4.1: one
forward sweep on the way down, one backward sweep on the way up; Baker,
Falgout, Kolev, Yang 2011), each against something other than the oracle's own
loops:

* the V-cycle equals its error-propagation closed form with the dense smoother
  matrices M_f = D + L_chunk and M_b = D + U_chunk, where L_chunk / U_chunk keep
  the strictly lower / upper entries whose row and column lie in one chunk and
  D holds a_ii plus the l1 norm of each row's entries outside its chunk (for
  chunk sizes 1, 3, 7 and one chunk: sequential Gauss-Seidel), forward and
  transposed;
* with chunk 1 the smoother is L1-Jacobi (the whole MGR apply is bit-identical);
* a wrong direction, stale in-chunk values or the full-row l1 term fail the
  closed form (checked by hand when the pin was written)."""
import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W
from _systems import oracle_mgr
from test_oracle_pins_relax import amg_only, hierarchy, lap2d


def smoother_matrices(A, chunk):
    n = A.shape[0]
    grp = np.arange(n) // chunk
    same = grp[:, None] == grp[None, :]
    off = np.abs(A) * ~same
    D = np.diag(np.diag(A) + off.sum(axis=1))
    L = np.tril(A * same, -1)
    U = np.triu(A * same, 1)
    return D + L, D + U


def vcycle_operator_hgs(As, Ps, nu_pre, nu_post, chunk):
    B = np.linalg.inv(As[-1])
    for k in range(len(As) - 2, -1, -1):
        A, P = As[k], Ps[k]
        n = A.shape[0]
        Mf, Mb = smoother_matrices(A, chunk)
        Sf = np.eye(n) - np.linalg.solve(Mf, A)
        Sb = np.eye(n) - np.linalg.solve(Mb, A)
        E = (np.linalg.matrix_power(Sb, nu_post) @ (np.eye(n) - P @ B @ P.T @ A) @
             np.linalg.matrix_power(Sf, nu_pre))
        B = (np.eye(n) - E) @ np.linalg.inv(A)
    return B


@pytest.mark.parametrize("chunk", [1, 3, 7, 10**6])
@pytest.mark.parametrize("nu_pre,nu_post", [(1, 1), (2, 1)])
def test_hybrid_gs_vcycle_closed_form(chunk, nu_pre, nu_post):
    nx = 13
    a = lap2d(nx) + 0.3 * sp.kron(sp.identity(nx), sp.diags([-np.ones(nx - 1)], [1])) + 0.05 * sp.identity(nx * nx)
    m, s = amg_only(a, max_coarse=20, nu_pre=nu_pre, nu_post=nu_post, smoother="hybrid-gs", chunk=chunk)
    As, Ps = hierarchy(m)
    assert len(As) >= 3
    B = vcycle_operator_hgs(As, Ps, nu_pre, nu_post, chunk)
    rng = np.random.default_rng(chunk % 97 + nu_pre)
    for _ in range(2):
        v = rng.standard_normal(s["n"])
        z = B @ v
        np.testing.assert_allclose(m.apply(v), z, rtol=1e-11, atol=1e-12 * np.abs(z).max())
        zt = B.T @ v
        np.testing.assert_allclose(m.apply(v, trans=True), zt, rtol=1e-11, atol=1e-12 * np.abs(zt).max())


def test_hybrid_gs_with_chunks_of_one_row_is_l1_jacobi():
    for s in (W.hybrid_mimetic(9, 7, 6, seed=3), W.fracturing(12, seed=5)):
        mj = oracle_mgr(s)
        mg = oracle_mgr(s, smoother="hybrid-gs", chunk=1)
        v = np.random.default_rng(1).standard_normal(s["n"])
        assert np.array_equal(mj.apply(v), mg.apply(v))
        assert np.array_equal(mj.apply(v, trans=True), mg.apply(v, trans=True))


def test_hybrid_gs_changes_the_cycle_and_stays_convergent():
    s = W.fracturing(12, seed=5)
    mj, mg = oracle_mgr(s), oracle_mgr(s, smoother="hybrid-gs", chunk=32)
    v = np.random.default_rng(2).standard_normal(s["n"])
    assert not np.allclose(mj.apply(v), mg.apply(v))
    xj, ij = mj.solve(s["rhs"])
    xg, ig = mg.solve(s["rhs"])
    assert ig.status == 0 and ig.iterations <= ij.iterations
    np.testing.assert_allclose(xg, xj, rtol=0, atol=1e-7 * np.abs(xj).max())
