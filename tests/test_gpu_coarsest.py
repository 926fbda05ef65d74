"""GPU: the dense inverse of the coarsest AMG level (Gauss-Jordan with partial
pivoting, one workgroup) against numpy's inverse of the exported coarsest
matrix.  Two kinds of input: AMG hierarchies of the small systems, and systems
whose coarse grid is a single dense-ish random block (the AMG then has one
level, so its whole coarse system is inverted), which needs real row pivoting.
Sizes cover both kernels: the register-resident one (n <= 128, including 1 and
128) and the global-memory one (n > 128)."""
import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W
from _systems import SMALL, gpu_solver, say

pytestmark = pytest.mark.gpu


def _coarsest_A(gs):
    last = len(gs.info()["amg_levels"]) - 1
    nr, nc, rp, ci, v = gs.export(1, last, 1)
    return sp.csr_matrix((v, ci, rp), shape=(nr, nc)).toarray()


def _check(gs, what):
    A = _coarsest_A(gs)
    G = gs.coarsest_inverse()
    ref = np.linalg.inv(A)
    err = np.abs(G - ref).max() / np.abs(ref).max()
    res = np.abs(G @ A - np.eye(A.shape[0])).max()
    say(f"{what}: n={A.shape[0]} rel err {err:.2e} |GA - I| {res:.2e}")
    assert err <= 1e-10 * max(1.0, np.linalg.cond(A) / 1e4)
    assert res <= 1e-10


@pytest.mark.parametrize("name", ["tpfa_7x6x5", "mimetic_9x7x6", "comp_8x8x6", "frac_12^3"])
def test_coarsest_of_amg(name):
    s = SMALL[name]()
    gs = gpu_solver(s)
    _check(gs, name)
    gs.close()


# (system, max_coarse) -> coarsest size: 256, 332 and 1024 unknowns
@pytest.mark.parametrize("name,max_coarse,n", [("tpfa_16^3", 300, 256), ("mimetic_20^3", 500, 332),
                                               ("comp_20x18x10", 2000, 1024)])
def test_coarsest_above_128(name, max_coarse, n):
    s = SMALL[name]()
    gs = gpu_solver(s, max_coarse=max_coarse)
    assert gs.info()["amg_levels"][-1][0] == n
    _check(gs, f"{name} max_coarse {max_coarse}")
    gs.close()


def _single_block_system(m, seed):
    """F = field 1 (identity rows, uncoupled), C = field 0 with a random
    nonsymmetric block of about 30% density whose diagonal is small, so the
    pivots come from other rows: the coarse grid is that block itself."""
    rng = np.random.default_rng(seed)
    C = rng.standard_normal((m, m)) * (rng.random((m, m)) < 0.3)
    C[np.arange(m), np.arange(m)] = 1e-3 * rng.standard_normal(m)
    C += np.eye(m, k=1) + np.eye(m, k=-(m - 1))  # keeps it nonsingular in practice
    n = 2 * m
    A = sp.lil_matrix((n, n))
    A[:m, :m] = C
    A[m:, m:] = sp.identity(m)
    A = A.tocsr()
    A.sort_indices()
    field = np.concatenate([np.zeros(m, np.int32), np.ones(m, np.int32)])
    return W._system(1, A.indptr, A.indices, A.data, field, rng.standard_normal(n),
                     [W.level(1 << 1, "jacobi")], f"single_block_{m}")


@pytest.mark.parametrize("m", [1, 2, 17, 64, 100, 127, 128, 129, 200])
def test_coarsest_with_pivoting(m):
    s = _single_block_system(m, seed=m)
    gs = gpu_solver(s, max_coarse=256)
    assert gs.info()["amg_levels"][-1][0] == m and len(gs.info()["amg_levels"]) == 1
    _check(gs, f"single block {m}")
    gs.close()
