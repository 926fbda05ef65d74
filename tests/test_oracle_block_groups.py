"""CPU pins of the oracle's block-Jacobi groups given per unknown: a b = 1
(scalar CSR) input with the group of every unknown set to its cell must give
the same hierarchy, apply and solution as the block-CSR input whose block rows
are those cells (the default grouping), and a group of more than 4 F-points is
refused."""
import numpy as np

import oracle as O
import workloads as W


def scalar_copy(s):
    """The same system as plain CSR (b = 1), stored zeros of the blocks kept."""
    A = W.csr_of(s)
    A.sort_indices()
    return dict(s, b=1, rp=A.indptr.astype(np.int32), ci=A.indices.astype(np.int32), vals=A.data.copy())


def _mgr(s, block=None):
    return O.MGR(s["b"], s["rp"], s["ci"], s["vals"], s["field"], [O.LevelOpts(**l) for l in s["levels"]],
                 block=block)


def test_scalar_input_with_cell_groups_equals_block_input():
    s = W.compositional_wells(6, 5, 4, seed=3, wells_per_axis=2)
    assert s["levels"][0]["frelax"] == "block_jacobi"
    sb = scalar_copy(s)
    mb = _mgr(s)
    ms = _mgr(sb, block=np.arange(s["n"], dtype=np.int32) // s["b"])
    assert mb.status == 0 and ms.status == 0
    assert mb.info() == ms.info()
    for l in range(len(s["levels"])):
        for what in (1, 2, 5):
            a, b = mb.export(0, l, what), ms.export(0, l, what)
            assert np.array_equal(a.rp, b.rp) and np.array_equal(a.ci, b.ci) and np.array_equal(a.v, b.v)
    # the block inverse is a true 4 x 4 (3 x 3 on the components) inverse: not the scalar Jacobi one
    mj = _mgr(sb)
    assert mj.export(0, 0, 5).v.size < ms.export(0, 0, 5).v.size
    v = np.random.default_rng(0).standard_normal(s["n"])
    assert np.array_equal(mb.apply(v), ms.apply(v))
    xb, ib = mb.solve(s["rhs"])
    xs, is_ = ms.solve(sb["rhs"])
    assert ib.iterations == is_.iterations and np.array_equal(xb, xs)


def test_group_larger_than_four_is_unsupported():
    s = W.compositional_wells(4, 4, 3, seed=1, wells_per_axis=1)
    sb = scalar_copy(s)
    grp = np.arange(s["n"], dtype=np.int32) // 8          # two cells per group: 6 F-points
    assert _mgr(sb, block=grp).status == -6
