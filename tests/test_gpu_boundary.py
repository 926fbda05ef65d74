"""GPU checks of the boundary's allocation and grouping arguments, through the
C-ABI: block-Jacobi groups given per unknown (block_of_dof) on a scalar CSR
input against the oracle and against the block-CSR input they mirror; the
caller's device memory provider (torch's caching allocator) against the
library's own allocations."""
import numpy as np
import pytest

from _systems import elem_err, gpu_solver, oracle_mgr, say
from test_oracle_block_groups import scalar_copy
import workloads as W

pytestmark = pytest.mark.gpu


def _csr_equal(g, o):
    nr, nc, rp, ci, v = g
    return (nr, nc) == (o.nr, o.nc) and np.array_equal(rp, o.rp) and np.array_equal(ci, o.ci) and \
        np.array_equal(v, o.v)


def test_block_groups_on_scalar_input():
    s = W.compositional_wells(12, 10, 6, seed=4, wells_per_axis=2)
    sb = scalar_copy(s)
    grp = np.arange(s["n"], dtype=np.int32) // s["b"]
    say(f"[block groups] compositional 12x10x6 as b = 1 CSR, n = {s['n']}")
    gs = gpu_solver(sb, block=grp)
    gb = gpu_solver(s)
    om = oracle_mgr(sb, block=grp)
    assert gs.info() == om.info() == gb.info()
    for l in range(len(s["levels"])):
        assert np.array_equal(gs.export(0, l, 0), om.export(0, l, 0))
        for what in (1, 2, 5):
            assert _csr_equal(gs.export(0, l, what), om.export(0, l, what)), (l, what)
            # the scalar input with cell groups builds the block input's operators
            a, b = gs.export(0, l, what), gb.export(0, l, what)
            assert all(np.array_equal(x, y) for x, y in zip(a[2:], b[2:])), (l, what)
    v = np.random.default_rng(5).standard_normal(s["n"])
    z = gs.apply(v).cpu().numpy()
    assert elem_err(z, om.apply(v), s["field"]) <= 1e-10
    assert np.array_equal(z, gb.apply(v).cpu().numpy())
    X, [ig] = gs.solve(sb["rhs"])
    xo, io = om.solve(sb["rhs"])
    assert ig.status == 0 and abs(ig.iterations - io.iterations) <= 1
    assert elem_err(X.cpu().numpy(), xo, s["field"]) <= 1e-8
    # groups survive a setup reuse
    gs.update_values(sb["vals"] * 1.01)
    gb.update_values(s["vals"] * 1.01)
    assert np.array_equal(gs.apply(v).cpu().numpy(), gb.apply(v).cpu().numpy())
    gs.close(); gb.close()


def test_block_group_above_four_is_unsupported():
    import paper_2101_11649_amd as P
    s = W.compositional_wells(4, 4, 3, seed=1, wells_per_axis=1)
    sb = scalar_copy(s)
    grp = np.arange(s["n"], dtype=np.int32) // 8
    with pytest.raises(P.MgrError) as e:
        gpu_solver(sb, block=grp)
    assert e.value.code == -6
    # the handle-less failure leaves the device usable
    g = gpu_solver(sb, block=np.arange(s["n"], dtype=np.int32) // 4)
    X, [ig] = g.solve(sb["rhs"])
    assert ig.status == 0
    g.close()


def test_caller_allocator_matches_library_allocations():
    import torch
    s = W.compositional_wells(16, 12, 8, seed=6, wells_per_axis=2)
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    gn = gpu_solver(s, allocator=None)       # the library's own stream-ordered allocations
    mid = torch.cuda.memory_allocated()
    gt = gpu_solver(s)                       # torch's caching allocator (the binding's default)
    after = torch.cuda.memory_allocated()
    say(f"[allocator] torch tensors of a solver: {(mid - before) / 2**20:.2f} MiB without the provider, "
        f"{(after - mid) / 2**20:.2f} MiB with it")
    # the hierarchy (at least the library's copy of A's values) came from torch
    assert (after - mid) > (mid - before) + 8 * s["vals"].size
    v = np.random.default_rng(2).standard_normal(s["n"])
    assert np.array_equal(gt.apply(v).cpu().numpy(), gn.apply(v).cpu().numpy())
    Xt, [it] = gt.solve(s["rhs"])
    Xn, [in_] = gn.solve(s["rhs"])
    assert it.iterations == in_.iterations and torch.equal(Xt, Xn)
    gn.close()
    gt.close()
    del Xt, Xn, gt, gn
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() <= before + 64 * 1024    # everything went back to torch
