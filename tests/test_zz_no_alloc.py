"""mgr_apply_noalloc (the apply whose work vectors live in the library's static
scratch array) against mgr_apply through the C-ABI: the same kernels on the
same operators, so the results must be identical.  Two calls in a row on two
handles, the second on a smaller system, so that the second reads a scratch
array that still holds the first call's values."""
import ctypes

import numpy as np
import pytest

from _systems import SMALL, gpu_solver, say

pytestmark = pytest.mark.gpu


def _noalloc(P, g, v, z):
    return P.lib().mgr_apply_noalloc(g._h, ctypes.c_void_p(v.data_ptr()), ctypes.c_void_p(z.data_ptr()))


@pytest.mark.parametrize("precision", [64, 32])
def test_noalloc_apply_equals_apply(precision):
    import torch

    import paper_2101_11649_amd as P
    big, small = SMALL["mimetic_20^3"](), SMALL["comp_8x8x6"]()
    assert big["n"] > small["n"]
    ga = gpu_solver(big, precision=precision)
    gb = gpu_solver(small, precision=precision)
    try:
        rng = np.random.default_rng(7)
        for g, s in ((ga, big), (gb, small)):
            v = torch.tensor(rng.standard_normal(s["n"]), device="cuda")
            z = torch.full_like(v, float("nan"))
            # before any apply on this setup the operator copies may not exist yet
            assert _noalloc(P, g, v, z) == -1
            zref = g.apply(v)
            rc = _noalloc(P, g, v, z)
            assert rc == 0, P.lib().mgr_last_error(g._h)
            torch.cuda.synchronize()
            a, b = z.cpu().numpy(), zref.cpu().numpy()
            say(f"{s['name']} fp{precision}: noalloc vs apply max |diff| {np.abs(a - b).max():.3e}")
            assert np.array_equal(a, b)
        # the first handle again, after the smaller call overwrote the front of the array
        v = torch.tensor(rng.standard_normal(big["n"]), device="cuda")
        z = torch.empty_like(v)
        assert _noalloc(P, ga, v, z) == 0
        assert np.array_equal(z.cpu().numpy(), ga.apply(v).cpu().numpy())
    finally:
        ga.close()
        gb.close()


def test_noalloc_needs_setup_and_a_first_apply():
    import torch

    import paper_2101_11649_amd as P
    s = SMALL["tpfa_7x6x5"]()
    g = gpu_solver(s)
    try:
        v = torch.ones(s["n"], dtype=torch.float64, device="cuda")
        z = torch.empty_like(v)
        assert _noalloc(P, g, v, z) == -1            # no apply on this setup yet
        g.apply(v)
        assert _noalloc(P, g, v, z) == 0
        g.setup(g.vals)                              # a new hierarchy: its copies are made by its first apply
        assert _noalloc(P, g, v, z) == -1
        g.solve(v)
        assert _noalloc(P, g, v, z) == 0
        assert P.lib().mgr_apply_noalloc(g._h, None, ctypes.c_void_p(z.data_ptr())) == -1
    finally:
        g.close()


def test_noalloc_at_full_size():
    """The compositional 128 x 128 x 64 system (4,194,368 unknowns): its work
    vectors (73.5 MB in FP64) fit the scratch array, in both apply precisions."""
    import torch

    import paper_2101_11649_amd as P
    import workloads as W
    s = W.compositional_wells(seed=2)
    vals = torch.tensor(s["vals"], device="cuda")
    v = torch.tensor(np.random.default_rng(8).standard_normal(s["n"]), device="cuda")
    for precision in (64, 32):
        g = P.Solver(s["b"], s["rp"], s["ci"], vals, s["field"], s["levels"], precision=precision)
        try:
            zref = g.apply(v)
            z = torch.full_like(v, float("nan"))
            rc = _noalloc(P, g, v, z)
            assert rc == 0, P.lib().mgr_last_error(g._h)
            torch.cuda.synchronize()
            say(f"compositional 128x128x64 fp{precision}: noalloc vs apply identical")
            assert torch.equal(z, zref)
        finally:
            g.close()
