"""Shared test helpers: seeded systems and builders for the oracle and the GPU solver."""
import numpy as np

import oracle as O
import workloads as W

SMALL = {
    # ragged sizes (not multiples of any tile), several AMG levels each
    "tpfa_7x6x5": lambda: W.two_field_tpfa(7, 6, 5, seed=11),
    "tpfa_16^3": lambda: W.two_field_tpfa(16, 16, 16, seed=0),
    "mimetic_9x7x6": lambda: W.hybrid_mimetic(9, 7, 6, seed=3),
    "mimetic_tpfa_sym_6^3": lambda: W.hybrid_mimetic(6, 6, 6, seed=4, consistent=False, upwind=False),
    "mimetic_20^3": lambda: W.hybrid_mimetic(20, 20, 20, seed=5),
    # 4x4 blocks + wells, two MGR levels (block-Jacobi, then Jacobi on wells)
    "comp_8x8x6": lambda: W.compositional_wells(8, 8, 6, seed=7),
    "comp_20x18x10": lambda: W.compositional_wells(20, 18, 10, seed=8, wells_per_axis=3),
    # the paper's four-level compositional order: rho_2 (exact Jacobi), rho_1, p
    # (AMG F-relaxation), wells with zero diagonals on the coarse grid
    "comp4_10x9x8": lambda: W.compositional_4level(10, 9, 8, seed=5, wells_per_axis=2),
    "comp4_20x18x12": lambda: W.compositional_4level(20, 18, 12, seed=6, wells_per_axis=3),
    # elasticity (3x3 blocks) + fracture pressures; F-relaxation = unknown-based AMG V-cycle
    "frac_12^3": lambda: W.fracturing(12, seed=5),
    "frac_18^3": lambda: W.fracturing(18, seed=6),
}


def _opts(s, kw):
    o = dict(s.get("solver_opts", {}))
    o.update(kw)
    return o


def oracle_mgr(s, levels=None, **kw):
    lv = [O.LevelOpts(**l) for l in (levels if levels is not None else s["levels"])]
    kw = {k: v for k, v in _opts(s, kw).items() if k in ("theta", "max_levels", "max_coarse", "nu_pre", "nu_post",
                                                         "coarse_unknown_based", "seed")}
    m = O.MGR(s["b"], s["rp"], s["ci"], s["vals"], s["field"], lv, **kw)
    assert m.status == 0, m.status
    return m


def gpu_solver(s, levels=None, **kw):
    import paper_2101_11649_amd as P
    return P.Solver(s["b"], s["rp"], s["ci"], s["vals"], s["field"],
                    levels if levels is not None else s["levels"], **_opts(s, kw))


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    d = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (d if d > 0 else 1.0)


def say(*args):
    print(*args, flush=True)
