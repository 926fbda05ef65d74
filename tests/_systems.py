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
    # MGR_Pi on the TPFA variant: F = faces (diagonal block), C = cells -> AMG
    "mimetic_tpfa_pi_9x7x6": lambda: W.hybrid_mimetic(9, 7, 6, seed=9, consistent=False, reduction="pi"),
    "mimetic_tpfa_pi_26x21x17": lambda: W.hybrid_mimetic(26, 21, 17, seed=10, consistent=False, reduction="pi"),
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
    # MGR_P (Sec. 3.3): F = fracture pressures (AMG F-relaxation), coarse
    # A_uu - A_up D_pp^-1 A_pu to unknown-based AMG
    "frac_p_12^3": lambda: W.fracturing(12, seed=5, reduction="p"),
    "frac_p_18^3": lambda: W.fracturing(18, seed=6, reduction="p"),
}


def perturbed_values(s, scale=0.05, seed=0, rows_field=None):
    """New values on the same pattern, as between two Newton solves: every
    scalar row scaled by 1 + U[-scale, scale] (only the rows whose unknown has
    field rows_field, if given).  Row scaling keeps the sign structure of every
    Schur complement the reduction forms."""
    rng = np.random.default_rng(seed)
    b, nb = s["b"], len(s["ci"])
    f = 1.0 + rng.uniform(-scale, scale, s["n"])
    if rows_field is not None:
        f[s["field"] != rows_field] = 1.0
    brow = np.repeat(np.arange(len(s["rp"]) - 1), np.diff(s["rp"]))        # block row of each block
    rows = brow[:, None] * b + np.arange(b)[None, :]                        # scalar row of each block row
    v = s["vals"].reshape(nb, b, b) * f[rows][:, :, None]
    return v.reshape(-1)


def _opts(s, kw):
    o = dict(s.get("solver_opts", {}))
    o.update(kw)
    return o


def oracle_mgr(s, levels=None, **kw):
    lv = [O.LevelOpts(**l) for l in (levels if levels is not None else s["levels"])]
    kw = _opts(s, kw)
    if "unknown_based" in kw:     # the binding's name for the coarse AMG's unknown-based option
        kw["coarse_unknown_based"] = kw.pop("unknown_based")
    kw = {k: v for k, v in kw.items() if k in ("theta", "max_levels", "max_coarse", "nu_pre", "nu_post",
                                                         "coarse_unknown_based", "seed", "interp", "block", "smoother",
                                                         "chunk", "agg_levels")}
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


def elem_err(a, b, field=None):
    """Entry-wise difference of a from the reference b: the largest |a_i - b_i|
    over the entries of each field label, relative to the largest |b_i| of that
    label, and the worst label.  Unlike a 2-norm over the whole vector it sees a
    wrong value in a small set of unknowns (the well pressures, the fracture
    pressures) however many other unknowns there are.  2-D arrays are taken
    row by row (one right-hand side per row) with the same labels."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    if field is not None and a.ndim == 2:
        field = np.tile(np.asarray(field), a.shape[0])
    a, b = a.reshape(-1), b.reshape(-1)
    groups = [np.ones(len(b), bool)] if field is None else [field == f for f in np.unique(field)]
    worst = 0.0
    for g in groups:
        d = np.abs(a[g] - b[g]).max() if g.any() else 0.0
        if d == 0.0:
            continue
        sc = np.abs(b[g]).max()
        worst = max(worst, d / sc if sc > 0 else np.inf)
    return worst


def say(*args):
    print(*args, flush=True)
