"""Seeded synthetic linear systems shaped like the paper's workloads.

This module only builds inputs (matrices, field labels, right-hand sides and
the reduction order to use); it holds none of the MGR / AMG / GMRES
arithmetic, so both the oracle and the GPU library can consume it.

The paper's own systems (HI24L meshes, the fracturing model) are not
available; these structured-grid generators stand in for them:

* ``two_field_tpfa``      -- cell-centred pressure + saturation, 7-point TPFA,
                             interleaved 2x2 blocks (the two-field flow system).
* ``hybrid_mimetic``      -- statically condensed hybrid mimetic system on a
                             hex grid: cell pressures + face multipliers
                             (the single-phase hybrid MFD system, Sec. 3.1 and
                             App. A of the paper).
* ``compositional_wells`` -- 4 unknowns per cell (pressure + 3 component
                             densities) on a 7-point stencil plus vertical
                             wells (the compositional system, Sec. 3.2).
* ``fracturing``          -- Q1 hex elasticity coupled to a planar fracture
                             with a cubic-law pressure stencil (Sec. 3.3, App. C).

Every generator takes an integer ``seed``; random streams come from
``numpy.random.SeedSequence(seed).spawn(8)`` in a fixed order (permeability,
accumulation, upwind, block noise, wells, RHS, FD sample, loss weights).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

STREAMS = ("perm", "accum", "upwind", "noise", "wells", "rhs", "fd", "loss")


def _rngs(seed):
    ss = np.random.SeedSequence(seed).spawn(len(STREAMS))
    return {name: np.random.Generator(np.random.PCG64(s)) for name, s in zip(STREAMS, ss)}


def _system(b, A_bsr_rp, A_bsr_ci, A_bsr_val, field, rhs, levels, name, **extra):
    out = dict(name=name, b=int(b), rp=np.ascontiguousarray(A_bsr_rp, np.int32),
               ci=np.ascontiguousarray(A_bsr_ci, np.int32), vals=np.ascontiguousarray(A_bsr_val, np.float64),
               field=np.ascontiguousarray(field, np.int32), rhs=np.ascontiguousarray(rhs, np.float64),
               levels=levels)
    out["n"] = (len(out["rp"]) - 1) * out["b"]
    out.update(extra)
    return out


def level(fmask, frelax="jacobi", sweeps=1, omega=1.0, restrict="injection", amg_unknown_based=False,
          amg_agg_levels=0):
    """One MGR reduction level: which fields are F-points and how they are handled."""
    return dict(fmask=int(fmask), frelax=frelax, sweeps=int(sweeps), omega=float(omega), restrict=restrict,
                amg_unknown_based=int(amg_unknown_based), amg_agg_levels=int(amg_agg_levels))


def _grid_neighbors(nx, ny, nz):
    """Faces of the 7-point stencil: arrays (c, d, axis) with d = c + offset."""
    idx = np.arange(nx * ny * nz).reshape(nz, ny, nx)
    out = []
    for axis, (sl_a, sl_b) in enumerate([((slice(None), slice(None), slice(0, -1)),
                                           (slice(None), slice(None), slice(1, None))),
                                          ((slice(None), slice(0, -1), slice(None)),
                                           (slice(None), slice(1, None), slice(None))),
                                          ((slice(0, -1), slice(None), slice(None)),
                                           (slice(1, None), slice(None), slice(None)))]):
        c = idx[sl_a].ravel()
        d = idx[sl_b].ravel()
        out.append((c, d, np.full(c.shape, axis)))
    c = np.concatenate([o[0] for o in out])
    d = np.concatenate([o[1] for o in out])
    ax = np.concatenate([o[2] for o in out])
    return c, d, ax


def _bsr_from_coo(nbr, b, brow, bcol, r, c, v):
    """Assemble b x b block-CSR from block-coordinate triplets (duplicates summed)."""
    key = brow.astype(np.int64) * nbr + bcol
    ukey, inv = np.unique(key, return_inverse=True)
    vals = np.zeros((len(ukey), b, b))
    np.add.at(vals, (inv, r, c), v)
    rows = (ukey // nbr).astype(np.int64)
    cols = (ukey % nbr).astype(np.int32)
    rp = np.zeros(nbr + 1, np.int64)
    np.add.at(rp, rows + 1, 1)
    rp = np.cumsum(rp)
    return rp.astype(np.int32), cols, vals.reshape(-1)


def two_field_tpfa(nx=16, ny=16, nz=16, seed=0):
    """Two-field cell-centred flow: p (field 0) and s (field 1) per cell,
    interleaved as 2c, 2c+1, stored as 2x2 blocks on the 7-point stencil.

    p-rows: TPFA Laplacian of harmonic transmissibilities + accumulation, and a
    saturation coupling at the upwind cell; s-rows: an upwind-weighted pressure
    Laplacian and an upwind transport operator + accumulation.
    log10 k ~ N(0,1) per cell; accumulation ~ U[0.1,1]; RHS ~ N(0,1)."""
    g = _rngs(seed)
    nc = nx * ny * nz
    k = 10.0 ** g["perm"].standard_normal(nc)
    ap = g["accum"].uniform(0.1, 1.0, nc)
    as_ = g["accum"].uniform(0.1, 1.0, nc)
    c, d, _ = _grid_neighbors(nx, ny, nz)
    T = 2.0 * k[c] * k[d] / (k[c] + k[d])
    gdir = g["upwind"].standard_normal(len(c))
    f = g["upwind"].uniform(0.0, 1.0, nc)
    fp = g["upwind"].uniform(0.0, 1.0, nc)
    u = np.where(gdir >= 0, c, d)
    o = np.where(gdir >= 0, d, c)
    ag = np.abs(gdir)
    trips = []  # (block row, block col, r, c, value)

    def add(br, bc, r, cc, v):
        trips.append((np.asarray(br), np.asarray(bc), np.full(np.shape(br), r), np.full(np.shape(br), cc),
                      np.asarray(v, dtype=np.float64)))

    # accumulation
    cells = np.arange(nc)
    add(cells, cells, 0, 0, ap)
    add(cells, cells, 1, 1, as_)
    # pressure Laplacian (p-row, p-col)
    add(c, c, 0, 0, T); add(c, d, 0, 0, -T); add(d, d, 0, 0, T); add(d, c, 0, 0, -T)
    # p-row, s-col at the upwind cell: + for the upstream cell's row, - downstream
    coup = 0.1 * T * ag * fp[u]
    add(c, u, 0, 1, np.where(u == c, coup, -coup))
    add(d, u, 0, 1, np.where(u == d, coup, -coup))
    # s-row, p-col: upwind-weighted Laplacian
    fu = f[u] * T
    add(c, c, 1, 0, fu); add(c, d, 1, 0, -fu); add(d, d, 1, 0, fu); add(d, c, 1, 0, -fu)
    # s-row, s-col: outflow on the upstream diagonal, inflow downstream
    tr = T * ag * fp[u]
    add(u, u, 1, 1, tr); add(o, u, 1, 1, -tr)
    # make sure every 7-point neighbour block exists (possibly with zeros)
    add(c, d, 0, 0, np.zeros(len(c))); add(d, c, 0, 0, np.zeros(len(c)))
    br = np.concatenate([t[0] for t in trips]); bc = np.concatenate([t[1] for t in trips])
    rr = np.concatenate([t[2] for t in trips]); cc = np.concatenate([t[3] for t in trips])
    vv = np.concatenate([t[4] for t in trips])
    rp, ci, vals = _bsr_from_coo(nc, 2, br, bc, rr, cc, vv)
    field = np.tile(np.array([0, 1], np.int32), nc)
    rhs = g["rhs"].standard_normal(2 * nc)
    levels = [level(1 << 1, "jacobi")]
    return _system(2, rp, ci, vals, field, rhs, levels, f"two_field_tpfa_{nx}x{ny}x{nz}", grid=(nx, ny, nz))


# G for the consistent-style local inner product: 1/8 between faces of
# different axes, 0 between a face and its opposite face.
def _g_matrix():
    ax = np.repeat(np.arange(3), 2)
    G = np.where(ax[:, None] != ax[None, :], 0.125, 0.0)
    return G


def hybrid_mimetic(nx=64, ny=64, nz=64, seed=1, consistent=True, upwind=True, nrhs=1, reduction="p"):
    """Statically condensed hybrid mimetic system on an nx x ny x nz hex grid.

    Unknowns: cell pressures (field 0, numbered first) then face multipliers
    (field 1: x-faces, y-faces, z-faces, each lexicographic).  Per cell K with
    half-transmissibilities t_f = 2 k_axis(f), T_K = diag(sqrt t)(I + G/2)diag(sqrt t)
    (G = 0 gives the TPFA variant), the local condensed block on [p_K; pi_f] is
        p-row:  a_K + sum_f u_f (T_K 1)_f,   -u_f (T_K 1)_f
        pi-row: -(T_K 1)_f,                  T_K
    with a_K ~ U[0.1,1] and upwind density factors u_f ~ U[0.9,1.1] (u_f = 1
    when upwind=False gives a symmetric system).  ln k_{x,y,z} ~ N(0, 2^2) i.i.d.
    So A_pp is diagonal, A_ppi has 6 entries per row and A_pipi is 11-point
    (diagonal in the TPFA variant, its off-diagonal entries stored as zeros).

    reduction="p" is MGR_P of Sec. 3.1 (F = cells, whose block A_pp is
    diagonal, so Jacobi interpolation is the ideal one; the faces go to AMG).
    reduction="pi" is MGR_Pi (F = faces, C = cells): ideal only where A_pipi is
    diagonal, that is in the TPFA variant, where the coarse system is the
    7-point cell Schur complement A_pp - A_ppi A_pipi^-1 A_pip."""
    if reduction not in ("p", "pi"):
        raise ValueError("reduction must be 'p' or 'pi'")
    g = _rngs(seed)
    ncell = nx * ny * nz
    nfx, nfy, nfz = (nx + 1) * ny * nz, nx * (ny + 1) * nz, nx * ny * (nz + 1)
    nface = nfx + nfy + nfz
    n = ncell + nface
    lnk = g["perm"].normal(0.0, 2.0, size=(ncell, 3))
    kk = np.exp(lnk)
    a = g["accum"].uniform(0.1, 1.0, ncell)
    uf = g["upwind"].uniform(0.9, 1.1, size=(ncell, 6)) if upwind else np.ones((ncell, 6))
    kz, ky, kx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    kx, ky, kz = kx.ravel(), ky.ravel(), kz.ravel()
    faces = np.stack([
        ncell + kx + (nx + 1) * (ky + ny * kz),
        ncell + (kx + 1) + (nx + 1) * (ky + ny * kz),
        ncell + nfx + kx + nx * (ky + (ny + 1) * kz),
        ncell + nfx + kx + nx * ((ky + 1) + (ny + 1) * kz),
        ncell + nfx + nfy + kx + nx * (ky + ny * kz),
        ncell + nfx + nfy + kx + nx * (ky + ny * (kz + 1)),
    ], axis=1)
    t = 2.0 * kk[:, np.repeat(np.arange(3), 2)]              # (ncell, 6)
    G = _g_matrix() if consistent else np.zeros((6, 6))
    st = np.sqrt(t)
    TK = st[:, :, None] * (np.eye(6)[None] + 0.5 * G[None]) * st[:, None, :]
    T1 = TK.sum(axis=2)
    cells = np.arange(ncell)
    rows = [cells, np.repeat(cells, 6), faces.ravel(), np.repeat(faces, 6, axis=1).ravel()]
    cols = [cells, faces.ravel(), np.repeat(cells, 6), np.tile(faces, (1, 6)).ravel()]
    vals = [a + (uf * T1).sum(axis=1), (-uf * T1).ravel(), (-T1).ravel(), TK.reshape(ncell, 36).ravel()]
    R = np.concatenate(rows); C = np.concatenate(cols); V = np.concatenate(vals)
    A = sp.coo_matrix((V, (R, C)), shape=(n, n)).tocsr()
    A.sum_duplicates()
    A.sort_indices()
    field = np.concatenate([np.zeros(ncell, np.int32), np.ones(nface, np.int32)])
    rhs = g["rhs"].standard_normal((nrhs, n)) if nrhs > 1 else g["rhs"].standard_normal(n)
    levels = [level(1 << 0 if reduction == "p" else 1 << 1, "jacobi")]
    extra = dict(grid=(nx, ny, nz), ncell=ncell, nface=nface)
    if nrhs > 1:
        extra["fd_rng"] = g["fd"]
        extra["loss_weights"] = g["loss"].standard_normal((nrhs, n))
    return _system(1, A.indptr, A.indices, A.data, field, rhs, levels,
                   f"hybrid_mimetic_{'consistent' if consistent else 'tpfa'}_{nx}x{ny}x{nz}"
                   + ("_mgr_pi" if reduction == "pi" else ""), **extra)


def compositional_wells(nx=128, ny=128, nz=64, seed=2, wells_per_axis=4, nperf=3, margin_p=1.1, margin_rho=2.0):
    """Compositional-style system: 4 unknowns per cell -- pressure (field 0) and
    three component densities (fields 1-3) -- as interleaved 4x4 blocks on the
    7-point stencil, plus vertical wells (well-pressure equation, field 4) each
    stored as one extra block row whose other three unknowns are identity
    padding (field 5).

    Off-diagonal block (c, d) = -T_cd W with W_00 = 1, W_{p,rho} and W_{rho,p}
    ~ U[0, 0.5], and W_{rho,rho'} ~ U[0, 0.5] only when d is upwind of c (random
    upwind direction per face); T_cd harmonic, log10 k ~ N(0,1).  Diagonal block:
    1.1 times the absolute row sum of the off-diagonal blocks plus an
    accumulation term U[0.1, 1] on the diagonal, intra-cell off-diagonals
    U[-0.1, 0.1] times the row's diagonal.  Wells sit at the centres of a
    wells_per_axis^2 lattice in (x, y), perforated in layers k = 0..nperf-1 with
    WI = 10^N(0,1) k_c: each equation e of a perforated cell gets -WI m_e in the
    well column and +WI m_e in its pressure column (m_e ~ U[0.5, 1]); the well
    row has sum(WI) + 1e-3 on the diagonal and -WI at each perforated pressure.
    Reduction order: components (+ padding) by block-Jacobi, then wells by
    Jacobi, then AMG on the cell pressures."""
    g = _rngs(seed)
    ncell = nx * ny * nz
    k = 10.0 ** g["perm"].standard_normal(ncell)
    acc = g["accum"].uniform(0.1, 1.0, (ncell, 4))
    kz, ky, kx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    kx, ky, kz = kx.ravel(), ky.ravel(), kz.ravel()
    cells = np.arange(ncell)
    offs = np.array([-nx * ny, -nx, -1, 0, 1, nx, nx * ny])
    exist = np.stack([kz > 0, ky > 0, kx > 0, np.ones(ncell, bool), kx < nx - 1, ky < ny - 1, kz < nz - 1], 1)
    # face flow direction for the + faces of every cell (x, y, z); >= 0 means from c to c+off
    gface = g["upwind"].standard_normal((ncell, 3))
    blocks = np.zeros((ncell, 8, 4, 4))
    for sl in (0, 1, 2, 4, 5, 6):
        m = exist[:, sl]
        c = cells[m]
        d = c + offs[sl]
        T = 2.0 * k[c] * k[d] / (k[c] + k[d])
        axis = {0: 2, 1: 1, 2: 0, 4: 0, 5: 1, 6: 2}[sl]
        if sl > 3:
            d_upwind = gface[c, axis] < 0.0       # flow from d to c
        else:
            d_upwind = gface[d, axis] >= 0.0      # flow from d (lower index) to c
        W = np.zeros((len(c), 4, 4))
        W[:, 0, 0] = 1.0
        W[:, 0, 1:] = g["noise"].uniform(0.0, 0.5, (len(c), 3))
        W[:, 1:, 0] = g["noise"].uniform(0.0, 0.5, (len(c), 3))
        W[:, 1:, 1:] = g["noise"].uniform(0.0, 0.5, (len(c), 3, 3)) * d_upwind[:, None, None]
        blocks[m, sl] = -T[:, None, None] * W
    rowabs = np.abs(blocks).sum(axis=(1, 3))            # (ncell, 4): off-diagonal blocks only so far
    diag = np.array([margin_p, margin_rho, margin_rho, margin_rho])[None, :] * rowabs + acc
    intra = g["noise"].uniform(-0.1, 0.1, (ncell, 4, 4)) * diag[:, :, None]
    intra[:, np.arange(4), np.arange(4)] = diag
    blocks[:, 3] = intra
    # wells
    pos = [(2 * m + 1) * nx // (2 * wells_per_axis) for m in range(wells_per_axis)]
    posy = [(2 * m + 1) * ny // (2 * wells_per_axis) for m in range(wells_per_axis)]
    wells = [(i, j) for j in posy for i in pos]
    nw = len(wells)
    nperf = min(nperf, nz)
    perf_cells = np.array([[i + nx * (j + ny * kk) for kk in range(nperf)] for (i, j) in wells])   # (nw, nperf)
    WI = (10.0 ** g["wells"].standard_normal((nw, nperf))) * k[perf_cells]
    me = g["wells"].uniform(0.5, 1.0, (nw, nperf, 4))
    wblk_cell = np.zeros((nw, nperf, 4, 4))       # block (cell, well): column 0 = well pressure
    wblk_cell[:, :, :, 0] = -WI[:, :, None] * me
    for w in range(nw):
        for q in range(nperf):
            blocks[perf_cells[w, q], 3, :, 0] += WI[w, q] * me[w, q]
    exist8 = np.concatenate([exist, np.zeros((ncell, 1), bool)], 1)
    has_well = np.zeros(ncell, np.int64) - 1
    for w in range(nw):
        for q in range(nperf):
            c = perf_cells[w, q]
            has_well[c] = w
            exist8[c, 7] = True
            blocks[c, 7] = wblk_cell[w, q]
    # block-CSR: cell rows (slots ascending by column), then well rows
    cnt = exist8.sum(1)
    well_cnt = np.full(nw, nperf + 1)
    rp = np.concatenate([[0], np.cumsum(np.concatenate([cnt, well_cnt]))]).astype(np.int64)
    colmat = cells[:, None] + np.concatenate([offs, [0]])[None, :]
    colmat[:, 7] = ncell + np.maximum(has_well, 0)
    ci_cells = colmat[exist8]
    vals_cells = blocks[exist8]
    del blocks
    ci_w, v_w = [], []
    for w in range(nw):
        for q in range(nperf):
            b = np.zeros((4, 4))
            b[0, 0] = -WI[w, q]
            ci_w.append(perf_cells[w, q]); v_w.append(b)
        b = np.eye(4)
        b[0, 0] = WI[w].sum() + 1e-3
        ci_w.append(ncell + w); v_w.append(b)
    ci = np.concatenate([ci_cells, np.array(ci_w, np.int64)]).astype(np.int32)
    vals = np.concatenate([vals_cells.reshape(-1), np.array(v_w).reshape(-1)])
    field = np.concatenate([np.tile(np.arange(4, dtype=np.int32), ncell),
                            np.tile(np.array([4, 5, 5, 5], np.int32), nw)])
    rhs = g["rhs"].standard_normal(4 * (ncell + nw))
    rhs[field == 5] = 0.0
    levels = [level((1 << 1) | (1 << 2) | (1 << 3) | (1 << 5), "block_jacobi"), level(1 << 4, "jacobi")]
    return _system(4, rp.astype(np.int32), ci, vals, field, rhs, levels,
                   f"compositional_wells_{nx}x{ny}x{nz}", grid=(nx, ny, nz), nwells=nw, ncell=ncell)


def compositional_4level(nx=128, ny=128, nz=64, seed=4, wells_per_axis=4, nperf=3, margin_p=1.1, margin_rho=2.0):
    """Compositional system in the paper's four-level form (Sec. 3.2): per cell
    the pressure p (field 0), the advected density rho_1 (field 1) and the
    density rho_2 of the volume-constraint equation (field 2), as interleaved
    3x3 blocks on the 7-point stencil; per well a bottom-hole pressure p_w
    (field 3) and a rate q_w (field 4), stored as one block row with an identity
    padding unknown (field 5).

    Cell rows: off-diagonal block (c, d) = -T_cd W with W_pp = 1, W_{p,rho} and
    W_{rho1,p} ~ U[0, 0.5], W_{rho1,rho} ~ U[0, 0.5] only when d is upwind of c,
    and a zero rho_2 row (the constraint is cell-local); diagonal = margin times
    the absolute off-diagonal row sum + U[0.1, 1] for p and rho_1, intra-cell
    couplings U[-0.1, 0.1] times the diagonal.  The rho_2 row couples only to
    its own cell: U[-0.5, 0.5] on p and rho_1, 1 + U[0, 1] on rho_2, so the
    rho_2 block and its couplings are diagonal.

    Wells at the centres of a wells_per_axis^2 lattice, perforated in layers
    0..nperf-1 with WI = 10^N(0,1) k_c.  A perforated cell's p and rho_1 rows
    gain WI m (p_c - p_w) (m = 1 for p, U[0.5, 1] for rho_1).  Well row p_w:
    sum(WI) p_w - sum(WI p_c) - q_w; well row q_w: q_w = target for a rate-
    controlled well, p_w = target for a pressure-controlled one (every other
    well), which leaves a zero on the diagonal of the well block.

    Reduction order (the paper's): rho_2 (+ padding) by Jacobi, which is exact
    here; rho_1 by Jacobi; p by an AMG V-cycle as F-relaxation; the well system
    is the coarse grid (solved directly: it has fewer unknowns than the AMG's
    coarsest size)."""
    g = _rngs(seed)
    ncell = nx * ny * nz
    k = 10.0 ** g["perm"].standard_normal(ncell)
    acc = g["accum"].uniform(0.1, 1.0, (ncell, 2))
    kz, ky, kx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    kx, ky, kz = kx.ravel(), ky.ravel(), kz.ravel()
    cells = np.arange(ncell)
    offs = np.array([-nx * ny, -nx, -1, 0, 1, nx, nx * ny])
    exist = np.stack([kz > 0, ky > 0, kx > 0, np.ones(ncell, bool), kx < nx - 1, ky < ny - 1, kz < nz - 1], 1)
    gface = g["upwind"].standard_normal((ncell, 3))
    blocks = np.zeros((ncell, 8, 3, 3))
    for sl in (0, 1, 2, 4, 5, 6):
        m = exist[:, sl]
        c = cells[m]
        d = c + offs[sl]
        T = 2.0 * k[c] * k[d] / (k[c] + k[d])
        axis = {0: 2, 1: 1, 2: 0, 4: 0, 5: 1, 6: 2}[sl]
        d_upwind = (gface[c, axis] < 0.0) if sl > 3 else (gface[d, axis] >= 0.0)
        W = np.zeros((len(c), 3, 3))
        W[:, 0, 0] = 1.0
        W[:, 0, 1:] = g["noise"].uniform(0.0, 0.5, (len(c), 2))
        W[:, 1, 0] = g["noise"].uniform(0.0, 0.5, len(c))
        W[:, 1, 1:] = g["noise"].uniform(0.0, 0.5, (len(c), 2)) * d_upwind[:, None]
        blocks[m, sl] = -T[:, None, None] * W
    rowabs = np.abs(blocks).sum(axis=(1, 3))[:, :2]
    diag = np.array([margin_p, margin_rho])[None, :] * rowabs + acc
    intra = np.zeros((ncell, 3, 3))
    intra[:, :2, :] = g["noise"].uniform(-0.1, 0.1, (ncell, 2, 3)) * diag[:, :, None]
    intra[:, 0, 0] = diag[:, 0]
    intra[:, 1, 1] = diag[:, 1]
    intra[:, 2, :2] = g["noise"].uniform(-0.5, 0.5, (ncell, 2))
    intra[:, 2, 2] = 1.0 + g["noise"].uniform(0.0, 1.0, ncell)
    blocks[:, 3] = intra
    # wells
    pos = [(2 * m + 1) * nx // (2 * wells_per_axis) for m in range(wells_per_axis)]
    posy = [(2 * m + 1) * ny // (2 * wells_per_axis) for m in range(wells_per_axis)]
    wells = [(i, j) for j in posy for i in pos]
    nw = len(wells)
    nperf = min(nperf, nz)
    perf_cells = np.array([[i + nx * (j + ny * kk) for kk in range(nperf)] for (i, j) in wells])
    WI = (10.0 ** g["wells"].standard_normal((nw, nperf))) * k[perf_cells]
    mob = np.stack([np.ones((nw, nperf)), g["wells"].uniform(0.5, 1.0, (nw, nperf))], -1)   # p, rho_1 rows
    exist8 = np.concatenate([exist, np.zeros((ncell, 1), bool)], 1)
    has_well = np.full(ncell, -1)
    for w in range(nw):
        for q in range(nperf):
            c = perf_cells[w, q]
            blocks[c, 3, :2, 0] += WI[w, q] * mob[w, q]
            has_well[c] = w
            exist8[c, 7] = True
            blocks[c, 7, :2, 0] = -WI[w, q] * mob[w, q]       # column 0 of the well block = p_w
    cnt = exist8.sum(1)
    rp = np.concatenate([[0], np.cumsum(np.concatenate([cnt, np.full(nw, nperf + 1)]))]).astype(np.int64)
    colmat = cells[:, None] + np.concatenate([offs, [0]])[None, :]
    colmat[:, 7] = ncell + np.maximum(has_well, 0)
    ci_cells = colmat[exist8]
    vals_cells = blocks[exist8]
    del blocks
    ci_w, v_w = [], []
    for w in range(nw):
        for q in range(nperf):
            b = np.zeros((3, 3))
            b[0, 0] = -WI[w, q]
            ci_w.append(perf_cells[w, q]); v_w.append(b)
        b = np.zeros((3, 3))
        b[0, 0] = WI[w].sum()
        b[0, 1] = -1.0
        if w % 2 == 0:
            b[1, 1] = 1.0            # rate control: q_w = target
        else:
            b[1, 0] = 1.0            # pressure control: p_w = target (zero diagonal at q_w)
        b[2, 2] = 1.0
        ci_w.append(ncell + w); v_w.append(b)
    ci = np.concatenate([ci_cells, np.array(ci_w, np.int64)]).astype(np.int32)
    vals = np.concatenate([vals_cells.reshape(-1), np.array(v_w).reshape(-1)])
    field = np.concatenate([np.tile(np.arange(3, dtype=np.int32), ncell),
                            np.tile(np.array([3, 4, 5], np.int32), nw)])
    rhs = g["rhs"].standard_normal(3 * (ncell + nw))
    rhs[field == 5] = 0.0
    levels = [level((1 << 2) | (1 << 5), "jacobi"), level(1 << 1, "jacobi"), level(1 << 0, "amg")]
    return _system(3, rp.astype(np.int32), ci, vals, field, rhs, levels,
                   f"compositional_4level_{nx}x{ny}x{nz}", grid=(nx, ny, nz), nwells=nw, ncell=ncell)


def _q1_reference_stiffness(nu):
    """24x24 stiffness of the unit trilinear hex for E = 1 (2x2x2 Gauss points),
    dofs ordered (node a, component c) -> 3a + c, nodes in (x fastest) order."""
    lam = nu / ((1 + nu) * (1 - 2 * nu))
    mu = 1.0 / (2 * (1 + nu))
    D = np.zeros((6, 6))
    D[:3, :3] = lam
    D[np.arange(3), np.arange(3)] += 2 * mu
    D[np.arange(3, 6), np.arange(3, 6)] = mu
    corners = np.array([[(a >> 0) & 1, (a >> 1) & 1, (a >> 2) & 1] for a in range(8)], float)
    gp = np.array([0.5 - 0.5 / np.sqrt(3), 0.5 + 0.5 / np.sqrt(3)])
    K = np.zeros((24, 24))
    for x in gp:
        for y in gp:
            for z in gp:
                q = np.array([x, y, z])
                dN = np.zeros((8, 3))
                for a in range(8):
                    f = np.where(corners[a] == 1, q, 1 - q)
                    sgn = np.where(corners[a] == 1, 1.0, -1.0)
                    dN[a] = [sgn[0] * f[1] * f[2], f[0] * sgn[1] * f[2], f[0] * f[1] * sgn[2]]
                B = np.zeros((6, 24))
                for a in range(8):
                    B[0, 3 * a] = dN[a, 0]; B[1, 3 * a + 1] = dN[a, 1]; B[2, 3 * a + 2] = dN[a, 2]
                    B[3, 3 * a] = dN[a, 1]; B[3, 3 * a + 1] = dN[a, 0]
                    B[4, 3 * a + 1] = dN[a, 2]; B[4, 3 * a + 2] = dN[a, 1]
                    B[5, 3 * a] = dN[a, 2]; B[5, 3 * a + 2] = dN[a, 0]
                K += B.T @ D @ B / 8.0
    return K, corners.astype(int)


def fracturing(nn=96, seed=3, nu=0.25, cs=0.1, storage=1e-2, reduction="u"):
    """Hydraulic-fracturing-style system (Sec. 3.3, App. C): Q1 hexahedral
    elasticity on an nn^3 node grid (3 displacement unknowns per node, fields
    0-2), Young's modulus per element with ln E ~ N(0,1), Poisson ratio 0.25,
    Dirichlet outer boundary (identity rows, couplings removed), coupled to a
    planar fracture of nn x nn cells on the node plane y = nn/2 (one pressure
    per cell, field 3, grouped three per 3x3 block row).

    Fracture flow: 5-point cubic-law stencil with T = harmonic mean of w^3/12
    (aperture ln w ~ N(0, 0.5^2), unit viscosity) plus a storage term 1e-2.
    Coupling at the node tied to each interior cell: -1 from pressure into the
    node's u_y equation (traction) and +cs from u_y into the cell's mass balance
    (aperture storage), so the pressure Schur complement gains a positive term.
    reduction="u" is MGR_U of Sec. 3.3: F = displacements, F-relaxation one
    unknown-based AMG V-cycle on A_uu, Jacobi interpolation, injection; AMG on
    the coarse pressure system.  reduction="p" is MGR_P, the other order of
    Sec. 3.3: F = fracture pressures, F-relaxation one AMG V-cycle on A_pp,
    Jacobi interpolation, injection; the coarse system A_uu - A_up D_pp^-1 A_pu
    goes to unknown-based AMG over the three displacement components."""
    if reduction not in ("u", "p"):
        raise ValueError("reduction must be 'u' or 'p'")
    if (nn * nn) % 3:
        raise ValueError("nn^2 must be a multiple of 3 (pressures are grouped three per block row)")
    g = _rngs(seed)
    ne = nn - 1
    nnode = nn ** 3
    E = np.exp(g["perm"].standard_normal(ne ** 3))
    K0, corners = _q1_reference_stiffness(nu)
    ez, ey, ex = np.meshgrid(np.arange(ne), np.arange(ne), np.arange(ne), indexing="ij")
    ex, ey, ez = ex.ravel(), ey.ravel(), ez.ravel()
    nid = lambda x, y, z: x + nn * (y + nn * z)
    # 27-slot layout: slot of offset (dx,dy,dz) = (dx+1) + 3(dy+1) + 9(dz+1); ascending slot = ascending column
    blocks = np.zeros((nnode, 27, 3, 3))
    for a in range(8):
        na = nid(ex + corners[a, 0], ey + corners[a, 1], ez + corners[a, 2])
        for b in range(8):
            d = corners[b] - corners[a]
            slot = (d[0] + 1) + 3 * (d[1] + 1) + 9 * (d[2] + 1)
            blocks[na, slot] += E[:, None, None] * K0[3 * a:3 * a + 3, 3 * b:3 * b + 3][None]
    kz, ky, kx = np.meshgrid(np.arange(nn), np.arange(nn), np.arange(nn), indexing="ij")
    kx, ky, kz = kx.ravel(), ky.ravel(), kz.ravel()
    interior = (kx > 0) & (kx < nn - 1) & (ky > 0) & (ky < nn - 1) & (kz > 0) & (kz < nn - 1)
    exist = np.zeros((nnode, 28), bool)
    cols = np.zeros((nnode, 28), np.int64)
    for slot in range(27):
        dx, dy, dz = slot % 3 - 1, (slot // 3) % 3 - 1, slot // 9 - 1
        x, y, z = kx + dx, ky + dy, kz + dz
        inside = (x >= 0) & (x < nn) & (y >= 0) & (y < nn) & (z >= 0) & (z < nn)
        nb = np.where(inside, nid(np.clip(x, 0, nn - 1), np.clip(y, 0, nn - 1), np.clip(z, 0, nn - 1)), 0)
        exist[:, slot] = interior & inside & interior[nb]
        cols[:, slot] = nb
    # Dirichlet boundary nodes: identity diagonal block only
    bnd = ~interior
    blocks[bnd] = 0.0
    blocks[bnd, 13] = np.eye(3)
    exist[bnd, 13] = True
    # fracture
    jf = nn // 2
    ncell = nn * nn
    w = np.exp(0.5 * g["noise"].standard_normal(ncell))
    tw = w ** 3 / 12.0
    ci_, ck_ = np.meshgrid(np.arange(nn), np.arange(nn), indexing="ij")   # cell q = i + nn k
    ci_, ck_ = ci_.T.ravel(), ck_.T.ravel()
    q_of = lambda i, k: i + nn * k
    node_of_cell = nid(ci_, np.full(ncell, jf), ck_)
    coupled = interior[node_of_cell]
    pr0 = nnode            # block row of the first pressure triple
    # node rows: one extra block in the node's row for its cell's pressure triple
    qc = np.arange(ncell)[coupled]
    mc = node_of_cell[coupled]
    exist[mc, 27] = True
    cols[mc, 27] = pr0 + qc // 3
    extra = np.zeros((nnode, 3, 3))
    extra[mc, 1, qc % 3] = -1.0
    # pressure rows as block triplets
    trip_r, trip_c, trip_i, trip_j, trip_v = [], [], [], [], []
    def addp(qa, col_block, i_in, j_in, v):
        trip_r.append(qa // 3); trip_c.append(col_block); trip_i.append(qa % 3); trip_j.append(j_in); trip_v.append(v)
    diag = np.full(ncell, storage)
    for (di, dk) in ((1, 0), (0, 1)):
        m = (ci_ + di < nn) & (ck_ + dk < nn)
        qa = np.arange(ncell)[m]
        qb = q_of(ci_[m] + di, ck_[m] + dk)
        T = 2 * tw[qa] * tw[qb] / (tw[qa] + tw[qb])
        np.add.at(diag, qa, T); np.add.at(diag, qb, T)
        addp(qa, pr0 + qb // 3, None, qb % 3, -T)
        addp(qb, pr0 + qa // 3, None, qa % 3, -T)
    q = np.arange(ncell)
    addp(q, pr0 + q // 3, None, q % 3, diag)
    addp(qc, mc, None, np.full(len(qc), 1), np.full(len(qc), cs))
    R = np.concatenate(trip_r); C = np.concatenate(trip_c); I = np.concatenate(trip_i)
    J = np.concatenate([np.broadcast_to(j, np.shape(r)) for j, r in zip(trip_j, trip_r)])
    V = np.concatenate(trip_v)
    npr = ncell // 3
    key = R.astype(np.int64) * (nnode + npr) + C
    ukey, inv = np.unique(key, return_inverse=True)
    pvals = np.zeros((len(ukey), 3, 3))
    np.add.at(pvals, (inv, I, J), V)
    prow = ukey // (nnode + npr)
    pcol = ukey % (nnode + npr)
    # assemble
    cnt_nodes = exist.sum(1)
    cnt_p = np.bincount(prow, minlength=npr)
    rp = np.concatenate([[0], np.cumsum(np.concatenate([cnt_nodes, cnt_p]))])
    allblocks = np.concatenate([blocks, extra[:, None]], axis=1)
    del blocks
    vals = np.concatenate([allblocks[exist].reshape(-1), pvals.reshape(-1)])
    ci = np.concatenate([cols[exist], pcol]).astype(np.int32)
    del allblocks
    field = np.concatenate([np.tile(np.arange(3, dtype=np.int32), nnode), np.full(ncell, 3, np.int32)])
    rhs = g["rhs"].standard_normal(3 * nnode + ncell)
    rhs[:3 * nnode][np.repeat(bnd, 3)] = 0.0
    # two L1-Jacobi sweeps per side stand in for the paper's hybrid L1 Gauss-Seidel
    if reduction == "u":
        levels = [level((1 << 0) | (1 << 1) | (1 << 2), "amg", amg_unknown_based=True)]
        opts = dict(nu_pre=2, nu_post=2)
    else:
        levels = [level(1 << 3, "amg")]
        opts = dict(nu_pre=2, nu_post=2, unknown_based=True)
    return _system(3, rp.astype(np.int32), ci, vals, field, rhs, levels,
                   f"fracturing_{nn}^3" + ("_mgr_p" if reduction == "p" else ""),
                   nnode=nnode, ncell=ncell, solver_opts=opts)


def csr_of(system):
    """Scalar scipy CSR view of a generated system (block layout expanded)."""
    b = system["b"]
    nbr = len(system["rp"]) - 1
    if b == 1:
        return sp.csr_matrix((system["vals"], system["ci"], system["rp"]), shape=(nbr, nbr))
    blocks = system["vals"].reshape(-1, b, b)
    return sp.bsr_matrix((blocks, system["ci"], system["rp"]), shape=(nbr * b, nbr * b)).tocsr()


WORKLOADS = {
    "two_field_tpfa_16^3": lambda: two_field_tpfa(16, 16, 16, seed=0),
    "hybrid_mimetic_64^3": lambda: hybrid_mimetic(64, 64, 64, seed=1),
    "compositional_wells_128x128x64": lambda: compositional_wells(128, 128, 64, seed=2),
    "fracturing_96^3": lambda: fracturing(96, seed=3),
}


def workload(name):
    """A full-size synthetic workload by name (the keys of WORKLOADS)."""
    return WORKLOADS[name]()
