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


def level(fmask, frelax="jacobi", sweeps=1, omega=1.0, restrict="injection", amg_unknown_based=False):
    """One MGR reduction level: which fields are F-points and how they are handled."""
    return dict(fmask=int(fmask), frelax=frelax, sweeps=int(sweeps), omega=float(omega), restrict=restrict,
                amg_unknown_based=bool(amg_unknown_based))


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


def hybrid_mimetic(nx=64, ny=64, nz=64, seed=1, consistent=True, upwind=True, nrhs=1):
    """Statically condensed hybrid mimetic system on an nx x ny x nz hex grid.

    Unknowns: cell pressures (field 0, numbered first) then face multipliers
    (field 1: x-faces, y-faces, z-faces, each lexicographic).  Per cell K with
    half-transmissibilities t_f = 2 k_axis(f), T_K = diag(sqrt t)(I + G/2)diag(sqrt t)
    (G = 0 gives the TPFA variant), the local condensed block on [p_K; pi_f] is
        p-row:  a_K + sum_f u_f (T_K 1)_f,   -u_f (T_K 1)_f
        pi-row: -(T_K 1)_f,                  T_K
    with a_K ~ U[0.1,1] and upwind density factors u_f ~ U[0.9,1.1] (u_f = 1
    when upwind=False gives a symmetric system).  ln k_{x,y,z} ~ N(0, 2^2) i.i.d.
    So A_pp is diagonal, A_ppi has 6 entries per row and A_pipi is 11-point."""
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
    levels = [level(1 << 0, "jacobi")]
    extra = dict(grid=(nx, ny, nz), ncell=ncell, nface=nface)
    if nrhs > 1:
        extra["fd_rng"] = g["fd"]
        extra["loss_weights"] = g["loss"].standard_normal((nrhs, n))
    return _system(1, A.indptr, A.indices, A.data, field, rhs, levels,
                   f"hybrid_mimetic_{'consistent' if consistent else 'tpfa'}_{nx}x{ny}x{nz}", **extra)


def csr_of(system):
    """Scalar scipy CSR view of a generated system (block layout expanded)."""
    b = system["b"]
    nbr = len(system["rp"]) - 1
    if b == 1:
        return sp.csr_matrix((system["vals"], system["ci"], system["rp"]), shape=(nbr, nbr))
    blocks = system["vals"].reshape(-1, b, b)
    return sp.bsr_matrix((blocks, system["ci"], system["rp"]), shape=(nbr * b, nbr * b)).tocsr()


CONFIGS = {
    0: lambda: two_field_tpfa(16, 16, 16, seed=0),
    1: lambda: hybrid_mimetic(64, 64, 64, seed=1),
}


def config(k):
    """The benchmark workloads by index (see the module docstring)."""
    return CONFIGS[k]()
