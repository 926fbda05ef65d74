"""FP64 CPU oracle for MGR-preconditioned FGMRES (test infrastructure only).

This package is the independent reference the HIP library is checked against.
Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
import it; the GPU library never calls it and shares no code with it.

The arithmetic lives in ``mgr_oracle.c`` (plain C, built with
``-O2 -ffp-contract=off``); this module only marshals numpy arrays through
ctypes.  Every step cites the paper (Bui et al., arXiv 2101.11649) in the C
source.  Parity is pinned by the CPU tests in ``tests/test_oracle_*.py``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mgr_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

FRELAX = {"jacobi": 0, "block_jacobi": 1, "ilu0": 2, "amg": 3}
SMOOTHER = {"l1-jacobi": 0, "hybrid-gs": 1}
RESTRICT = {"injection": 0, "jacobi": 1}


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no contraction, no fast-math, no -march;
    OpenMP for the solve phase's row loops, whose results do not depend on
    the thread count)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c11", "-fopenmp", "-fPIC", "-shared",
               "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i32, f64, u64 = ctypes.c_int, ctypes.c_double, ctypes.c_ulonglong
        L.orc_setup.restype = P
        L.orc_setup.argtypes = [i32, i32, P, P, P, P, i32, P, P, P, P, P, P, P, f64, i32, i32, i32, i32, i32, i32,
                                i32, i32, i32, u64, P, P]
        L.orc_update.restype = P
        L.orc_update.argtypes = [P, i32, i32, P, P, P, P, i32, P, P, P, P, P, P, P, f64, i32, i32, i32, i32, i32,
                                 i32, i32, i32, i32, u64, P, i32, P]
        L.orc_free.argtypes = [P]
        L.orc_apply.argtypes = [P, P, P, i32]
        L.orc_matvec.argtypes = [P, P, P, i32]
        L.orc_solve.argtypes = [P, i32, P, P, i32, i32, f64, i32, P, P, P, P]
        L.orc_grad_values.argtypes = [i32, i32, P, P, i32, P, P, P]
        L.orc_info.argtypes = [P, P, i32]
        L.orc_export.argtypes = [P, i32, i32, i32, i32, P, P, P, P]
        L.orc_csr_spgemm.restype = P
        L.orc_csr_spgemm.argtypes = [i32, i32, P, P, P, i32, i32, P, P, P]
        L.orc_csr_add.restype = P
        L.orc_csr_add.argtypes = [i32, i32, P, P, P, P, P, P]
        L.orc_csr_transpose.restype = P
        L.orc_csr_transpose.argtypes = [i32, i32, P, P, P]
        L.orc_box_sizes.argtypes = [P, P]
        L.orc_box_copy.argtypes = [P, P, P, P]
        L.orc_box_free.argtypes = [P]
        L.orc_strength.argtypes = [i32, P, P, P, f64, P, P]
        L.orc_pmis.argtypes = [i32, P, P, P, u64, i32, P]
        L.orc_pmis_uniform.restype = f64
        L.orc_pmis_uniform.argtypes = [u64, i32, i32]
        L.orc_direct_interp.restype = P
        L.orc_direct_interp.argtypes = [i32, P, P, P, P, P, P, P]
        L.orc_aggressive_split.argtypes = [i32, P, P, P, u64, i32, P]
        L.orc_multipass_interp.restype = P
        L.orc_multipass_interp.argtypes = [i32, P, P, P, P, P, P, P]
        L.orc_ext_interp.restype = P
        L.orc_ext_interp.argtypes = [i32, P, P, P, P, P, P, P]
        L.orc_lu_solve.argtypes = [i32, P, P, P, i32]
        L.orc_small_inverse.argtypes = [i32, P, P]
        L.orc_set_threads.argtypes = [i32]
        L.orc_ilu0.argtypes = [i32, P, P, P, P, P]
        L.orc_ilu0_solve.argtypes = [i32, P, P, P, P, P, P, i32]
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


@dataclass
class Csr:
    nr: int
    nc: int
    rp: np.ndarray
    ci: np.ndarray
    v: np.ndarray

    def to_scipy(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.v, self.ci, self.rp), shape=(self.nr, self.nc))


def _unbox(box) -> Csr:
    L = lib()
    sizes = np.zeros(3, np.int64)
    L.orc_box_sizes(box, _p(sizes))
    nr, nc, nnz = (int(s) for s in sizes)
    rp = np.zeros(nr + 1, np.int32)
    ci = np.zeros(max(nnz, 1), np.int32)
    v = np.zeros(max(nnz, 1), np.float64)
    L.orc_box_copy(box, _p(rp), _p(ci), _p(v))
    L.orc_box_free(box)
    return Csr(nr, nc, rp, ci[:nnz], v[:nnz])


def _csr_args(a):
    a = a.tocsr() if hasattr(a, "tocsr") else a
    if hasattr(a, "indptr"):
        a.sort_indices()
        return a.shape[0], a.shape[1], _i32(a.indptr), _i32(a.indices), _f64(a.data)
    return a.nr, a.nc, _i32(a.rp), _i32(a.ci), _f64(a.v)


def spgemm(a, b) -> Csr:
    """C = A B (Gustavson order, symbolic pattern kept)."""
    an, am, arp, aci, av = _csr_args(a)
    bn, bm, brp, bci, bv = _csr_args(b)
    return _unbox(lib().orc_csr_spgemm(an, am, _p(arp), _p(aci), _p(av), bn, bm, _p(brp), _p(bci), _p(bv)))


def csr_add(a, b) -> Csr:
    an, am, arp, aci, av = _csr_args(a)
    _, _, brp, bci, bv = _csr_args(b)
    return _unbox(lib().orc_csr_add(an, am, _p(arp), _p(aci), _p(av), _p(brp), _p(bci), _p(bv)))


def transpose(a) -> Csr:
    an, am, arp, aci, av = _csr_args(a)
    return _unbox(lib().orc_csr_transpose(an, am, _p(arp), _p(aci), _p(av)))


def strength(a, theta: float, label=None) -> np.ndarray:
    n, _, rp, ci, v = _csr_args(a)
    strong = np.zeros(max(len(ci), 1), np.uint8)
    lab = None if label is None else _i32(label)
    lib().orc_strength(n, _p(rp), _p(ci), _p(v), float(theta), _p(lab), _p(strong))
    return strong[: len(ci)]


def pmis(a, strong, seed: int, level: int = 0):
    """Returns (cf with +1 = C / -1 = F, number of rounds)."""
    n, _, rp, ci, _ = _csr_args(a)
    cf = np.zeros(n, np.int32)
    s = np.ascontiguousarray(strong, dtype=np.uint8)
    if s.size == 0:
        s = np.zeros(1, np.uint8)
    rounds = lib().orc_pmis(n, _p(rp), _p(ci), _p(s), int(seed), int(level), _p(cf))
    return cf, rounds


def pmis_uniform(seed: int, level: int, i: int) -> float:
    return lib().orc_pmis_uniform(int(seed), int(level), int(i))


def direct_interp(a, strong, cf, label=None):
    n, _, rp, ci, v = _csr_args(a)
    st = ctypes.c_int(0)
    s = np.ascontiguousarray(strong, dtype=np.uint8)
    if s.size == 0:
        s = np.zeros(1, np.uint8)
    lab = None if label is None else _i32(label)
    box = lib().orc_direct_interp(n, _p(rp), _p(ci), _p(v), _p(s), _p(_i32(cf)), _p(lab), ctypes.byref(st))
    return _unbox(box), st.value


def aggressive_split(a, strong, seed: int, level: int = 0):
    """C/F split of an aggressively coarsened level (+1 = C, -1 = F)."""
    n, _, rp, ci, _ = _csr_args(a)
    cf = np.zeros(n, np.int32)
    s = np.ascontiguousarray(strong, dtype=np.uint8)
    if s.size == 0:
        s = np.zeros(1, np.uint8)
    lib().orc_aggressive_split(n, _p(rp), _p(ci), _p(s), int(seed), int(level), _p(cf))
    return cf


def multipass_interp(a, strong, cf, label=None):
    """Multi-pass interpolation of an aggressively coarsened level: (P, status)."""
    n, _, rp, ci, v = _csr_args(a)
    st = ctypes.c_int(0)
    s = np.ascontiguousarray(strong, dtype=np.uint8)
    if s.size == 0:
        s = np.zeros(1, np.uint8)
    lab = None if label is None else _i32(label)
    box = lib().orc_multipass_interp(n, _p(rp), _p(ci), _p(v), _p(s), _p(_i32(cf)), _p(lab), ctypes.byref(st))
    return _unbox(box), st.value


def ext_interp(a, strong, cf, label=None):
    """Extended+i interpolation (distance two) of the AMG setup: (P, status)."""
    n, _, rp, ci, v = _csr_args(a)
    st = ctypes.c_int(0)
    s = np.ascontiguousarray(strong, dtype=np.uint8)
    if s.size == 0:
        s = np.zeros(1, np.uint8)
    lab = None if label is None else _i32(label)
    box = lib().orc_ext_interp(n, _p(rp), _p(ci), _p(v), _p(s), _p(_i32(cf)), _p(lab), ctypes.byref(st))
    return _unbox(box), st.value


INTERP = {"direct": 0, "ext+i": 1}


def lu_solve(dense, b, trans: bool = False):
    m = _f64(dense)
    n = m.shape[0]
    x = np.zeros(n)
    st = lib().orc_lu_solve(n, _p(m), _p(_f64(b)), _p(x), int(trans))
    return x, st


def small_inverse(blk):
    b = _f64(blk)
    bs = b.shape[0]
    inv = np.zeros((bs, bs))
    st = lib().orc_small_inverse(bs, _p(b), _p(inv))
    return inv, st


def set_threads(n: int) -> int:
    """Threads for the oracle's solve phase (matvec, cycles, FGMRES vector
    work); 0 keeps the current setting.  Returns the number in use."""
    return lib().orc_set_threads(int(n))


def ilu0(a):
    """ILU(0) of a square CSR matrix on its own pattern: (lu values on a's
    pattern with L strictly below the diagonal (unit diagonal implied) and U on
    and above it, positions of the diagonal entries, status)."""
    n, _, rp, ci, v = _csr_args(a)
    lu = np.zeros(max(len(ci), 1))
    diag = np.zeros(n, np.int32)
    st = lib().orc_ilu0(n, _p(rp), _p(ci), _p(v), _p(lu), _p(diag))
    return lu[: len(ci)], diag, st


def ilu0_solve(a, lu, diag, r, trans: bool = False):
    """z = (LU)^{-1} r, or (LU)^{-T} r, with the factors of ilu0(a)."""
    n, _, rp, ci, _ = _csr_args(a)
    z = np.zeros(n)
    lib().orc_ilu0_solve(n, _p(rp), _p(ci), _p(_f64(lu)), _p(_i32(diag)), _p(_f64(r)), _p(z), int(trans))
    return z


def grad_values(b: int, rp, ci, lam, x):
    """dL/dA on the block pattern: -sum_k lam_k[row] x_k[col]; lam, x are (nrhs, n)."""
    rp, ci = _i32(rp), _i32(ci)
    lam = _f64(np.atleast_2d(lam))
    x = _f64(np.atleast_2d(x))
    nbr = len(rp) - 1
    out = np.zeros(int(rp[-1]) * b * b)
    lib().orc_grad_values(b, nbr, _p(rp), _p(ci), lam.shape[0], _p(lam), _p(x), _p(out))
    return out


@dataclass
class SolveInfo:
    status: int
    iterations: int
    restarts: int
    rel_res_est: float
    rel_res_true: float


@dataclass
class LevelOpts:
    fmask: int
    frelax: str = "jacobi"
    sweeps: int = 1
    omega: float = 1.0
    restrict: str = "injection"
    amg_unknown_based: int = 0      # 0 scalar, 1 unknown approach, 2 on the separate-component approximation
    amg_agg_levels: int = 0


class MGR:
    """Oracle MGR hierarchy + FGMRES for a block-CSR system.

    Parameters mirror the C-ABI of the GPU library: block size ``b`` (1 = CSR),
    block row pointers / columns / values (b*b row-major per block), the field
    label of every scalar unknown, a list of LevelOpts (one per MGR level), and
    AMG options for the final coarse system (``interp``: "direct" or "ext+i"
    interpolation, also used by the F-relaxation AMG hierarchies).  ``block``:
    optional group id of every scalar unknown for block-Jacobi F-relaxation
    (a block is a run of consecutive F-points with one id); default: the
    block row of the input layout.  ``smoother``: the AMG smoother, "l1-jacobi"
    or "hybrid-gs" (hybrid L1 Gauss-Seidel, forward on the way down and
    backward on the way up, over chunks of ``chunk`` consecutive rows).
    ``agg_levels``: the coarse AMG's first levels with aggressive coarsening
    and multi-pass interpolation (LevelOpts.amg_agg_levels for the AMG used as
    F-relaxation).
    """

    def __init__(self, b, rp, ci, vals, field, levels, theta=0.25, max_levels=25, max_coarse=128,
                 nu_pre=1, nu_post=1, coarse_unknown_based=False, seed=12345, interp="direct", block=None,
                 smoother="l1-jacobi", chunk=32, agg_levels=0):
        L = lib()
        self.b = int(b)
        self.rp, self.ci, self.vals = _i32(rp), _i32(ci), _f64(vals)
        self.n = (len(self.rp) - 1) * self.b
        self.field = _i32(field)
        nl = len(levels)
        fmask = np.array([lv.fmask for lv in levels] or [0], np.uint32)
        frelax = _i32([FRELAX[lv.frelax] for lv in levels] or [0])
        sweeps = _i32([lv.sweeps for lv in levels] or [0])
        omega = _f64([lv.omega for lv in levels] or [0])
        restr = _i32([RESTRICT[lv.restrict] for lv in levels] or [0])
        aub = _i32([int(lv.amg_unknown_based) for lv in levels] or [0])
        aag = _i32([int(lv.amg_agg_levels) for lv in levels] or [0])
        self._lv = (nl, fmask, frelax, sweeps, omega, restr, aub, aag)
        self._amg = (float(theta), int(max_levels), int(max_coarse), int(nu_pre), int(nu_post),
                     int(coarse_unknown_based), int(agg_levels), INTERP[interp], SMOOTHER[smoother], int(chunk),
                     int(seed))
        self.block = None if block is None else _i32(block)
        st = ctypes.c_int(0)
        self.h = L.orc_setup(self.b, len(self.rp) - 1, _p(self.rp), _p(self.ci), _p(self.vals), _p(self.field),
                             nl, *[_p(a) for a in self._lv[1:]], *self._amg,
                             None if self.block is None else _p(self.block), ctypes.byref(st))
        self.status = st.value

    def update(self, vals, keep_frelax_amg=False):
        """Setup reuse for new values on the same pattern: a new hierarchy whose
        AMG parts keep this one's C/F splits and interpolation (their Galerkin
        products are formed again), or, with keep_frelax_amg, keep the
        F-relaxation AMG hierarchies whole.  Returns the new MGR."""
        new = MGR.__new__(MGR)
        new.b, new.rp, new.ci, new.n, new.field, new.block = self.b, self.rp, self.ci, self.n, self.field, self.block
        new.vals = _f64(vals)
        new._lv, new._amg = self._lv, self._amg
        st = ctypes.c_int(0)
        new.h = lib().orc_update(self.h, self.b, len(self.rp) - 1, _p(self.rp), _p(self.ci), _p(new.vals),
                                 _p(self.field), self._lv[0], *[_p(a) for a in self._lv[1:]], *self._amg,
                                 None if self.block is None else _p(self.block), int(bool(keep_frelax_amg)),
                                 ctypes.byref(st))
        new.status = st.value
        return new

    def __del__(self):
        if getattr(self, "h", None):
            lib().orc_free(self.h)
            self.h = None

    def apply(self, v, trans=False):
        v = _f64(v)
        z = np.zeros(self.n)
        st = lib().orc_apply(self.h, _p(v), _p(z), int(trans))
        if st != 0:
            raise RuntimeError(f"oracle apply failed with status {st}")
        return z

    def matvec(self, x, trans=False):
        y = np.zeros(self.n)
        lib().orc_matvec(self.h, _p(_f64(x)), _p(y), int(trans))
        return y

    def solve(self, b, trans=False, restart=50, maxiter=1000, rtol=1e-8, mgs=False):
        x = np.zeros(self.n)
        it, rs = ctypes.c_int(0), ctypes.c_int(0)
        est, tr = ctypes.c_double(0), ctypes.c_double(0)
        st = lib().orc_solve(self.h, int(trans), _p(_f64(b)), _p(x), int(restart), int(maxiter), float(rtol),
                             int(mgs), ctypes.byref(it), ctypes.byref(rs), ctypes.byref(est), ctypes.byref(tr))
        return x, SolveInfo(st, it.value, rs.value, est.value, tr.value)

    def info(self):
        out = np.zeros(512, np.int64)
        k = lib().orc_info(self.h, _p(out), 512)
        out = out[:k].tolist()
        nm, na = out[0], out[1]
        mgr = [tuple(out[2 + 4 * i: 6 + 4 * i]) for i in range(nm)]
        off = 2 + 4 * nm
        amg = [tuple(out[off + 2 * i: off + 2 * i + 2]) for i in range(na)]
        return {"mgr_levels": mgr, "amg_levels": amg}

    def export(self, kind: int, level: int, what: int, sub: int = -1):
        """kind 0 = MGR level, 1 = coarse AMG, 2 = F-relax AMG of MGR level `sub`.
        what 0 = C/F vector, else a CSR (see mgr_oracle.c)."""
        L = lib()
        sizes = np.zeros(3, np.int64)
        st = L.orc_export(self.h, kind, level, what, sub, _p(sizes), None, None, None)
        if st != 0:
            raise KeyError((kind, level, what))
        if what == 0:
            out = np.zeros(int(sizes[0]), np.int32)
            L.orc_export(self.h, kind, level, what, sub, _p(sizes), _p(out), None, None)
            return out
        nr, nc, nnz = (int(s) for s in sizes)
        rp = np.zeros(nr + 1, np.int32)
        ci = np.zeros(max(nnz, 1), np.int32)
        v = np.zeros(max(nnz, 1), np.float64)
        L.orc_export(self.h, kind, level, what, sub, _p(sizes), _p(rp), _p(ci), _p(v))
        return Csr(nr, nc, rp, ci[:nnz], v[:nnz])
