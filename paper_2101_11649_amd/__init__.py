"""Python binding of libmgrhip.so: MGR-preconditioned FGMRES on MI355X (gfx950).

Argument marshalling only: every numeric step runs in the library's HIP
kernels.  PyTorch supplies device memory (tensor data pointers) and the HIP
stream (``torch.cuda.current_stream()``).  If the library is not built, or no
GPU is present, the calls raise; there is no CPU fallback.

Method: Bui et al., "Multigrid reduction preconditioning framework for coupled
processes in porous and fractured media" (arXiv 2101.11649), Sec. 2
(Algorithm 1, eqs. (3)-(5)) and Sec. 4.1 (right-preconditioned GMRES, AMG
coarse solve).  The C-ABI is documented in include/mgr.h.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmgrhip.so")

FRELAX = {"jacobi": 0, "block_jacobi": 1, "ilu0": 2, "amg": 3}
RESTRICT = {"injection": 0, "jacobi": 1}
STATUS = {0: "OK", 1: "NOT_CONVERGED", -1: "ERR_ARG", -2: "ERR_HIP", -3: "ERR_ZERO_PIVOT", -4: "ERR_OOM",
          -5: "ERR_BAD_LABELS", -6: "ERR_UNSUPPORTED"}

EXPORTED = ["mgr_default_opts", "mgr_create", "mgr_set_opts", "mgr_setup", "mgr_apply", "mgr_apply_transpose",
            "mgr_matvec", "mgr_solve", "mgr_solve_transpose", "mgr_grad_values", "mgr_hierarchy_info",
            "mgr_export", "mgr_last_error", "mgr_destroy", "mgr_update_values", "mgr_apply_noalloc"]


class MgrError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


INTERP = {"direct": 0, "ext+i": 1}
SMOOTHER = {"l1-jacobi": 0, "hybrid-gs": 1}


class mgr_matrix(ctypes.Structure):
    _fields_ = [("block_size", ctypes.c_int32), ("n_block_rows", ctypes.c_int32), ("row_ptr", ctypes.c_void_p),
                ("col_idx", ctypes.c_void_p), ("values", ctypes.c_void_p)]


class mgr_level_opts(ctypes.Structure):
    _fields_ = [("f_field_mask", ctypes.c_uint32), ("frelax", ctypes.c_int32), ("sweeps", ctypes.c_int32),
                ("omega", ctypes.c_double), ("restrict_type", ctypes.c_int32),
                ("amg_unknown_based", ctypes.c_int32), ("amg_agg_levels", ctypes.c_int32)]


class mgr_amg_opts(ctypes.Structure):
    _fields_ = [("theta", ctypes.c_double), ("max_levels", ctypes.c_int32), ("max_coarse", ctypes.c_int32),
                ("nu_pre", ctypes.c_int32), ("nu_post", ctypes.c_int32), ("unknown_based", ctypes.c_int32),
                ("interp", ctypes.c_int32), ("smoother", ctypes.c_int32), ("gs_chunk", ctypes.c_int32),
                ("agg_levels", ctypes.c_int32), ("seed", ctypes.c_uint64)]


class mgr_opts(ctypes.Structure):
    _fields_ = [("apply_precision", ctypes.c_int32), ("restart", ctypes.c_int32), ("maxiter", ctypes.c_int32),
                ("rtol", ctypes.c_double), ("ortho", ctypes.c_int32), ("amg", mgr_amg_opts)]


class mgr_solve_info(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iterations", ctypes.c_int32), ("restarts", ctypes.c_int32),
                ("rel_res_est", ctypes.c_double), ("rel_res_true", ctypes.c_double)]


# Device memory provider passed to mgr_create: torch's caching allocator, so
# the solver's arrays come from (and go back to) the same pool as the caller's
# tensors.  The callbacks run while the library holds the call; they take the
# GIL themselves (ctypes) and must not raise across the ABI.
_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)


def _torch_alloc(nbytes, stream, ctx):
    try:
        import torch
        return torch.cuda.caching_allocator_alloc(int(nbytes), stream=int(stream or 0))
    except Exception:
        return None


def _torch_free(ptr, stream, ctx):
    try:
        import torch
        torch.cuda.caching_allocator_delete(int(ptr))
    except Exception:
        pass


TORCH_ALLOC = _ALLOC_FN(_torch_alloc)
TORCH_FREE = _FREE_FN(_torch_free)

_lib = None


def lib():
    """Load libmgrhip.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2101_11649_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        P, i32 = ctypes.c_void_p, ctypes.c_int32
        L.mgr_default_opts.argtypes = [ctypes.POINTER(mgr_opts)]
        L.mgr_default_opts.restype = None
        L.mgr_create.argtypes = [ctypes.POINTER(P), ctypes.POINTER(mgr_opts), P, _ALLOC_FN, _FREE_FN, P]
        L.mgr_set_opts.argtypes = [P, ctypes.POINTER(mgr_opts)]
        L.mgr_setup.argtypes = [P, ctypes.POINTER(mgr_matrix), P, i32, ctypes.POINTER(mgr_level_opts), P]
        L.mgr_update_values.argtypes = [P, P, i32]
        L.mgr_apply.argtypes = [P, P, P]
        L.mgr_apply_transpose.argtypes = [P, P, P]
        L.mgr_apply_noalloc.argtypes = [P, P, P]
        L.mgr_matvec.argtypes = [P, i32, P, P]
        L.mgr_solve.argtypes = [P, i32, P, P, ctypes.POINTER(mgr_solve_info)]
        L.mgr_solve_transpose.argtypes = [P, i32, P, P, ctypes.POINTER(mgr_solve_info)]
        L.mgr_grad_values.argtypes = [P, i32, P, P, P]
        L.mgr_hierarchy_info.argtypes = [P, P, i32]
        L.mgr_export.argtypes = [P, i32, i32, i32, i32, P, P, P, P]
        L.mgr_last_error.argtypes = [P]
        L.mgr_last_error.restype = ctypes.c_char_p
        L.mgr_destroy.argtypes = [P]
        L.mgr_destroy.restype = None
        _lib = L
    return _lib


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("paper_2101_11649_amd needs a ROCm GPU (torch.cuda.is_available() is False)")
    return torch


def _dev(t, dtype):
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        t = torch.as_tensor(np.asarray(t))
    return t.to(device="cuda", dtype=dtype).contiguous()


@dataclass
class SolveInfo:
    status: int
    iterations: int
    restarts: int
    rel_res_est: float
    rel_res_true: float


def level_opts(fmask, frelax="jacobi", sweeps=1, omega=1.0, restrict="injection", amg_unknown_based=False,
               amg_agg_levels=0):
    return dict(fmask=int(fmask), frelax=frelax, sweeps=int(sweeps), omega=float(omega), restrict=restrict,
                amg_unknown_based=int(amg_unknown_based), amg_agg_levels=int(amg_agg_levels))


class Solver:
    """MGR hierarchy + FGMRES on the current GPU.

    ``b``: block size (1 = CSR); ``rp``, ``ci``, ``vals``: block-CSR arrays (any
    array-like or device tensor; copied by the library); ``field``: field label
    of every scalar unknown; ``levels``: list of dicts (fmask, frelax, sweeps,
    omega, restrict, amg_unknown_based: 0 scalar AMG, 1 the unknown approach,
    2 the unknown approach on the separate-component approximation) -- one per
    MGR level; ``interp``: AMG
    interpolation, "direct" or "ext+i" (extended+i, distance two);
    ``smoother``: "l1-jacobi" or "hybrid-gs" (hybrid L1 Gauss-Seidel over chunks
    of ``chunk`` rows); ``block``: block-Jacobi group of every unknown;
    ``allocator``: "torch" (device memory from torch's caching allocator) or
    None (the library's own stream-ordered allocations); ``agg_levels``: the
    coarse AMG's levels with aggressive coarsening (a level's
    "amg_agg_levels" for its F-relaxation AMG).
    """

    def __init__(self, b, rp, ci, vals, field, levels, precision=64, restart=50, maxiter=1000, rtol=1e-8,
                 theta=0.25, max_levels=25, max_coarse=128, nu_pre=1, nu_post=1, unknown_based=False, seed=12345,
                 interp="direct", block=None, allocator="torch", smoother="l1-jacobi", chunk=32, agg_levels=0):
        torch = _torch()
        L = lib()
        self._h = ctypes.c_void_p()
        self.opts = mgr_opts()
        L.mgr_default_opts(ctypes.byref(self.opts))
        self._fill_opts(precision=precision, restart=restart, maxiter=maxiter, rtol=rtol, theta=theta,
                        max_levels=max_levels, max_coarse=max_coarse, nu_pre=nu_pre, nu_post=nu_post,
                        unknown_based=unknown_based, seed=seed, interp=interp, smoother=smoother, chunk=chunk,
                        agg_levels=agg_levels)
        self.stream = torch.cuda.current_stream()
        if allocator == "torch":
            fa, ff = TORCH_ALLOC, TORCH_FREE
        elif allocator is None:
            fa, ff = _ALLOC_FN(), _FREE_FN()        # NULL: the library's own stream-ordered allocations
        else:
            raise ValueError("allocator must be 'torch' or None")
        self._check(L.mgr_create(ctypes.byref(self._h), ctypes.byref(self.opts),
                                 ctypes.c_void_p(self.stream.cuda_stream), fa, ff, None))
        self.b = int(b)
        self.rp = _dev(rp, torch.int32)
        self.ci = _dev(ci, torch.int32)
        self.nbr = self.rp.numel() - 1
        self.n = self.nbr * self.b
        self.nnzb = int(self.rp[-1].item())
        self.levels = list(levels)
        self.field = _dev(field, torch.int32)
        self.block = None if block is None else _dev(block, torch.int32)
        self.setup(vals)

    def _fill_opts(self, precision=None, restart=None, maxiter=None, rtol=None, theta=None, max_levels=None,
                   max_coarse=None, nu_pre=None, nu_post=None, unknown_based=None, seed=None, interp=None,
                   smoother=None, chunk=None, agg_levels=None):
        o = self.opts
        if precision is not None: o.apply_precision = int(precision)
        if restart is not None: o.restart = int(restart)
        if maxiter is not None: o.maxiter = int(maxiter)
        if rtol is not None: o.rtol = float(rtol)
        if theta is not None: o.amg.theta = float(theta)
        if max_levels is not None: o.amg.max_levels = int(max_levels)
        if max_coarse is not None: o.amg.max_coarse = int(max_coarse)
        if nu_pre is not None: o.amg.nu_pre = int(nu_pre)
        if nu_post is not None: o.amg.nu_post = int(nu_post)
        if unknown_based is not None: o.amg.unknown_based = int(bool(unknown_based))
        if seed is not None: o.amg.seed = int(seed)
        if interp is not None: o.amg.interp = INTERP[interp]
        if smoother is not None: o.amg.smoother = SMOOTHER[smoother]
        if chunk is not None: o.amg.gs_chunk = int(chunk)
        if agg_levels is not None: o.amg.agg_levels = int(agg_levels)

    def _check(self, code):
        if code < 0:
            msg = lib().mgr_last_error(self._h).decode() if self._h else ""
            raise MgrError(code, msg)
        return code

    def setup(self, vals):
        """(Re)build the hierarchy for new values on the same pattern."""
        torch = _torch()
        self.vals = _dev(vals, torch.float64)
        A = mgr_matrix(self.b, self.nbr, self.rp.data_ptr(), self.ci.data_ptr(), self.vals.data_ptr())
        arr = (mgr_level_opts * max(1, len(self.levels)))()
        for i, lv in enumerate(self.levels):
            arr[i] = mgr_level_opts(int(lv["fmask"]), FRELAX[lv.get("frelax", "jacobi")], int(lv.get("sweeps", 1)),
                                    float(lv.get("omega", 1.0)), RESTRICT[lv.get("restrict", "injection")],
                                    int(lv.get("amg_unknown_based", 0)),
                                    int(lv.get("amg_agg_levels", 0)))
        self._check(lib().mgr_setup(self._h, ctypes.byref(A), ctypes.c_void_p(self.field.data_ptr()),
                                    len(self.levels), arr,
                                    None if self.block is None else ctypes.c_void_p(self.block.data_ptr())))

    def update_values(self, vals, keep_frelax_amg=False):
        """Setup reuse for new values on the same pattern (mgr_update_values):
        AMG C/F splits and interpolation are kept, or, with keep_frelax_amg,
        the F-relaxation AMG hierarchies whole."""
        torch = _torch()
        self.vals = _dev(vals, torch.float64)
        self._check(lib().mgr_update_values(self._h, ctypes.c_void_p(self.vals.data_ptr()),
                                            1 if keep_frelax_amg else 0))

    def set_opts(self, **kw):
        self._fill_opts(**kw)
        self._check(lib().mgr_set_opts(self._h, ctypes.byref(self.opts)))

    def apply(self, r, transpose=False, out=None):
        torch = _torch()
        r = _dev(r, torch.float64)
        z = out if out is not None else torch.empty_like(r)
        f = lib().mgr_apply_transpose if transpose else lib().mgr_apply
        self._check(f(self._h, ctypes.c_void_p(r.data_ptr()), ctypes.c_void_p(z.data_ptr())))
        return z

    def apply_noalloc(self, r, out):
        """z = M^{-1} r through mgr_apply_noalloc: work vectors in the library's
        static scratch array, nothing allocated (needs one apply or solve on
        this setup first).  out: a float64 device tensor of n entries."""
        torch = _torch()
        r = _dev(r, torch.float64)
        self._check(lib().mgr_apply_noalloc(self._h, ctypes.c_void_p(r.data_ptr()), ctypes.c_void_p(out.data_ptr())))
        return out

    def matvec(self, x, transpose=False):
        torch = _torch()
        x = _dev(x, torch.float64)
        y = torch.empty_like(x)
        self._check(lib().mgr_matvec(self._h, int(transpose), ctypes.c_void_p(x.data_ptr()),
                                     ctypes.c_void_p(y.data_ptr())))
        return y

    def solve(self, B, transpose=False):
        """Solve A X = B (or A^T X = B).  B: (n,) or (nrhs, n).  Returns (X, [SolveInfo])."""
        torch = _torch()
        B = _dev(B, torch.float64)
        nrhs = 1 if B.dim() == 1 else B.shape[0]
        X = torch.empty_like(B)
        infos = (mgr_solve_info * nrhs)()
        f = lib().mgr_solve_transpose if transpose else lib().mgr_solve
        self._check(f(self._h, nrhs, ctypes.c_void_p(B.data_ptr()), ctypes.c_void_p(X.data_ptr()), infos))
        return X, [SolveInfo(i.status, i.iterations, i.restarts, i.rel_res_est, i.rel_res_true) for i in infos]

    def grad_values(self, lam, X):
        """-sum_k lam_k[row] X_k[col] on the block pattern (same layout as vals)."""
        torch = _torch()
        lam = _dev(lam, torch.float64)
        X = _dev(X, torch.float64)
        nrhs = 1 if X.dim() == 1 else X.shape[0]
        dv = torch.empty(self.nnzb * self.b * self.b, dtype=torch.float64, device="cuda")
        self._check(lib().mgr_grad_values(self._h, nrhs, ctypes.c_void_p(lam.data_ptr()),
                                          ctypes.c_void_p(X.data_ptr()), ctypes.c_void_p(dv.data_ptr())))
        return dv

    def info(self):
        out = np.zeros(512, np.int64)
        k = self._check(lib().mgr_hierarchy_info(self._h, out.ctypes.data_as(ctypes.c_void_p), 512))
        out = out[:k].tolist()
        nm, na = out[0], out[1]
        mgr = [tuple(out[2 + 4 * i: 6 + 4 * i]) for i in range(nm)]
        off = 2 + 4 * nm
        amg = [tuple(out[off + 2 * i: off + 2 * i + 2]) for i in range(na)]
        return {"mgr_levels": mgr, "amg_levels": amg}

    def export(self, kind, level, what, sub=-1):
        """kind 0 = MGR level, 1 = coarse AMG, 2 = F-relaxation AMG of MGR level `sub`.
        what 0 = C/F vector (numpy int32); otherwise (nr, nc, rp, ci, v) numpy arrays."""
        L = lib()
        sizes = np.zeros(3, np.int64)
        P = lambda a: a.ctypes.data_as(ctypes.c_void_p)
        self._check(L.mgr_export(self._h, kind, level, what, sub, P(sizes), None, None, None))
        if what == 0:
            out = np.zeros(int(sizes[0]), np.int32)
            self._check(L.mgr_export(self._h, kind, level, what, sub, P(sizes), P(out), None, None))
            return out
        nr, nc, nnz = (int(s) for s in sizes)
        rp = np.zeros(nr + 1, np.int32)
        ci = np.zeros(max(nnz, 1), np.int32)
        v = np.zeros(max(nnz, 1), np.float64)
        self._check(L.mgr_export(self._h, kind, level, what, sub, P(sizes), P(rp), P(ci), P(v)))
        return nr, nc, rp, ci[:nnz], v[:nnz]

    def export_sizes(self, kind, level, what, sub=-1):
        """(rows, cols, nnz) of an exported item (mgr_export with no buffers), or
        None when the hierarchy has no such item (MGR_ERR_ARG)."""
        sizes = np.zeros(3, np.int64)
        rc = lib().mgr_export(self._h, kind, level, what, sub, sizes.ctypes.data_as(ctypes.c_void_p), None, None,
                              None)
        if rc == -1:
            return None
        self._check(rc)
        return tuple(int(x) for x in sizes)

    def coarsest_inverse(self):
        """Dense inverse of the coarse AMG's coarsest level, an (n, n) numpy array."""
        L = lib()
        last = len(self.info()["amg_levels"]) - 1
        sizes = np.zeros(3, np.int64)
        P = lambda a: a.ctypes.data_as(ctypes.c_void_p)
        self._check(L.mgr_export(self._h, 1, last, 3, -1, P(sizes), None, None, None))
        n = int(sizes[0])
        out = np.zeros(max(n * n, 1), np.float64)
        self._check(L.mgr_export(self._h, 1, last, 3, -1, P(sizes), None, None, P(out)))
        return out[: n * n].reshape(n, n)

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().mgr_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def solver_for(system, **kw):
    """Solver for a generated system dict (keys b, rp, ci, vals, field, levels)."""
    return Solver(system["b"], system["rp"], system["ci"], system["vals"], system["field"], system["levels"], **kw)


from .autograd import MGRSolve, NotConvergedError  # noqa: E402  (needs the names above)
