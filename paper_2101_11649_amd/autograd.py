"""torch.autograd.Function around solve(A, b) with an adjoint backward.

Forward: X = A^{-1} B by MGR-preconditioned FGMRES (optionally with the FP32
MGR apply).  Backward, for an upstream gradient G = dL/dX: Lambda = A^{-T} G by
FGMRES on A^T right-preconditioned with the exact transpose M^{-T} of the MGR
cycle; then dL/dB = Lambda and dL/dA_ij = -sum_k Lambda_k[i] X_k[j] on A's
sparsity pattern (the adjoint of a linear solve).  Both steps run in the HIP
library; this module only passes tensors through.

A solve that stops at maxiter before reaching rtol (status MGR_NOT_CONVERGED)
raises NotConvergedError in the forward and in the backward pass: an
unconverged X or Lambda would give a wrong gradient without any sign of it.
The solver handle lives as long as the autograd context, so a graph kept with
retain_graph=True can be differentiated more than once.
"""
from __future__ import annotations

import torch


class NotConvergedError(RuntimeError):
    """FGMRES stopped before the relative residual reached rtol."""


def _require_converged(infos, what):
    bad = [(k, i) for k, i in enumerate(infos) if i.status != 0]
    if bad:
        k, i = bad[0]
        raise NotConvergedError(
            f"MGRSolve {what}: {len(bad)} of {len(infos)} right-hand sides did not converge "
            f"(first: column {k}, status {i.status}, {i.iterations} iterations, "
            f"true relative residual {i.rel_res_true:.3e}); raise maxiter or loosen rtol")


class MGRSolve(torch.autograd.Function):
    """X = MGRSolve.apply(values, B, structure) with structure a dict of
    b, rp, ci, field, levels and solver keyword options (precision, rtol, ...).
    values: (nnzb*b*b,) float64 CUDA tensor; B: (n,) or (nrhs, n)."""

    @staticmethod
    def forward(ctx, values, B, structure):
        from . import Solver
        opts = dict(structure.get("opts", {}))
        solver = Solver(structure["b"], structure["rp"], structure["ci"], values.detach(), structure["field"],
                        structure["levels"], **opts)
        X, infos = solver.solve(B.detach())
        _require_converged(infos, "forward solve")
        # the handle is closed when the context (and with it the solver) is freed
        ctx.solver = solver
        ctx.infos = infos
        ctx.save_for_backward(X)
        return X

    @staticmethod
    def backward(ctx, G):
        (X,) = ctx.saved_tensors
        solver = ctx.solver
        lam, infos_t = solver.solve(G.contiguous(), transpose=True)
        _require_converged(infos_t, "adjoint solve")
        ctx.infos_adjoint = infos_t
        grad_values = solver.grad_values(lam, X)
        return grad_values, lam, None
