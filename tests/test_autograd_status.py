"""CPU checks of MGRSolve's handling of solver status (no GPU needed): the
library's Solver is replaced by a stand-in that reports a chosen status, so
the autograd function's own logic is what is tested.  An unconverged forward
or adjoint solve must raise, and the backward pass must leave the solver open
so a retained graph can be differentiated twice."""
import pytest
import torch

import paper_2101_11649_amd as P
from paper_2101_11649_amd.autograd import MGRSolve, NotConvergedError


class FakeSolver:
    """Stands in for paper_2101_11649_amd.Solver: X = B / 2, A^T Lambda = G with
    Lambda = G / 2, and the status chosen per direction."""
    instances = []

    def __init__(self, b, rp, ci, vals, field, levels, fwd_status=0, adj_status=0, **kw):
        self.fwd_status, self.adj_status = fwd_status, adj_status
        self.closed = False
        FakeSolver.instances.append(self)

    def solve(self, B, transpose=False):
        st = self.adj_status if transpose else self.fwd_status
        nrhs = 1 if B.dim() == 1 else B.shape[0]
        infos = [P.SolveInfo(st, 7, 0, 1e-3 if st else 1e-9, 1e-3 if st else 1e-9) for _ in range(nrhs)]
        return B / 2, infos

    def grad_values(self, lam, X):
        assert not self.closed, "backward used a closed solver"
        return -(lam * X).sum() * torch.ones(3, dtype=torch.float64)

    def close(self):
        self.closed = True


@pytest.fixture
def fake(monkeypatch):
    FakeSolver.instances.clear()
    monkeypatch.setattr(P, "Solver", FakeSolver)
    return FakeSolver


def _inputs(**opts):
    vals = torch.ones(3, dtype=torch.float64, requires_grad=True)
    B = torch.arange(1.0, 5.0, dtype=torch.float64, requires_grad=True)
    struct = dict(b=1, rp=[0], ci=[], field=[], levels=[], opts=opts)
    return vals, B, struct


def test_unconverged_forward_raises(fake):
    vals, B, struct = _inputs(fwd_status=1)
    with pytest.raises(NotConvergedError, match="forward solve"):
        MGRSolve.apply(vals, B, struct)


def test_unconverged_adjoint_raises(fake):
    vals, B, struct = _inputs(adj_status=1)
    X = MGRSolve.apply(vals, B, struct)
    with pytest.raises(NotConvergedError, match="adjoint solve"):
        X.sum().backward()


def test_backward_keeps_the_solver_open(fake):
    vals, B, struct = _inputs()
    X = MGRSolve.apply(vals, B, struct)
    L = (X * X).sum()
    L.backward(retain_graph=True)
    g1 = B.grad.clone()
    B.grad = None
    L.backward()
    assert torch.equal(B.grad, g1)
    assert not fake.instances[0].closed
