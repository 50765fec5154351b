"""Host logic of the autograd Function: a solve that stops before its
tolerance raises in the forward and in the backward pass (no GPU: the solver
is a stand-in that returns the status the library would)."""
import pytest
import torch

from paper_2112_12397_amd.autograd import (DEFAULT_RTOL, NotConvergedError,
                                           SolveFn)


class _FakeSolver:
    n_u, n_t, n_p = 3, 3, 1

    def __init__(self, fwd_status="FPC_OK", adj_status="FPC_OK"):
        self.fwd_status, self.adj_status = fwd_status, adj_status
        self.rtols = []

    def solve(self, b, rtol=0.0):
        self.rtols.append(rtol)
        return b.clone(), {"status": self.fwd_status, "iterations": 7,
                           "true_rel_residual": 3e-6}

    def solve_T(self, g, rtol=0.0):
        self.rtols.append(rtol)
        return g.clone(), {"status": self.adj_status, "iterations": 9,
                           "true_rel_residual": 2e-6}

    def grad_log_trans(self, pairs, ndir, ups, lam_p, p):
        return torch.zeros(self.n_p, dtype=torch.float64)


def _inputs():
    b = torch.ones(7, dtype=torch.float64, requires_grad=True)
    logu = torch.zeros(1, dtype=torch.float64, requires_grad=True)
    flow = (torch.zeros((0, 2), dtype=torch.int64),
            torch.zeros(1, dtype=torch.int64))
    return b, logu, flow


def test_forward_not_converged_raises():
    b, logu, flow = _inputs()
    with pytest.raises(NotConvergedError, match="forward"):
        SolveFn.apply(b, logu, _FakeSolver(fwd_status="FPC_NOT_CONVERGED"),
                      flow)


def test_backward_not_converged_raises():
    b, logu, flow = _inputs()
    x = SolveFn.apply(b, logu, _FakeSolver(adj_status="FPC_NOT_CONVERGED"),
                      flow)
    with pytest.raises(NotConvergedError, match="adjoint"):
        x.sum().backward()


def test_converged_passes_and_default_rtol():
    b, logu, flow = _inputs()
    s = _FakeSolver()
    x = SolveFn.apply(b, logu, s, flow)
    x.sum().backward()
    assert torch.equal(b.grad, torch.ones(7, dtype=torch.float64))
    assert s.rtols == [DEFAULT_RTOL, DEFAULT_RTOL]
