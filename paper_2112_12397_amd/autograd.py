"""``torch.autograd.Function`` around the preconditioned solve.

Forward: ``x = J^{-1} b`` (FGMRES with the block preconditioner).  Backward:
the adjoint ``J^T lam = dL/dx`` (FGMRES with ``M^{-T}``) gives ``dL/db = lam``
and ``dL/d log Upsilon_K = -lam_p^T (dT/d log Upsilon_K) p``, computed by the
library's edge-wise gradient kernel.  The solver must have been set up with
the pressure block T assembled at ``Upsilon = exp(log_upsilon)``.

A solve that stops before its tolerance (FPC_NOT_CONVERGED) raises in either
pass: gradients formed from an unconverged ``x`` or ``lam`` would be silently
wrong.
"""
import torch

DEFAULT_RTOL = 1e-10


class NotConvergedError(RuntimeError):
    """The forward or adjoint solve did not reach its tolerance."""


def _require_converged(info, what):
    if info.get("status") != "FPC_OK":
        raise NotConvergedError(
            f"{what} stopped at true relative residual "
            f"{info.get('true_rel_residual', float('nan')):.3e} after "
            f"{info.get('iterations')} iterations ({info.get('status')})")


class SolveFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, b, log_upsilon, solver, flow, rtol=DEFAULT_RTOL):
        x, info = solver.solve(b.detach().contiguous(), rtol=rtol)
        _require_converged(info, "forward solve J x = b")
        ctx.solver, ctx.flow, ctx.rtol = solver, flow, rtol
        ctx.save_for_backward(x, log_upsilon)
        ctx.info = info
        return x

    @staticmethod
    def backward(ctx, gx):
        x, log_upsilon = ctx.saved_tensors
        s = ctx.solver
        lam, info = s.solve_T(gx.detach().contiguous(), rtol=ctx.rtol)
        _require_converged(info, "adjoint solve J^T lam = dL/dx")
        off = s.n_u + s.n_t
        pairs, ndir = ctx.flow
        grad_u = s.grad_log_trans(pairs, ndir, torch.exp(log_upsilon),
                                  lam[off:].contiguous(), x[off:].contiguous())
        return lam, grad_u, None, None, None
