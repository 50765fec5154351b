"""``torch.autograd.Function`` around the preconditioned solve.

Forward: ``x = J^{-1} b`` (FGMRES with the block preconditioner).  Backward:
the adjoint ``J^T lam = dL/dx`` (FGMRES with ``M^{-T}``) gives ``dL/db = lam``
and ``dL/d log Upsilon_K = -lam_p^T (dT/d log Upsilon_K) p``, computed by the
library's edge-wise gradient kernel.  The solver must have been set up with
the pressure block T assembled at ``Upsilon = exp(log_upsilon)``.
"""
import torch


class SolveFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, b, log_upsilon, solver, flow, rtol=1e-12):
        x, info = solver.solve(b.detach().contiguous(), rtol=rtol)
        ctx.solver, ctx.flow, ctx.rtol = solver, flow, rtol
        ctx.save_for_backward(x, log_upsilon)
        ctx.info = info
        return x

    @staticmethod
    def backward(ctx, gx):
        x, log_upsilon = ctx.saved_tensors
        s = ctx.solver
        lam, _ = s.solve_T(gx.detach().contiguous(), rtol=ctx.rtol)
        off = s.n_u + s.n_t
        pairs, ndir = ctx.flow
        grad_u = s.grad_log_trans(pairs, ndir, torch.exp(log_upsilon),
                                  lam[off:].contiguous(), x[off:].contiguous())
        return lam, grad_u, None, None, None
