"""torch.autograd wrapper of the pressure solve with a hand-written adjoint.

Forward: p_b = A(rho)^+ P f_b for a batch of right-hand sides (multigrid in the HIP
library, face products built from rho on the device).  Backward for a loss L(p):
  * dL/df_b = mu_b, the solution of A mu_b = P dL/dp_b: a second multigrid solve with
    the same hierarchy, because A is symmetric;
  * dL/drho_c = -1/2 sum over the faces f of c of beta_f^2 g_f with
    g_f = h^-2 sum_b (mu_b,R - mu_b,L)(p_b,R - p_b,L), from one fused kernel.
The paper (section 3.1) solves but never differentiates; the adjoint follows from
differentiating A p = P f with the face products of section 3.1.
"""
from __future__ import annotations

import torch

from .solver import MG

# right-hand sides of a batch solved at once by default (the context's own stream plus
# three lanes)
DEFAULT_CONCURRENCY = 4


class PoissonSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, f, rho, mask, tol=1e-10, precision="fp64", max_cycles=100, krylov=False, lanes=None):
        if precision not in ("fp64", "mixed"):
            raise ValueError("precision must be 'fp64' or 'mixed'")
        if lanes is None:   # a batch runs up to DEFAULT_CONCURRENCY right-hand sides at once
            lanes = min(f.shape[0], DEFAULT_CONCURRENCY) - 1 if f.dim() == 4 else 0
        mg = MG.from_rho(rho.detach().contiguous(), mask.contiguous(), mixed=(precision == "mixed"), krylov=krylov,
                         lanes=lanes)
        p, _, stats = mg.solve(f.detach().contiguous(), tol=tol, max_cycles=max_cycles)
        ctx.mg = mg
        ctx.tol = tol
        ctx.max_cycles = max_cycles
        ctx.stats = stats
        ctx.save_for_backward(p)
        return p

    @staticmethod
    def backward(ctx, grad_p):
        (p,) = ctx.saved_tensors
        mg = ctx.mg
        mu, _, _ = mg.solve(grad_p.contiguous(), tol=ctx.tol, max_cycles=ctx.max_cycles)
        grad_f = mu if ctx.needs_input_grad[0] else None
        grad_rho = mg.coeff_grad(mu, p) if ctx.needs_input_grad[1] else None
        return grad_f, grad_rho, None, None, None, None, None, None


def poisson_solve(f, rho, mask, tol=1e-10, precision="fp64", max_cycles=100, krylov=False, lanes=None):
    """p with A(rho) p = P f; differentiable in f and rho.  lanes: extra streams for the
    right-hand sides of a batch (None: up to DEFAULT_CONCURRENCY at once; 0: one by one);
    the results do not depend on it."""
    return PoissonSolve.apply(f, rho, mask, tol, precision, max_cycles, krylov, lanes)
