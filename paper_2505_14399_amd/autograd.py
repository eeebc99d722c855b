"""Differentiation through the multigrid solve.

MGSolveFn(U, b, mg) returns x = D[U]^-1 b computed by the MG-preconditioned solve of the
hierarchy `mg` (built for the same links U).  Its backward, given g = dL/dx (PyTorch's
convention dL/dRe + i dL/dIm), performs one adjoint solve lambda = D^-dagger g with the same
hierarchy (gamma5 D^-1 gamma5) and returns

  dL/db = lambda
  dL/dU_mu(x) = 1/2 c_mu s_mu(x) G^dagger,
  G = tr_spin[(1 - gamma_mu) x(x+mu) lambda(x)^dagger] + tr_spin[(1 + gamma_mu) lambda(x+mu) x(x)^dagger]

(the link gradient is computed by the library's force kernel).  Argument marshalling only.
"""
import torch

from . import link_force, mg_solve


class MGSolveFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, U, b, mg, tol=1e-12):
        x, info = mg_solve(mg, b.contiguous(), tol=tol)
        ctx.mg = mg
        ctx.tol = tol
        ctx.save_for_backward(x)
        ctx.info = info
        return x

    @staticmethod
    def backward(ctx, g):
        (x,) = ctx.saved_tensors
        mg = ctx.mg
        lam, _ = mg_solve(mg, g.contiguous(), tol=ctx.tol, adjoint=True)
        gU = link_force(mg.lat, x, lam) if ctx.needs_input_grad[0] else None
        gb = lam if ctx.needs_input_grad[1] else None
        return gU, gb, None, None


def solve(U, b, mg, tol=1e-12):
    """x = D^-1 b, differentiable with respect to U and b."""
    return MGSolveFn.apply(U, b, mg, tol)
