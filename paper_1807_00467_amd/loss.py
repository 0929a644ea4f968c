"""Differentiable registration loss for learning-based registration.

L(u, T) = D_NGF(R, T(y)) + alpha S(u) + gamma Vhat(u)  (eq. 1, 5, 9; eq. 11 without the
keypoint and lung-boundary terms), with y = x + u trilinear on the 4-voxel node grid.
The forward pass evaluates the objective with the library's kernels; the backward pass
returns the hand-written adjoints: dL/du from the gradient passes (ngf_grad,
curvature_apply, volchange_eval) and dL/dT from ngf_grad_T.  Nothing is recorded on
PyTorch's tape inside: this Function is the whole derivative.
"""
from __future__ import annotations

from typing import Sequence

import torch

from .disco import Disco


class NGFLossFn(torch.autograd.Function):
    """loss = D + alpha S + gamma Vhat for one pair; R is fixed in the context."""

    @staticmethod
    def forward(fctx, u: torch.Tensor, T: torch.Tensor, ctx: Disco, R: torch.Tensor, eta: float, alpha: float,
                gamma: float):
        u = u.detach().contiguous()
        T = T.detach().contiguous()
        ctx.set_images(R, T)
        D = ctx.ngf_eval(u, eta)
        S, _, _ = ctx.curvature_apply(alpha, u, None, energy=True, grad=False, diag=False)
        V = ctx.volchange_eval(gamma, u, None, energy=True, grad=False, diag=False)["V"]
        fctx.disco = ctx
        fctx.consts = (eta, alpha, gamma)
        fctx.save_for_backward(u)
        return (D + S + V)[0]

    @staticmethod
    def backward(fctx, grad_out: torch.Tensor):
        (u,) = fctx.saved_tensors
        ctx: Disco = fctx.disco
        eta, alpha, gamma = fctx.consts
        need_u, need_T = fctx.needs_input_grad[0], fctx.needs_input_grad[1]
        gu = gT = None
        if need_u:
            _, g, _ = ctx.ngf_grad(u, eta, diag=False)
            _, gs, _ = ctx.curvature_apply(alpha, u, None, energy=False, grad=True, diag=False)
            gv = ctx.volchange_eval(gamma, u, None, energy=False, grad=True, diag=False)["g"]
            gu = (g + gs + gv) * grad_out
        if need_T:
            gT = ctx.ngf_grad_T(u, eta) * grad_out
        return gu, gT, None, None, None, None, None


def ngf_loss(ctx: Disco, u: torch.Tensor, T: torch.Tensor, R: torch.Tensor, eta: float = 10.0, alpha: float = 1.0,
             gamma: float = 0.1) -> torch.Tensor:
    """Differentiable loss of one pair (see NGFLossFn)."""
    return NGFLossFn.apply(u, T, ctx, R, eta, alpha, gamma)


class NGFLoss(torch.nn.Module):
    """Sum of the pair losses over a batch of pairs with a shared geometry.

    One library context per pair keeps each pair's gradient volumes resident."""

    def __init__(self, shape: Sequence[int], spacing: Sequence[float], fixed: Sequence[torch.Tensor],
                 eta: float = 10.0, alpha: float = 1.0, gamma: float = 0.1, storage: str = "fp32"):
        super().__init__()
        self.fixed = [R.contiguous() for R in fixed]
        self.ctxs = [Disco(shape, spacing, storage=storage, device=R.device) for R in self.fixed]
        self.eta, self.alpha, self.gamma = eta, alpha, gamma

    def forward(self, u: torch.Tensor, T: torch.Tensor) -> torch.Tensor:
        """u: [B][3][nz][ny][nx], T: [B][Nz][Ny][Nx]."""
        total = u.new_zeros(())
        for b, (ctx, R) in enumerate(zip(self.ctxs, self.fixed)):
            total = total + ngf_loss(ctx, u[b], T[b], R, self.eta, self.alpha, self.gamma)
        return total
