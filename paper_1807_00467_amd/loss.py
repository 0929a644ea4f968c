"""Differentiable registration loss for learning-based registration.

L(u, T) = D_NGF(R, T(y)) + alpha S(u) + gamma Vhat(u)  (eq. 1, 5, 9; eq. 11 without the
keypoint and lung-boundary terms), with y = x + u trilinear on the 4-voxel node grid.
The forward pass evaluates the objective with the library (objective_eval); the backward
pass returns the hand-written adjoints: dL/du from the library's linearisation
(objective_linearise) and dL/dT from ngf_grad_T.  Nothing is recorded on PyTorch's tape
inside: each Function is the whole derivative, and the binding only scales the
library's gradients by the incoming gradient (the chain rule).

A context keeps the gradient volumes of one (R, T) pair.  The forward pass saves R and
T, and the backward pass rebuilds the context's volumes from them when the context has
been given other images in between (several forward passes on one context before one
backward pass, gradient accumulation); autograd's version check rejects a T modified in
place after the forward pass.  ngf_loss is the loss of one pair; NGFLoss sums a batch of
pairs in one Function whose backward pass writes every pair's gradients directly into
the batch gradients.
"""
from __future__ import annotations

from typing import Sequence

import torch

from .disco import Disco, Params


class NGFLossFn(torch.autograd.Function):
    """loss = D + alpha S + gamma Vhat for one pair."""

    @staticmethod
    def forward(fctx, u: torch.Tensor, T: torch.Tensor, ctx: Disco, R: torch.Tensor, eta: float, alpha: float,
                gamma: float):
        u = u.detach().contiguous()
        Td = T.detach()
        Tc = Td.contiguous()
        ctx.use_images(R, Tc)
        params = Params(eta=eta, alpha=alpha, gamma=gamma, delta=0.0, beta=0.0)
        terms = ctx.objective_eval(params, u)
        fctx.disco = ctx
        fctx.params = params
        # Tc is T itself when T is contiguous, so the saved tensor keeps T's version check
        fctx.save_for_backward(u, Tc, R)
        return terms[0].clone()

    @staticmethod
    def backward(fctx, grad_out: torch.Tensor):
        u, T, R = fctx.saved_tensors
        ctx: Disco = fctx.disco
        params: Params = fctx.params
        need_u, need_T = fctx.needs_input_grad[0], fctx.needs_input_grad[1]
        ctx.use_images(R, T)
        gu = gT = None
        if need_u:
            gu = ctx.objective_linearise(params, u, grad=True, diag=False, terms=False)["g"] * grad_out
        if need_T:
            # the upstream gradient scales dL/dT inside the stencil pass
            gT = ctx.ngf_grad_T(u, params.eta, scale=grad_out.detach().to(device=u.device, dtype=torch.float64).reshape(1))
        return gu, gT, None, None, None, None, None


def ngf_loss(ctx: Disco, u: torch.Tensor, T: torch.Tensor, R: torch.Tensor, eta: float = 10.0, alpha: float = 1.0,
             gamma: float = 0.1) -> torch.Tensor:
    """Differentiable loss of one pair (see NGFLossFn)."""
    return NGFLossFn.apply(u, T, ctx, R, eta, alpha, gamma)


class NGFLossBatchFn(torch.autograd.Function):
    """loss = sum over the pairs b of D_b + alpha S_b + gamma Vhat_b, one context per pair.
    The backward pass writes each pair's gradients straight into the batch gradients."""

    @staticmethod
    def forward(fctx, u: torch.Tensor, T: torch.Tensor, ctxs: Sequence[Disco], Rs: Sequence[torch.Tensor],
                eta: float, alpha: float, gamma: float):
        u = u.detach().contiguous()
        # T itself when T is contiguous, so the saved tensor keeps T's version check
        Tc = T.detach().contiguous()
        params = Params(eta=eta, alpha=alpha, gamma=gamma, delta=0.0, beta=0.0)
        terms = torch.empty((len(ctxs), 8), dtype=torch.float64, device=u.device)
        for b, (ctx, R) in enumerate(zip(ctxs, Rs)):
            ctx.use_images(R, Tc[b])
            ctx.objective_eval(params, u[b], terms[b])
        fctx.ctxs = list(ctxs)
        fctx.params = params
        fctx.save_for_backward(u, Tc, *Rs)
        return terms[:, 0].sum()

    @staticmethod
    def backward(fctx, grad_out: torch.Tensor):
        u, T, *Rs = fctx.saved_tensors
        params: Params = fctx.params
        need_u, need_T = fctx.needs_input_grad[0], fctx.needs_input_grad[1]
        gu = torch.empty_like(u) if need_u else None
        gT = torch.empty_like(T) if need_T else None
        scale = grad_out.detach().to(device=u.device, dtype=torch.float64).reshape(1)
        for b, (ctx, R) in enumerate(zip(fctx.ctxs, Rs)):
            ctx.use_images(R, T[b])
            if need_u:
                ctx.objective_linearise(params, u[b], grad=True, diag=False, terms=False, g_out=gu[b])
            if need_T:
                # the upstream gradient scales dL/dT inside the stencil pass
                ctx.ngf_grad_T(u[b], params.eta, out=gT[b], scale=scale)
        if need_u:
            gu.mul_(grad_out)
        return gu, gT, None, None, None, None, None


class NGFLoss(torch.nn.Module):
    """Sum of the pair losses over a batch of pairs with a shared geometry.

    One library context per pair keeps that pair's grad R and grad T resident: a forward
    pass rebuilds a gradient volume only when it is given a different (or modified) image."""

    def __init__(self, shape: Sequence[int], spacing: Sequence[float], fixed: Sequence[torch.Tensor],
                 eta: float = 10.0, alpha: float = 1.0, gamma: float = 0.1, storage: str = "fp32"):
        super().__init__()
        self.fixed = [R.contiguous() for R in fixed]
        self.ctxs = [Disco(shape, spacing, storage=storage, device=R.device) for R in self.fixed]
        self.eta, self.alpha, self.gamma = eta, alpha, gamma

    def close(self):
        """Release the library contexts."""
        for c in self.ctxs:
            c.close()

    def forward(self, u: torch.Tensor, T: torch.Tensor) -> torch.Tensor:
        """u: [B][3][nz][ny][nx], T: [B][Nz][Ny][Nx] (B = the number of fixed images)."""
        if u.shape[0] != len(self.ctxs) or T.shape[0] != len(self.ctxs):
            raise ValueError(f"expected {len(self.ctxs)} pairs, got u {tuple(u.shape)} and T {tuple(T.shape)}")
        return NGFLossBatchFn.apply(u, T, self.ctxs, self.fixed, self.eta, self.alpha, self.gamma)
