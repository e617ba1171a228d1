"""Differentiable gridding and degridding (torch.autograd.Function).

Degridding V = D(G) and gridding G = D^H(V) are exact adjoints of each other on
complex tensors (the gridder applies A_p^H . A_q and the forward FFT where the
degridder applies A_p . A_q^H and the inverse FFT, with the same taper and
phasors conjugated).  For a C-linear map y = M x, PyTorch's vector-Jacobian
product with an incoming gradient g is M^H g, so
    DegridFn.backward(gV) = grid(gV)       GridFn.backward(gG) = degrid(gG),
each computed by the other hand-written kernel chain on the current stream.
Visibilities that belong to no subgrid are ignored by gridding and set to zero
by degridding, which keeps the pair adjoint.

The image level pairs the same way: prediction G = P(I) (Eq. wunstack) is the exact
adjoint of imaging I = P^H(G) (Eq. wstack), so
    PredictFn.backward(gG) = invert(gG)    InvertFn.backward(gI) = predict(gI),
and ``predict_vis`` (image -> visibilities, degrid after predict) is differentiable
end to end.

The backward passes call the library's adjoint pair (aidg_grid_adjoint,
aidg_degrid_adjoint), which equals gridding and degridding except on Stokes-I plans:
there gridding reduces to I = (XX + YY) / 2 and degridding expands I to [[I, 0], [0, I]],
and the library applies the adjoints' factors 2 and 1/2 itself.

A plan in the inverse A-term mode grids with normalised A^-1 and divides its image by
the normalisation map: neither is the adjoint of degridding or prediction, so these
functions refuse such plans (the library refuses its adjoint pair for them as well).
"""
from __future__ import annotations

import torch


def _adjoint_plan(plan):
    if getattr(plan.geometry, "aterm_mode", 0) != 0:
        raise ValueError("autograd needs a plan in the adjoint A-term mode (aterm_mode = 0): "
                         "inverse-mode gridding is not the adjoint of degridding")
    return plan


class DegridFn(torch.autograd.Function):
    """V = degrid(G): grid [W, 4, N, N] -> visibilities [nbl, nt, nc, 4]."""

    @staticmethod
    def forward(ctx, grid: torch.Tensor, plan) -> torch.Tensor:
        ctx.plan = _adjoint_plan(plan)
        return plan.degrid(grid.contiguous())

    @staticmethod
    def backward(ctx, g_vis: torch.Tensor):
        plan = ctx.plan
        g_grid = None
        if ctx.needs_input_grad[0]:
            g_grid = plan.grid_adjoint(g_vis.contiguous())
        return g_grid, None


class GridFn(torch.autograd.Function):
    """G = grid(V): visibilities [nbl, nt, nc, 4] -> grid [W, 4, N, N]."""

    @staticmethod
    def forward(ctx, vis: torch.Tensor, plan) -> torch.Tensor:
        ctx.plan = _adjoint_plan(plan)
        return plan.grid(vis.contiguous())

    @staticmethod
    def backward(ctx, g_grid: torch.Tensor):
        plan = ctx.plan
        g_vis = None
        if ctx.needs_input_grad[0]:
            g_vis = plan.degrid_adjoint(g_grid.contiguous())
        return g_vis, None


def degrid(grid: torch.Tensor, plan) -> torch.Tensor:
    return DegridFn.apply(grid, plan)


def grid(vis: torch.Tensor, plan) -> torch.Tensor:
    return GridFn.apply(vis, plan)


class PredictFn(torch.autograd.Function):
    """G = predict(I): image [4, N, N] -> grid layers [W, 4, N, N]."""

    @staticmethod
    def forward(ctx, image: torch.Tensor, plan) -> torch.Tensor:
        ctx.plan = _adjoint_plan(plan)
        return plan.predict(image.contiguous())

    @staticmethod
    def backward(ctx, g_grid: torch.Tensor):
        g_image = None
        if ctx.needs_input_grad[0]:
            g_image = ctx.plan.invert(g_grid.contiguous())
        return g_image, None


class InvertFn(torch.autograd.Function):
    """I = invert(G): grid layers [W, 4, N, N] -> image [4, N, N]."""

    @staticmethod
    def forward(ctx, grid: torch.Tensor, plan) -> torch.Tensor:
        ctx.plan = _adjoint_plan(plan)
        return plan.invert(grid.contiguous())

    @staticmethod
    def backward(ctx, g_image: torch.Tensor):
        g_grid = None
        if ctx.needs_input_grad[0]:
            g_grid = ctx.plan.predict(g_image.contiguous())
        return g_grid, None


def predict(image: torch.Tensor, plan) -> torch.Tensor:
    return PredictFn.apply(image, plan)


def invert(grid: torch.Tensor, plan) -> torch.Tensor:
    return InvertFn.apply(grid, plan)


def predict_vis(image: torch.Tensor, plan) -> torch.Tensor:
    """Visibilities of an image: degridding of its predicted grid layers."""
    return DegridFn.apply(PredictFn.apply(image, plan), plan)
