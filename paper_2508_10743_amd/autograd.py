"""torch.autograd.Function wrappers around the DARC kernels.

Each wrapper's forward calls the C ABI and its backward calls the matching
hand-written adjoint kernel, so ``loss.backward()`` on a composition of them
reproduces the gradient Algorithm 1 of the paper obtains by automatic
differentiation (``loss.backward()`` in ``diffeo_pairwise_reg``), without any
autograd graph inside the kernels.

- :class:`ExpSVF`: u = Exp(v) - id by scaling and squaring (§3
  "Diffeomorphisms"); the squaring steps are either kept (checkpoints, one
  field per step) or recomputed in the backward pass (two fields of scratch).
- :class:`Warp3d`: I o phi, gradient with respect to the displacement.
- :class:`Dissimilarity`: MSE or squared local NCC per subject (§3
  "Dissimilarity metrics"), gradient with respect to the warped image.
- :class:`Diffusion`: lam R(u), the diffusion regulariser of Eq. (2).

All tensors are FP32 on the GPU; losses are FP64 per subject.
"""

from __future__ import annotations

import torch

from . import darc as D


class ExpSVF(torch.autograd.Function):
    """u = Exp(v) - id; ``checkpoint=False`` recomputes the squarings in backward."""

    @staticmethod
    def forward(ctx, v: torch.Tensor, n_sq: int = 7, checkpoint: bool = True):
        v = v.contiguous()
        u, ck = D.exp_svf(v, n_sq, checkpoints=checkpoint)
        ctx.n_sq = n_sq
        ctx.has_ck = ck is not None
        ctx.save_for_backward(v, ck if ck is not None else v.new_empty(0))
        return u

    @staticmethod
    def backward(ctx, g_u: torch.Tensor):
        v, ck = ctx.saved_tensors
        g_v = D.exp_svf_bwd(v, ck if ctx.has_ck else None, g_u.contiguous(), ctx.n_sq)
        return g_v, None, None


class Warp3d(torch.autograd.Function):
    """out_i(x) = I_i(x + u_i(x)); differentiable with respect to u only."""

    @staticmethod
    def forward(ctx, img: torch.Tensor, u: torch.Tensor):
        img, u = img.contiguous(), u.contiguous()
        ctx.save_for_backward(img, u)
        return D.warp3d(img, u)

    @staticmethod
    def backward(ctx, g_out: torch.Tensor):
        img, u = ctx.saved_tensors
        if ctx.needs_input_grad[0]:
            raise NotImplementedError("the gradient with respect to the image is not provided")
        return None, D.warp3d_bwd(img, u, g_out.contiguous())


class Dissimilarity(torch.autograd.Function):
    """Per-subject D(warped_i, atlas) (FP64 [n]); differentiable in warped."""

    @staticmethod
    def forward(ctx, warped: torch.Tensor, atlas: torch.Tensor, metric: str = "mse",
                win: int = 9, eps: float = 1e-5):
        loss, g = D.sim_grad(warped.contiguous(), atlas.contiguous(), metric, win, eps, grad=True)
        ctx.save_for_backward(g)
        return loss

    @staticmethod
    def backward(ctx, g_loss: torch.Tensor):
        (g,) = ctx.saved_tensors
        if ctx.needs_input_grad[1]:
            raise NotImplementedError("the gradient with respect to the atlas is not provided")
        scale = g_loss.to(g.dtype).view(-1, *([1] * (g.dim() - 1)))
        return g * scale, None, None, None, None


class Diffusion(torch.autograd.Function):
    """Per-subject lam R(u) (FP64 [n]) of an ncomp-component field."""

    @staticmethod
    def forward(ctx, u: torch.Tensor, lam: float):
        grad, loss = D.diffusion(u.contiguous(), lam)
        ctx.save_for_backward(grad)
        return loss

    @staticmethod
    def backward(ctx, g_loss: torch.Tensor):
        (grad,) = ctx.saved_tensors
        scale = g_loss.to(grad.dtype).view(-1, *([1] * (grad.dim() - 1)))
        return grad * scale, None


def subject_loss(images: torch.Tensor, v: torch.Tensor, atlas: torch.Tensor, metric: str = "mse",
                 lam: float = 0.01, win: int = 9, eps: float = 1e-5, n_sq: int = 7,
                 checkpoint: bool = True) -> torch.Tensor:
    """Per-subject L_i = D(I_i o Exp(v_i), A) + lam R(Exp(v_i) - id) (Algorithm 1,
    ``diffeo_pairwise_reg``), differentiable in v."""
    u = ExpSVF.apply(v, n_sq, checkpoint)
    warped = Warp3d.apply(images, u)
    loss = Dissimilarity.apply(warped, atlas, metric, win, eps)
    if lam != 0.0:
        loss = loss + Diffusion.apply(u, lam)
    return loss
