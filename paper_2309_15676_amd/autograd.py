"""torch.autograd.Function around the renderer: the forward pass renders, the
backward pass replays the same paths from their random numbers (no tape is
stored; only the parameters, seed, stream and sample count are saved)."""
from __future__ import annotations

import torch

from .problem import Problem


class RenderFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, params: torch.Tensor, problem: Problem, seed: int, iteration: int,
                tag: int, spp: int, flags: int = 0):
        p = params.detach().to(torch.float32).contiguous()
        img = problem.render(p, seed, iteration, tag, spp, flags)
        ctx.save_for_backward(p)
        ctx.problem, ctx.seed, ctx.iteration, ctx.tag, ctx.spp, ctx.flags = (
            problem, seed, iteration, tag, spp, flags)
        return img

    @staticmethod
    def backward(ctx, grad_img: torch.Tensor):
        (p,) = ctx.saved_tensors
        g = ctx.problem.render_bwd(p, grad_img.contiguous(), ctx.seed, ctx.iteration, ctx.tag,
                                   ctx.spp, ctx.flags)
        return g, None, None, None, None, None, None


def render(params: torch.Tensor, problem: Problem, seed: int, iteration: int = 0,
           tag: int = 8, spp: int = 1, flags: int = 0) -> torch.Tensor:
    """Differentiable render (H, W, 3) of `problem` at `params`."""
    return RenderFunction.apply(params, problem, seed, iteration, tag, spp, flags)
