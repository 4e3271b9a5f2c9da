"""torch.autograd.Function over the library's render and render_backward."""
from __future__ import annotations

import torch


class TranslucentRender(torch.autograd.Function):
    """B = render(sh, theta) on a loaded Renderer; gradients w.r.t. the SH
    lighting and the per-channel (sigma_a, sigma_s', eta) come from the
    library's adjoint kernels."""

    @staticmethod
    def forward(ctx, renderer, sh, theta):
        sh_in = sh.detach().contiguous()
        renderer.set_lighting(sh_in)
        renderer.set_material(theta.detach().contiguous())
        B = renderer.render(save=True)
        ctx.renderer = renderer
        ctx.generation = renderer.generation
        # the adjoint reads the lighting buffer again: saving the inputs makes
        # autograd refuse a backward after they were modified in place
        ctx.save_for_backward(sh, theta)
        return B

    @staticmethod
    def backward(ctx, dB):
        # the library keeps the state of its latest render only: a render or
        # load after this forward would give the gradients of other inputs
        if ctx.renderer.generation != ctx.generation:
            raise RuntimeError("the renderer rendered again after this forward; backward would use "
                               "the state of the later render")
        ctx.saved_tensors  # raises if sh or theta changed in place since forward
        dSH, dTheta = ctx.renderer.render_backward(dB.contiguous())
        return None, dSH, dTheta


def render(renderer, sh, theta):
    return TranslucentRender.apply(renderer, sh, theta)
