"""torch.autograd.Function over render_fwd / render_bwd.

The backward is the library's hand-written adjoint (App. A.1 blend and projection): it walks
each tile's list in reverse recovering the transmittance from T_final, so nothing per pixel
beyond (T_final, n_contrib) is kept between forward and backward.  The context given to the
function must not run another render_fwd before the backward (checked).
"""
from __future__ import annotations

import torch

from .api import Context, GaussianBuffers


class RasterizeFunction(torch.autograd.Function):
    @staticmethod
    def forward(fctx, mean, quat, log_scale, logit, sh, dass_ctx: Context, cams, bg, sh_degree: int):
        n = int(mean.shape[1])
        g = GaussianBuffers(mean.detach().contiguous(), quat.detach().contiguous(), log_scale.detach().contiguous(),
                            logit.detach().contiguous(), sh.detach().contiguous(), n, n, sh_degree)
        outs = dass_ctx.render_fwd(g, cams, bg)
        fctx.dass = dass_ctx
        fctx.g = g
        fctx.outs = outs
        fctx.cams = cams
        fctx.bg = bg
        fctx.generation = dass_ctx.generation
        return tuple(o.rgb for o in outs)

    @staticmethod
    def backward(fctx, *grad_rgb):
        dass_ctx = fctx.dass
        if dass_ctx.generation != fctx.generation:
            raise RuntimeError("another render_fwd ran on this context between forward and backward")
        g = fctx.g
        dls = [(gr if gr is not None else torch.zeros_like(o.rgb)).contiguous() for gr, o in zip(grad_rgb, fctx.outs)]
        grads = g.zeros_like()
        dass_ctx.render_bwd(g, fctx.cams, fctx.bg, fctx.outs, dls, grads)
        return grads.mean, grads.quat, grads.log_scale, grads.logit, grads.sh, None, None, None, None


def rasterize(mean, quat, log_scale, logit, sh, dass_ctx: Context, cams, bg=(0.0, 0.0, 0.0), sh_degree: int = 0):
    """Differentiable render of every camera; returns one (3, H, W) image per camera.

    Parameters are (P, n) structure-of-arrays tensors on the GPU: mean (3, n), quat (4, n),
    log_scale (3, n), logit (n,), sh (3 (deg+1)^2, n)."""
    return RasterizeFunction.apply(mean, quat, log_scale, logit, sh, dass_ctx, list(cams), tuple(bg), sh_degree)
