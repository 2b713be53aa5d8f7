"""torch.autograd.Function over the libnk Myrtle NNGP: the forward calls
nk_myrtle_nngp, the backward nk_myrtle_nngp_backward (which recomputes the
covariances from the saved inputs; nothing else is saved).

x2=None, or x2 passed as the very same tensor as x1, is the symmetric block
K(x1, x1): one adjoint call gives the whole gradient, returned at x1 (autograd
adds the gradients of a tensor passed twice, so nothing is returned for the
second use).  Any other x2 gets its own gradient."""
from __future__ import annotations

from typing import Sequence

import torch

from . import ops


class MyrtleNNGP(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x1, x2, sigma_w2, sigma_b2, depth: Sequence[int]):
        sw2 = float(sigma_w2)
        sb2 = float(sigma_b2)
        sym = x2 is None or x2 is x1
        K = ops.myrtle_nngp(x1.contiguous(), None if sym else x2.contiguous(), depth, sw2, sb2)
        ctx.save_for_backward(x1, x1 if sym else x2)
        ctx.sym = sym
        ctx.depth = tuple(depth)
        ctx.sw2, ctx.sb2 = sw2, sb2
        ctx.sig_like = tuple((v.dtype, v.device) if isinstance(v, torch.Tensor) else None for v in (sigma_w2, sigma_b2))
        return K.clone()

    @staticmethod
    def backward(ctx, gK):
        x1, x2 = ctx.saved_tensors
        dx1, dx2, ds = ops.myrtle_nngp_backward(x1.contiguous(), None if ctx.sym else x2.contiguous(),
                                                gK.contiguous().float(), ctx.depth, ctx.sw2, ctx.sb2,
                                                need_dx2=ctx.sym or ctx.needs_input_grad[1])
        gw, gb = (None if like is None else ds[i].to(dtype=like[0], device=like[1])
                  for i, like in enumerate(ctx.sig_like))
        return dx1, None if ctx.sym else dx2, gw, gb, None


def myrtle_nngp(x1, x2, sigma_w2, sigma_b2, depth):
    """Differentiable Myrtle NNGP block (x2=None: symmetric block of x1)."""
    return MyrtleNNGP.apply(x1, x2, sigma_w2, sigma_b2, depth)
