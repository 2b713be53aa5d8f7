"""Gradient of a kernel-ridge-regression loss through the Myrtle NNGP with
respect to learnable support images and both sigmas (the differentiable
use of the kernel: support images regress onto target images).

    loss = mean((K_ts alpha - Y_t)^2),   alpha = (K_ss + lambda I)^{-1} Y_s,
    lambda = ridge_rel * mean(diag K_ss) fixed at the evaluation point.

The whole step is one library call, nk_krr_mse_grad: the two Gram blocks,
the float64 ridge solve and its cotangents, the kernel adjoint of both
blocks and the sum of their contributions to the support images."""
from __future__ import annotations

from typing import Sequence

import torch

from . import ops


def krr_mse_loss_and_grad(x_s: torch.Tensor, y_s: torch.Tensor, x_t: torch.Tensor, y_t: torch.Tensor,
                          depth: Sequence[int], sigma_w2: float, sigma_b2: float, ridge_rel: float = 1e-4,
                          lam: float | None = None, keep_checkpoints: bool = False):
    """Returns (loss, d loss / d x_s, d loss / d[sigma_w2, sigma_b2], lambda).
    keep_checkpoints: keep every pair's first-stage output between the forward
    and the adjoint pass instead of recomputing it (ops.krr_mse_grad)."""
    if lam is None:
        return ops.krr_mse_grad(x_s, y_s, x_t, y_t, depth, sigma_w2, sigma_b2, ridge_rel, relative=True,
                                keep_checkpoints=keep_checkpoints)
    return ops.krr_mse_grad(x_s, y_s, x_t, y_t, depth, sigma_w2, sigma_b2, lam, relative=False,
                            keep_checkpoints=keep_checkpoints)
