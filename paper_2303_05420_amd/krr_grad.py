"""Gradient of a kernel-ridge-regression loss through the Myrtle NNGP with
respect to learnable support images and both sigmas (the differentiable
use of the kernel: support images regress onto target images).

    loss = mean((K_ts alpha - Y_t)^2),   alpha = (K_ss + lambda I)^{-1} Y_s,
    lambda = ridge_rel * mean(diag K_ss) fixed at the evaluation point.

Every step runs in libnk: the two Gram blocks (nk_myrtle_nngp), the float64
ridge solve and its cotangents (nk_krr_mse_backward) and the kernel adjoint
(nk_myrtle_nngp_backward); this module only sequences the calls."""
from __future__ import annotations

from typing import Sequence

import torch

from . import ops


def krr_mse_loss_and_grad(x_s: torch.Tensor, y_s: torch.Tensor, x_t: torch.Tensor, y_t: torch.Tensor,
                          depth: Sequence[int], sigma_w2: float, sigma_b2: float, ridge_rel: float = 1e-4,
                          lam: float | None = None):
    """Returns (loss, d loss / d x_s, d loss / d[sigma_w2, sigma_b2], lambda)."""
    k_ss = ops.myrtle_nngp(x_s, None, depth, sigma_w2, sigma_b2).clone()
    k_ts = ops.myrtle_nngp(x_t, x_s, depth, sigma_w2, sigma_b2).clone()
    if lam is None:
        dss, dts, loss, lam = ops.krr_mse_backward(k_ss, k_ts, y_s, y_t, ridge_rel, relative=True)
    else:
        dss, dts, loss, lam = ops.krr_mse_backward(k_ss, k_ts, y_s, y_t, lam)
    dxs1, _, ds1 = ops.myrtle_nngp_backward(x_s, None, dss, depth, sigma_w2, sigma_b2)
    dxs1 = dxs1.clone()
    ds1 = ds1.clone()
    _, dxs2, ds2 = ops.myrtle_nngp_backward(x_t, x_s, dts, depth, sigma_w2, sigma_b2)
    return loss, dxs1 + dxs2, ds1 + ds2, lam
