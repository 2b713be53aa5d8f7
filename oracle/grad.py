"""Float64 PyTorch (CPU) form of the Myrtle NNGP recursion, for gradients.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The forward is the same recursion as ``nk_oracle.c`` (seed, 3x3 SAME conv,
ReLU arc-cosine map, 2x2 average pool, global average pool + Dense readout;
App. A, Myrtle listing), written on dense (h, w, h, w) pair tensors with
plain tensor ops so that autograd differentiates it.  The only hand-written
derivative is that of the ReLU map, whose closed-form partials

    dF/ds  = (pi - t) / (2 pi)
    dF/dq  = sin t * sqrt(q'/q) / (4 pi)
    dF/dq' = sin t * sqrt(q/q') / (4 pi),       cos t = s / sqrt(q q'),

stay finite at cos t = 1 (the diagonal of every self recursion), where
differentiating acos and sqrt separately would give 0 * inf.  The variance
maps q are the diagonals of the images' own recursions, so gradients flow
through them into the inputs and both sigmas.
"""
from __future__ import annotations

import math
from typing import Sequence

import numpy as np
import torch

_PI = math.pi


class _ReluMap(torch.autograd.Function):
    @staticmethod
    def forward(ctx, s, q1, q2):
        qq = q1 * q2
        pos = qq > 0
        nrm = torch.sqrt(torch.where(pos, qq, torch.ones_like(qq)))
        rho = torch.clamp(s / nrm, -1.0, 1.0)
        th = torch.acos(rho)
        sin = torch.sqrt(torch.clamp(1.0 - rho * rho, min=0.0))
        a = torch.where(pos, nrm / (2 * _PI) * (sin + (_PI - th) * rho), torch.zeros_like(nrm))
        ctx.save_for_backward(th, sin, q1, q2, pos)
        return a

    @staticmethod
    def backward(ctx, g):
        th, sin, q1, q2, pos = ctx.saved_tensors
        zero = torch.zeros_like(g)
        ds = torch.where(pos, g * (_PI - th) / (2 * _PI), zero)
        safe1 = torch.where(pos, q1.expand_as(g), torch.ones_like(g))
        safe2 = torch.where(pos, q2.expand_as(g), torch.ones_like(g))
        dq1 = torch.where(pos, g * sin * torch.sqrt(safe2 / safe1) / (4 * _PI), zero)
        dq2 = torch.where(pos, g * sin * torch.sqrt(safe1 / safe2) / (4 * _PI), zero)
        return ds, _sum_to(dq1, q1.shape), _sum_to(dq2, q2.shape)


def _sum_to(t: torch.Tensor, shape) -> torch.Tensor:
    dims = [i for i, (a, b) in enumerate(zip(t.shape, shape)) if b == 1 and a != 1]
    if dims:
        t = t.sum(dim=dims, keepdim=True)
    return t


def relu_map(s, q1, q2):
    return _ReluMap.apply(s, q1, q2)


def _conv(a: torch.Tensor, sw2, sb2) -> torch.Tensor:
    """3x3 SAME conv on a batch of (P, h, w, h, w) pair tensors."""
    p, h, w = a.shape[0], a.shape[1], a.shape[2]
    ap = torch.nn.functional.pad(a, (1, 1, 1, 1, 1, 1, 1, 1))
    s = torch.zeros_like(a)
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            s = s + ap[:, 1 + dy:1 + dy + h, 1 + dx:1 + dx + w, 1 + dy:1 + dy + h, 1 + dx:1 + dx + w]
    return sw2 / 9.0 * s + sb2


def _pool(a: torch.Tensor) -> torch.Tensor:
    p, h, w = a.shape[0], a.shape[1], a.shape[2]
    return a.reshape(p, h // 2, 2, w // 2, 2, h // 2, 2, w // 2, 2).mean(dim=(2, 4, 6, 8))


def _diag(s: torch.Tensor) -> torch.Tensor:
    p, h, w = s.shape[0], s.shape[1], s.shape[2]
    return s.reshape(p, h * w, h * w).diagonal(dim1=1, dim2=2).reshape(p, h, w)


def _recursion(x1, x2, depth, sw2, sb2, q1maps=None, q2maps=None):
    """Pair recursion on batches x1, x2 (P, h, w, c).  Self mode if q1maps is None
    (x2 must be x1); then returns (K, qmaps list)."""
    c = x1.shape[-1]
    a = torch.einsum("pyxc,pzwc->pyxzw", x1, x2) / c
    qs = []
    li = 0
    for s, d in enumerate(depth):
        for _ in range(d):
            sig = _conv(a, sw2, sb2)
            if q1maps is None:
                q = _diag(sig)
                qs.append(q)
                qa, qb = q, q
            else:
                qa, qb = q1maps[li], q2maps[li]
            li += 1
            a = relu_map(sig, qa[:, :, :, None, None], qb[:, None, None, :, :])
        if s + 1 < len(depth):
            a = _pool(a)
    k = sw2 * a.mean(dim=(1, 2, 3, 4)) + sb2
    return k, qs


def myrtle_pair_kernel(x1: torch.Tensor, x2: torch.Tensor, depth: Sequence[int], sw2, sb2) -> torch.Tensor:
    """K(x1[p], x2[p]) for a batch of P pairs, differentiable (float64)."""
    _, q1 = _recursion(x1, x1, depth, sw2, sb2)
    _, q2 = _recursion(x2, x2, depth, sw2, sb2)
    k, _ = _recursion(x1, x2, depth, sw2, sb2, q1, q2)
    return k


def myrtle_self_kernel(x: torch.Tensor, depth: Sequence[int], sw2, sb2) -> torch.Tensor:
    k, _ = _recursion(x, x, depth, sw2, sb2)
    return k


def myrtle_vjp(x1: np.ndarray, x2: np.ndarray, pairs: np.ndarray, gk: np.ndarray, depth: Sequence[int],
               sigma_w2: float, sigma_b2: float, chunk: int = 4):
    """Vector-Jacobian product of the kernel entries K(x1[a], x2[b]) at the
    listed (a, b) pairs with cotangents gk.  Returns (dx1, dx2, dsigma[2], K).

    Pairs with a == b and x1 is x2 are self entries (both arguments the same
    image); pass ``x2=None`` for a symmetric block so those entries
    differentiate through both arguments at once.
    """
    torch.set_num_threads(max(1, torch.get_num_threads()))
    sym = x2 is None
    t1 = torch.tensor(np.asarray(x1, dtype=np.float64), requires_grad=True)
    t2 = t1 if sym else torch.tensor(np.asarray(x2, dtype=np.float64), requires_grad=True)
    sw2 = torch.tensor(float(sigma_w2), dtype=torch.float64, requires_grad=True)
    sb2 = torch.tensor(float(sigma_b2), dtype=torch.float64, requires_grad=True)
    pairs = np.asarray(pairs, dtype=np.int64).reshape(-1, 2)
    gk = np.asarray(gk, dtype=np.float64).reshape(-1)
    kout = np.zeros(len(pairs))
    for s in range(0, len(pairs), chunk):
        pa = torch.as_tensor(pairs[s:s + chunk, 0])
        pb = torch.as_tensor(pairs[s:s + chunk, 1])
        k = myrtle_pair_kernel(t1[pa], t2[pb], depth, sw2, sb2)
        kout[s:s + chunk] = k.detach().numpy()
        (k * torch.as_tensor(gk[s:s + chunk])).sum().backward()
    dx1 = t1.grad.numpy().copy() if t1.grad is not None else np.zeros(t1.shape)
    dx2 = None if sym else (t2.grad.numpy().copy() if t2.grad is not None else np.zeros(t2.shape))
    ds = np.array([sw2.grad.item() if sw2.grad is not None else 0.0,
                   sb2.grad.item() if sb2.grad is not None else 0.0])
    return dx1, dx2, ds, kout
