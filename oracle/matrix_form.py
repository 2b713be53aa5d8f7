"""Joint-covariance-matrix form of the Myrtle NNGP for tiny images.

TEST INFRASTRUCTURE ONLY: an independent second derivation used to pin the
loop recursion of ``nk_oracle.c`` on images of at most a few hundred pixels.

Instead of a pair tensor indexed by (pixel of x, pixel of x'), it carries the
full covariance matrix M of the stacked feature vector [f(x); f(x')]
(2 h w entries, channel-averaged) through the network of App. A:

* input:   M = X X^T / C, X the (2hw, C) stacked pixel matrix;
* conv:    M <- (sw2 / 9) sum_d T_d M T_d^T + sb2 (on both diagonal blocks and
           the cross block), T_d = diag(S_d, S_d), (S_d v)(i) = v(i + d) inside
           the image and 0 outside -- the covariance of a weight-shared linear
           map with i.i.d. N(0, sw2 / (9 C_in)) weights;
* ReLU:    M_ab <- F(M_ab, M_aa, M_bb) entry-wise (the arc-cosine map);
* pool:    M <- Q M Q^T with Q = diag(R, R), R the 2x2 averaging matrix;
* readout: K(x, x') = sw2 * mean of the cross block + sb2.

The variance maps are the diagonal of M itself, so no separate self recursion
is needed.
"""
from __future__ import annotations

import math
from typing import Sequence

import numpy as np


def _F(s, q1, q2):
    qq = q1 * q2
    out = np.zeros_like(s)
    pos = qq > 0
    nrm = np.sqrt(np.where(pos, qq, 1.0))
    rho = np.clip(s / nrm, -1.0, 1.0)
    th = np.arccos(rho)
    val = nrm / (2 * math.pi) * (np.sqrt(np.clip(1 - rho * rho, 0, None)) + (math.pi - th) * rho)
    out[pos] = val[pos]
    return out


def _shift(h: int, w: int, dy: int, dx: int) -> np.ndarray:
    s = np.zeros((h * w, h * w))
    for y in range(h):
        for x in range(w):
            yy, xx = y + dy, x + dx
            if 0 <= yy < h and 0 <= xx < w:
                s[y * w + x, yy * w + xx] = 1.0
    return s


def _avg2(h: int, w: int) -> np.ndarray:
    r = np.zeros(((h // 2) * (w // 2), h * w))
    for y in range(h // 2):
        for x in range(w // 2):
            for a in range(2):
                for b in range(2):
                    r[y * (w // 2) + x, (2 * y + a) * w + 2 * x + b] = 0.25
    return r


def _blockdiag(a: np.ndarray) -> np.ndarray:
    z = np.zeros_like(a)
    return np.block([[a, z], [z, a]])


def myrtle_pair(x1: np.ndarray, x2: np.ndarray, depth: Sequence[int], sw2: float, sb2: float) -> float:
    x1 = np.asarray(x1, dtype=np.float64)
    x2 = np.asarray(x2, dtype=np.float64)
    h, w, c = x1.shape
    X = np.concatenate([x1.reshape(h * w, c), x2.reshape(h * w, c)], axis=0)
    M = X @ X.T / c
    for s, d in enumerate(depth):
        T = [_blockdiag(_shift(h, w, dy, dx)) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]
        for _ in range(d):
            M = sw2 / 9.0 * sum(t @ M @ t.T for t in T) + sb2
            q = np.diag(M).copy()
            M = _F(M, q[:, None], q[None, :])
        if s + 1 < len(depth):
            Q = _blockdiag(_avg2(h, w))
            M = Q @ M @ Q.T
            h, w = h // 2, w // 2
    n = h * w
    return float(sw2 * M[:n, n:].mean() + sb2)


def cv_pair(x1: np.ndarray, x2: np.ndarray, depth: int, sw2: float, sb2: float) -> float:
    """CNN-VEC NNGP of one pair in the joint-matrix form: ``depth`` conv/ReLU
    blocks at full resolution, then the Flatten + Dense readout, i.e.
    sw2 times the mean over pixels i of the cross-block entry (i, i), + sb2."""
    x1 = np.asarray(x1, dtype=np.float64)
    x2 = np.asarray(x2, dtype=np.float64)
    h, w, c = x1.shape
    X = np.concatenate([x1.reshape(h * w, c), x2.reshape(h * w, c)], axis=0)
    M = X @ X.T / c
    T = [_blockdiag(_shift(h, w, dy, dx)) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]
    for _ in range(depth):
        M = sw2 / 9.0 * sum(t @ M @ t.T for t in T) + sb2
        q = np.diag(M).copy()
        M = _F(M, q[:, None], q[None, :])
    n = h * w
    return float(sw2 * np.mean(np.diag(M[:n, n:])) + sb2)


def _Fdot(s, q1, q2):
    """E[relu'(u) relu'(v)] = (pi - t) / (2 pi), entry-wise."""
    qq = q1 * q2
    out = np.zeros_like(s)
    pos = qq > 0
    nrm = np.sqrt(np.where(pos, qq, 1.0))
    rho = np.clip(s / nrm, -1.0, 1.0)
    val = (math.pi - np.arccos(rho)) / (2 * math.pi)
    out[pos] = val[pos]
    return out


def myrtle_pair_ntk(x1: np.ndarray, x2: np.ndarray, depth: Sequence[int], sw2: float, sb2: float):
    """(NNGP, NTK) of one pair in the joint-matrix form: beside the covariance
    M of the stacked pre-activations it carries their tangent-kernel matrix
    Th; a conv maps the post-activation tangent matrix P to
    Th = M_new + (sw2 / 9) sum_d T_d P T_d^T, a ReLU sets P = Fdot(M) * Th
    entry-wise, pools act on P like on M, and the readout adds
    sw2 * mean of P's cross block."""
    x1 = np.asarray(x1, dtype=np.float64)
    x2 = np.asarray(x2, dtype=np.float64)
    h, w, c = x1.shape
    X = np.concatenate([x1.reshape(h * w, c), x2.reshape(h * w, c)], axis=0)
    M = X @ X.T / c
    P = np.zeros_like(M)
    for s, d in enumerate(depth):
        T = [_blockdiag(_shift(h, w, dy, dx)) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]
        for _ in range(d):
            M = sw2 / 9.0 * sum(t @ M @ t.T for t in T) + sb2
            Th = M + sw2 / 9.0 * sum(t @ P @ t.T for t in T)
            q = np.diag(M).copy()
            P = _Fdot(M, q[:, None], q[None, :]) * Th
            M = _F(M, q[:, None], q[None, :])
        if s + 1 < len(depth):
            Q = _blockdiag(_avg2(h, w))
            M = Q @ M @ Q.T
            P = Q @ P @ Q.T
            h, w = h // 2, w // 2
    n = h * w
    k = float(sw2 * M[:n, n:].mean() + sb2)
    return k, k + float(sw2 * P[:n, n:].mean())
