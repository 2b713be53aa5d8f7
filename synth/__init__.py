"""Seeded synthetic inputs shared by the oracle tests and the HIP path.

This module draws images and labels only; it holds none of the kernel
arithmetic.  The datasets the paper measures on (CIFAR-10/5m at 32x32x3 and
Tiny ImageNet at 64x64x3, paper Sec. 3) are not available here, so these
generators stand in for them with the same shapes and per-channel
standardisation.

Recipes (NumPy PCG64 ``default_rng``):

* ``iid_images``: i.i.d. N(0, 1) pixels.
* ``correlated_images``: each channel an independent 2-D Gaussian process
  with squared-exponential covariance exp(-|p - p'|^2 / (2 l^2)), sampled
  separably as L_y Z L_x^T with L = chol(K_1d + 1e-6 I).
* Both are standardised per channel with the dataset-wide mean and standard
  deviation (computed in float64 over all images and pixels), then cast once
  to float32.  Layout is NHWC.
* ``teacher_labels``: one-hot of argmax_k <W_k, x_flat>, W ~ N(0, 1).
* ``balanced_labels``: class = index mod n_classes, one-hot.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "iid_images",
    "correlated_images",
    "teacher_labels",
    "balanced_labels",
    "uneven_tile_shapes",
    "WORKLOADS",
]


def _standardise(x: np.ndarray) -> np.ndarray:
    x = x.astype(np.float64)
    mean = x.mean(axis=(0, 1, 2), keepdims=True)
    std = x.std(axis=(0, 1, 2), keepdims=True)
    std[std == 0] = 1.0
    return np.ascontiguousarray(((x - mean) / std).astype(np.float32))


def iid_images(n: int, h: int, w: int, c: int, seed: int) -> np.ndarray:
    """n images of h x w x c with i.i.d. N(0,1) pixels, standardised per channel."""
    rng = np.random.default_rng(seed)
    return _standardise(rng.standard_normal((n, h, w, c)))


def _se_chol(m: int, length: float) -> np.ndarray:
    p = np.arange(m, dtype=np.float64)
    k = np.exp(-((p[:, None] - p[None, :]) ** 2) / (2.0 * length * length))
    return np.linalg.cholesky(k + 1e-6 * np.eye(m))


def correlated_images(n: int, h: int, w: int, c: int, length: float, seed: int) -> np.ndarray:
    """n images whose channels are squared-exponential GPs (length in pixels)."""
    rng = np.random.default_rng(seed)
    ly = _se_chol(h, length)
    lx = _se_chol(w, length)
    z = rng.standard_normal((n, c, h, w))
    img = np.einsum("yk,nckl,xl->nyxc", ly, z, lx, optimize=True)
    return _standardise(img)


def teacher_labels(x: np.ndarray, n_classes: int, seed: int) -> np.ndarray:
    """One-hot labels from a random linear teacher on the flattened images."""
    rng = np.random.default_rng(seed)
    flat = x.reshape(x.shape[0], -1).astype(np.float64)
    w = rng.standard_normal((n_classes, flat.shape[1]))
    cls = np.argmax(flat @ w.T, axis=1)
    y = np.zeros((x.shape[0], n_classes), dtype=np.float32)
    y[np.arange(x.shape[0]), cls] = 1.0
    return y


def balanced_labels(n: int, n_classes: int) -> np.ndarray:
    y = np.zeros((n, n_classes), dtype=np.float32)
    y[np.arange(n), np.arange(n) % n_classes] = 1.0
    return y


def uneven_tile_shapes(n_tiles: int, lo: int, hi: int, seed: int) -> np.ndarray:
    """(n_tiles, 2) int64 array of (rows, cols) drawn uniformly from lo..hi."""
    rng = np.random.default_rng(seed)
    return rng.integers(lo, hi + 1, size=(n_tiles, 2)).astype(np.int64)


# Named workloads: the sizes and seeds every test and benchmark uses.
WORKLOADS = {
    # Myrtle-5 on 8x8x3 i.i.d. images, full symmetric 128 x 128 Gram.
    "myrtle5_8x8_gram128": dict(kind="iid", n=128, hw=8, c=3, seed=1001,
                                depth=(2, 1, 1), sigma_w2=2.0, sigma_b2=0.0),
    # FC-3 and Myrtle-5 on 32x32x3 correlated images, 1024 x 1024 block + KRR.
    "fc3_myrtle5_32x32_1024": dict(kind="corr", n1=1024, n2=1024, hw=32, c=3,
                                   length=3.0, seeds=(2001, 2002, 2003),
                                   depth=(2, 1, 1), sigma_w2=2.0, sigma_b2=0.0,
                                   fc_depth=3, fc_sigma_w2=2.0, fc_sigma_b2=0.01,
                                   ridge_rel=1e-4, n_classes=10),
    # Myrtle-10 on 32x32x3 correlated images, one 4096 x 4096 block.
    "myrtle10_32x32_4096": dict(kind="corr", n1=4096, n2=4096, hw=32, c=3,
                                length=3.0, seeds=(3001, 3002),
                                depth=(3, 3, 3), sigma_w2=2.0, sigma_b2=0.0),
    # 64 uneven Myrtle-7 tiles on 32x32x3, plus a 256 x 256 block at 64x64x3.
    "myrtle7_uneven64": dict(kind="corr", pool=2048, hw=32, c=3, length=3.0,
                             seeds=(4001, 4002, 4003), n_tiles=64, lo=32, hi=2048,
                             depth=(2, 2, 2), sigma_w2=2.0, sigma_b2=0.0,
                             big_hw=64, big_n=256, big_length=6.0, big_seeds=(4004, 4005)),
    # CV8 (CNN-VEC, depth 8, flatten readout) on 32x32x3 correlated images.
    "cv8_32x32_4096": dict(kind="corr", n1=4096, n2=4096, hw=32, c=3, length=3.0, seeds=(7001, 7002),
                           depth=8, sigma_w2=2.0, sigma_b2=0.01),
    # Kernel regression by preconditioned CG: a 32768 x 32768 float32 Gram
    # (the FC-3 NNGP of 32x32x3 correlated images) and 10 one-hot targets.
    "fc3_pcg_32768": dict(kind="corr", n=32768, hw=32, c=3, length=3.0, seeds=(6001, 6002),
                          fc_depth=3, fc_sigma_w2=2.0, fc_sigma_b2=0.01, ridge_rel=1e-4,
                          n_classes=10, rank=512, tol=1e-8, max_iter=3000, cpu_n=4096),
    # Approximate solvers on the PCG workload's training images: random
    # subset of 2048 points (Nystrom, SoR), random partition into 16 blocks of
    # 2048 (block-diagonal, committee machine), 2048 test images.
    "fc3_approx_32768": dict(kind="corr", n=32768, m=2048, hw=32, c=3, length=3.0,
                             seeds=(6001, 6002, 6003, 6004, 6005), rank=2048, blocks=16,
                             fc_depth=3, fc_sigma_w2=2.0, fc_sigma_b2=0.01, ridge_rel=1e-4, jitter=1e-6,
                             n_classes=10),
    # Myrtle-5 KRR distillation: 256 support + 2048 targets at 32x32x3.
    "myrtle5_krr_grad": dict(kind="corr", n_support=256, n_target=2048, hw=32, c=3,
                             length=3.0, seeds=(5001, 5002, 5003, 5004),
                             depth=(2, 1, 1), sigma_w2=2.0, sigma_b2=0.0,
                             ridge_rel=1e-4, n_classes=10, fd_h=1e-3),
}
