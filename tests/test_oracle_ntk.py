"""Pins of the oracle's Myrtle neural tangent kernel (CPU only).

The paper's large-scale runs use the Myrtle NTK (Sec. "Approaches to
large-scale kernel methods").  The oracle's NTK recursion is checked against
facts that do not come from itself: the ReLU derivative kernel against a
library bivariate-normal probability, an independent joint-matrix
derivation, empirical tangent kernels of finite random networks, the
closed-form diagonal on 1 x 1 images, homogeneity, the sigma_w2 power law,
symmetry and positive semi-definiteness."""
import math

import numpy as np
import pytest
from scipy.stats import multivariate_normal

from tests import mc_nets
import oracle
import synth
from oracle import matrix_form


@pytest.mark.parametrize("rho", [-0.95, -0.4, 0.0, 0.3, 0.8, 0.999, 1.0])
def test_relu_dot_is_orthant_probability(rho):
    # E[relu'(u) relu'(v)] = P(u > 0, v > 0) for unit-variance (u, v) with
    # correlation rho; (-u, -v) has the same covariance, so it is the CDF at 0
    q1, q2 = 1.7, 0.6
    s = rho * math.sqrt(q1 * q2)
    if rho == 1.0:
        p = 0.5  # u = v: P(u > 0)
    else:
        p = multivariate_normal(mean=[0, 0], cov=[[1, rho], [rho, 1]]).cdf([0, 0])
    assert abs(oracle.relu_dot(s, q1, q2) - p) <= 2e-6


@pytest.mark.parametrize("hw,depth,sb2", [(4, (1, 1), 0.0), (4, (2, 1), 0.1), (8, (1, 1, 1), 0.0)])
def test_ntk_matches_joint_matrix_form(hw, depth, sb2):
    x = synth.correlated_images(3, hw, hw, 3, 1.5, 41)
    net = oracle.Myrtle(depth, 2.0, sb2)
    kn, kt = oracle.myrtle_ntk_gram(x, None, net)
    for a in range(3):
        for b in range(3):
            mk, mt = matrix_form.myrtle_pair_ntk(x[a], x[b], depth, 2.0, sb2)
            assert abs(kn[a, b] - mk) <= 1e-12 * abs(mk)
            assert abs(kt[a, b] - mt) <= 1e-12 * abs(mt)


def _ntk_planted(x1, x2, depth, sw2, sb2, bias_in_T=True, readout_tangent=True):
    """The joint-matrix NTK with a mistake planted on request: the bias
    dropped from the pre-activation tangent kernel (T' = box(C) instead of
    box(C) + sigma_b2), or the readout's own tangent (the NNGP term) left out."""
    x1 = np.asarray(x1, dtype=np.float64)
    x2 = np.asarray(x2, dtype=np.float64)
    h, w, c = x1.shape
    X = np.concatenate([x1.reshape(h * w, c), x2.reshape(h * w, c)], axis=0)
    M = X @ X.T / c
    P = np.zeros_like(M)
    for s, d in enumerate(depth):
        T = [matrix_form._blockdiag(matrix_form._shift(h, w, dy, dx)) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]
        for _ in range(d):
            M = sw2 / 9.0 * sum(t @ M @ t.T for t in T) + sb2
            Th = (M if bias_in_T else M - sb2) + sw2 / 9.0 * sum(t @ P @ t.T for t in T)
            q = np.diag(M).copy()
            P = matrix_form._Fdot(M, q[:, None], q[None, :]) * Th
            M = matrix_form._F(M, q[:, None], q[None, :])
        if s + 1 < len(depth):
            Q = matrix_form._blockdiag(matrix_form._avg2(h, w))
            M = Q @ M @ Q.T
            P = Q @ P @ Q.T
            h, w = h // 2, w // 2
    n = h * w
    tangent = float(sw2 * P[:n, n:].mean())
    return tangent + (float(sw2 * M[:n, n:].mean() + sb2) if readout_tangent else 0.0)


@pytest.mark.parametrize("depth,sb2", [((1, 1), 0.0), ((2, 1), 0.5)])
def test_ntk_matches_finite_width_networks(depth, sb2):
    x = synth.correlated_images(3, 4, 4, 3, 1.5, 77)
    net = oracle.Myrtle(depth, 2.0, sb2)
    _, kt = oracle.myrtle_ntk_gram(x, None, net)
    width, seeds = 1024, 24
    ests = np.array([mc_nets.myrtle_empirical_ntk(x, depth, 2.0, sb2, width, s) for s in range(seeds)])
    m = ests.mean(0)
    se = ests.std(0, ddof=1) / math.sqrt(seeds)
    # sampling error (about 0.9 % of each entry here) plus an O(1/width)
    # finite-width bias of at most 5 / width (0.5 %)
    band = 4 * se + 5.0 * np.abs(kt) / width
    assert np.all(np.abs(m - kt) <= band)
    # The band is narrow enough to reject plausible mistakes of the recursion,
    # planted in a copy of the joint-matrix form: without the readout's
    # tangent the kernel drops by 50-85 %, without the bias in T (sb2 > 0) by
    # about 20 %.
    planted = [dict(readout_tangent=False)] + ([dict(bias_in_T=False)] if sb2 > 0 else [])
    for kw in planted:
        kv = np.array([[_ntk_planted(x[a], x[b], depth, 2.0, sb2, **kw) for b in range(3)] for a in range(3)])
        assert np.all(np.abs(m - kv) > band), kw


@pytest.mark.parametrize("depth,sb2,sw2", [((2, 1, 1), 0.0, 2.0), ((1, 2), 0.3, 1.5)])
def test_ntk_diagonal_closed_form_on_1x1_images(depth, sb2, sw2):
    # 1x1 images: every 3x3 conv sees only its centre tap, so along the
    # diagonal (rho = 1: F = q/2, Fdot = 1/2) the recursion is scalar.
    x = synth.iid_images(2, 1, 1, 3, 5)
    # pools need even sizes: one stage per network on 1x1 inputs
    net = oracle.Myrtle((sum(depth),), sw2, sb2)
    kn, kt = oracle.myrtle_ntk_gram(x, None, net)
    for a in range(2):
        q = float(np.dot(x[a, 0, 0].astype(np.float64), x[a, 0, 0].astype(np.float64))) / 3
        S = sw2 / 9 * q + sb2
        T = S
        for _ in range(sum(depth) - 1):
            S, T = sw2 / 9 * S / 2 + sb2, (sw2 / 9 * S / 2 + sb2) + sw2 / 9 * 0.5 * T
        k = sw2 * S / 2 + sb2
        t = k + sw2 * 0.5 * T
        assert abs(kn[a, a] - k) <= 1e-13 * k
        assert abs(kt[a, a] - t) <= 1e-13 * t


def test_ntk_homogeneity_power_law_symmetry_psd():
    x = synth.correlated_images(5, 8, 8, 3, 2.0, 91)
    depth = (2, 1, 1)
    net = oracle.Myrtle(depth, 2.0, 0.0)
    kn, kt = oracle.myrtle_ntk_gram(x, None, net)
    assert np.allclose(kt, kt.T, rtol=0, atol=1e-14 * np.abs(kt).max())
    assert np.linalg.eigvalsh(kt).min() >= -1e-12 * np.trace(kt)
    # homogeneity of degree (1, 1) at sigma_b2 = 0
    _, k2 = oracle.myrtle_ntk_pairs(2.0 * x[:2], 0.5 * x[2:4], np.array([[0, 0], [1, 1]]), net)
    assert np.allclose(k2, [kt[0, 2], kt[1, 3]], rtol=1e-12)
    # every term carries sigma_w2 once per affine layer (4 convs + readout)
    net3 = oracle.Myrtle(depth, 3.0, 0.0)
    _, k3 = oracle.myrtle_ntk_pairs(x, x, np.array([[0, 1], [2, 4]]), net3)
    assert np.allclose(k3, (1.5 ** 5) * np.array([kt[0, 1], kt[2, 4]]), rtol=1e-12)
    # flipping both images horizontally (and transposing both) leaves it unchanged
    _, kf = oracle.myrtle_ntk_pairs(x[:, :, ::-1].copy(), x[:, :, ::-1].copy(), np.array([[0, 3]]), net)
    _, ktr = oracle.myrtle_ntk_pairs(x.transpose(0, 2, 1, 3).copy(), x.transpose(0, 2, 1, 3).copy(),
                                     np.array([[0, 3]]), net)
    assert abs(kf[0] - kt[0, 3]) <= 1e-12 * kt[0, 3] and abs(ktr[0] - kt[0, 3]) <= 1e-12 * kt[0, 3]
