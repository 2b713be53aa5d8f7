"""Pins of the FP64 oracle against facts that do not come from the oracle:
quadrature, closed forms, an independent matrix derivation, exact
invariances of the network, and Monte-Carlo finite-width networks.

All CPU (not marked gpu)."""
import math

import numpy as np
import pytest
import scipy.integrate as si
import scipy.stats as ss

import oracle
import synth
from oracle import matrix_form
from tests import mc_nets


# --------------------------------------------------------------------------
# ReLU arc-cosine map: E[relu(u) relu(v)] for a bivariate normal
# --------------------------------------------------------------------------

def _relu_expectation_quad(s, q1, q2):
    """Integrate E[relu(u) relu(v)] numerically: u = sqrt(q1) z1,
    v = a z1 + b z2; the inner expectation over z2 is the mean of a rectified
    normal, E[relu(m + b z)] = m Phi(m/b) + b phi(m/b)."""
    su = math.sqrt(q1)
    a = s / su
    b = math.sqrt(max(q2 - a * a, 0.0))

    def inner(z1):
        m = a * z1
        if b == 0.0:
            rv = max(m, 0.0)
        else:
            rv = m * ss.norm.cdf(m / b) + b * ss.norm.pdf(m / b)
        return su * z1 * rv * ss.norm.pdf(z1)

    val, _ = si.quad(inner, 0.0, np.inf, epsabs=1e-15, epsrel=1e-13, limit=200)
    return val


def _relu_expectation_dblquad(s, q1, q2):
    cov = np.array([[q1, s], [s, q2]])
    inv = np.linalg.inv(cov)
    det = np.linalg.det(cov)

    def f(v, u):
        z = np.array([u, v])
        return u * v * math.exp(-0.5 * z @ inv @ z) / (2 * math.pi * math.sqrt(det))

    lim = 12 * math.sqrt(max(q1, q2))
    val, _ = si.dblquad(f, 0, lim, 0, lim, epsabs=1e-13, epsrel=1e-11)
    return val


@pytest.mark.parametrize("s,q1,q2", [(0.3, 1.0, 2.0), (-0.7, 1.5, 0.8), (0.999999, 1.0, 1.0), (0.0, 2.0, 3.0),
                                     (1.2, 0.9, 1.7), (-1.3, 1.1, 1.6)])
def test_relu_map_matches_quadrature(s, q1, q2):
    ref = _relu_expectation_quad(s, q1, q2)
    assert abs(oracle.relu_map(s, q1, q2) - ref) <= 1e-12 * max(1.0, abs(ref))


@pytest.mark.parametrize("s,q1,q2", [(0.4, 1.0, 1.3), (-0.5, 1.2, 0.9)])
def test_relu_map_matches_2d_quadrature(s, q1, q2):
    ref = _relu_expectation_dblquad(s, q1, q2)
    assert abs(oracle.relu_map(s, q1, q2) - ref) <= 1e-9


def test_relu_map_special_values():
    # perfectly correlated: E[relu(u)^2] = q/2
    for q in (0.5, 1.0, 7.0):
        assert abs(oracle.relu_map(q, q, q) - q / 2) < 1e-15 * q
    # independent: E[relu(u)] E[relu(v)] = sqrt(q1 q2) / (2 pi)
    assert abs(oracle.relu_map(0.0, 2.0, 8.0) - 4.0 / (2 * math.pi)) < 1e-15
    # anti-correlated: relu(u) relu(-u) = 0
    assert abs(oracle.relu_map(-3.0, 3.0, 3.0)) < 1e-15
    # zero variance: the feature is identically zero
    assert oracle.relu_map(0.0, 0.0, 1.0) == 0.0


def test_relu_map_near_one_series():
    """J1(rho) - rho = (2 sqrt 2 / (3 pi)) t^{3/2} + O(t^{5/2}), t = 1 - rho."""
    for t in (1e-4, 1e-3):
        rho = 1 - t
        j1 = 2 * oracle.relu_map(rho, 1.0, 1.0)
        lead = 2 * math.sqrt(2) / (3 * math.pi) * t ** 1.5
        assert abs((j1 - rho) - lead) < 0.1 * lead * t * 10


# --------------------------------------------------------------------------
# FC NNGP
# --------------------------------------------------------------------------

def test_fc_diagonal_closed_form():
    """With sw2 = 2, each ReLU layer maps K(x,x) to K(x,x) + sb2, so after
    three hidden layers K(x,x) = 2 |x|^2 / d + 4 sb2."""
    x = synth.iid_images(5, 4, 4, 3, 7).reshape(5, -1)
    sb2 = 0.01
    K = oracle.fc_nngp(x, x, depth=3, sigma_w2=2.0, sigma_b2=sb2)
    d = x.shape[1]
    ref = 2.0 * (x.astype(np.float64) ** 2).sum(1) / d + 4 * sb2
    assert np.max(np.abs(np.diag(K) - ref)) < 1e-13


def test_fc_matches_finite_width_networks():
    x = synth.correlated_images(4, 8, 8, 3, 3.0, 11)
    K = oracle.fc_nngp(x, x, depth=3, sigma_w2=2.0, sigma_b2=0.01)
    ks = np.array([mc_nets.fc_empirical(x, 3, 2.0, 0.01, 4096, s) for s in range(24)])
    m = ks.mean(0)
    se = ks.std(0, ddof=1) / math.sqrt(len(ks))
    # 4 standard errors of sampling plus an O(depth/width) finite-width bias allowance
    assert np.all(np.abs(m - K) <= 4 * se + 3.0 / 4096 * np.abs(K))


# --------------------------------------------------------------------------
# Myrtle NNGP
# --------------------------------------------------------------------------

@pytest.mark.parametrize("hw,depth,sb2", [(8, (2, 1, 1), 0.0), (4, (1, 1, 1), 0.05), (8, (1, 2), 0.1),
                                          (6, (2, 1), 0.0)])
def test_myrtle_matches_matrix_form(hw, depth, sb2):
    x = synth.iid_images(3, hw, hw, 3, 21)
    net = oracle.Myrtle(depth, 2.0, sb2)
    K = oracle.myrtle_gram(x, None, net)
    for a in range(3):
        for b in range(3):
            ref = matrix_form.myrtle_pair(x[a], x[b], depth, 2.0, sb2)
            assert abs(K[a, b] - ref) <= 1e-12 * abs(ref)


@pytest.mark.parametrize("depth,sb2", [(1, 0.0), (3, 0.05), (2, 0.01)])
def test_conv_reduces_to_fc_on_1x1_inputs(depth, sb2):
    """On 1x1xC images a [3x3 SAME conv, ReLU] stack sees only its centre tap
    (the eight others fall in the zero padding while the fan-in 9 C stays),
    and the global pool over one pixel is the identity: the network is an FC
    network with hidden weight variance sigma_w2 / 9 and readout variance
    sigma_w2.  Composed here from the scalar ReLU map (itself pinned by
    quadrature): K_1 = sw2/9 x.x'/C + sb2, K_{l+1} = sw2/9 F(K_l) + sb2,
    K = sw2 F(K_D) + sb2."""
    x = synth.iid_images(4, 1, 1, 5, 31)
    net = oracle.Myrtle((depth,), 2.0, sb2)
    K = oracle.myrtle_gram(x, None, net)
    xf = x.reshape(4, -1).astype(np.float64)
    c, sw2 = xf.shape[1], 2.0

    def fc(a, b):
        s = sw2 / 9 * (xf[a] @ xf[b]) / c + sb2
        qa = sw2 / 9 * (xf[a] @ xf[a]) / c + sb2
        qb = sw2 / 9 * (xf[b] @ xf[b]) / c + sb2
        for layer in range(depth):
            f, fa, fb = oracle.relu_map(s, qa, qb), oracle.relu_map(qa, qa, qa), oracle.relu_map(qb, qb, qb)
            scale = sw2 / 9 if layer + 1 < depth else sw2
            s, qa, qb = scale * f + sb2, scale * fa + sb2, scale * fb + sb2
        return s

    ref = np.array([[fc(a, b) for b in range(4)] for a in range(4)])
    assert np.max(np.abs(K - ref) / np.abs(ref)) <= 1e-13


def test_myrtle_nonsquare_matches_matrix_form():
    x = synth.iid_images(2, 4, 8, 2, 22)
    net = oracle.Myrtle((1, 1), 1.5, 0.02)
    K = oracle.myrtle_gram(x, None, net)
    ref = matrix_form.myrtle_pair(x[0], x[1], (1, 1), 1.5, 0.02)
    assert abs(K[0, 1] - ref) <= 1e-12 * abs(ref)


def test_myrtle_invariances():
    x = synth.correlated_images(4, 8, 8, 3, 3.0, 31)
    net = oracle.Myrtle((2, 1, 1), 2.0, 0.0)
    K = oracle.myrtle_gram(x, None, net)
    # symmetry K(x, x') = K(x', x): compute an ordered block and its transpose
    Kab = oracle.myrtle_gram(x[:2], x[2:], net)
    Kba = oracle.myrtle_gram(x[2:], x[:2], net)
    assert np.max(np.abs(Kab - Kba.T)) <= 1e-14 * np.abs(Kab).max()
    # horizontal flip and transpose of both images leave the kernel unchanged
    Kf = oracle.myrtle_gram(x[:, :, ::-1, :].copy(), None, net)
    Kt = oracle.myrtle_gram(x.transpose(0, 2, 1, 3).copy(), None, net)
    assert np.max(np.abs(Kf - K)) <= 1e-14 * np.abs(K).max()
    assert np.max(np.abs(Kt - K)) <= 1e-14 * np.abs(K).max()
    # positivity, Cauchy-Schwarz, PSD
    assert np.all(K > 0)
    d = np.sqrt(np.diag(K))
    assert np.all(np.abs(K) <= np.outer(d, d) * (1 + 1e-14))
    assert np.linalg.eigvalsh(K).min() >= -1e-12 * np.trace(K)


def test_myrtle_homogeneity_and_sigma_power_law():
    """With sb2 = 0 every layer is positively homogeneous: K(a x, b x') =
    a b K(x, x'), and K scales as sw2^(#conv + readout)."""
    x = synth.correlated_images(2, 8, 8, 3, 3.0, 41)
    depth = (2, 1, 1)
    net = oracle.Myrtle(depth, 2.0, 0.0)
    k = oracle.myrtle_pairs(x, x, np.array([[0, 1]]), net)[0]
    ks = oracle.myrtle_pairs(x * np.float32(0.5), x * np.float32(4.0), np.array([[0, 1]]), net)[0]
    assert abs(ks - 2.0 * k) <= 1e-13 * k
    net3 = oracle.Myrtle(depth, 3.0, 0.0)
    k3 = oracle.myrtle_pairs(x, x, np.array([[0, 1]]), net3)[0]
    n_aff = sum(depth) + 1
    assert abs(k3 - k * (3.0 / 2.0) ** n_aff) <= 1e-13 * k3


def test_myrtle_gram_psd_larger():
    x = synth.iid_images(24, 8, 8, 3, 51)
    K = oracle.myrtle_gram(x, None, oracle.Myrtle((2, 1, 1), 2.0, 0.0))
    assert np.linalg.eigvalsh(K).min() >= -1e-12 * np.trace(K)


def test_repeated_pooling_equals_global_pool():
    """An extra 2x2 pool down to 1x1 (a stage with no layers) before the
    global average pool changes nothing."""
    x = synth.iid_images(3, 8, 8, 3, 61)
    a = oracle.myrtle_gram(x, None, oracle.Myrtle((2, 1, 1), 2.0, 0.0))
    b = oracle.myrtle_gram(x, None, oracle.Myrtle((2, 1, 1, 0), 2.0, 0.0))
    assert np.max(np.abs(a - b)) <= 1e-14 * np.abs(a).max()


def test_myrtle_self_pairs_equal_self_recursion():
    x = synth.iid_images(3, 8, 8, 3, 71)
    net = oracle.Myrtle((2, 1, 1), 2.0, 0.01)
    _, kself = oracle.myrtle_self(x, net)
    kp = oracle.myrtle_pairs(x, x, np.array([[0, 0], [1, 1], [2, 2]]), net)
    assert np.max(np.abs(kself - kp)) <= 1e-14 * kself.max()


@pytest.mark.slow
def test_myrtle_matches_finite_width_conv_nets():
    """Monte-Carlo width-4096 conv-ReLU networks on 8x8x3 inputs."""
    x = synth.iid_images(3, 8, 8, 3, 1001)
    depth = (2, 1, 1)
    K = oracle.myrtle_gram(x, None, oracle.Myrtle(depth, 2.0, 0.0))
    ks = np.array([mc_nets.myrtle_empirical(x, depth, 2.0, 0.0, 4096, s) for s in range(6)])
    m = ks.mean(0)
    se = ks.std(0, ddof=1) / math.sqrt(len(ks))
    assert np.all(np.abs(m - K) <= 4 * se + 5.0 / 4096 * np.abs(K))
    # and the estimate is tight enough to reject a 10 % scale error
    assert np.all(4 * se + 5.0 / 4096 * np.abs(K) < 0.1 * np.abs(K))


def test_myrtle_matches_finite_width_conv_nets_bias():
    """Same pin with a bias (sb2 > 0) on 4x4 inputs, lighter widths."""
    x = synth.iid_images(3, 4, 4, 3, 1002)
    depth = (1, 1, 1)
    K = oracle.myrtle_gram(x, None, oracle.Myrtle(depth, 2.0, 0.1))
    ks = np.array([mc_nets.myrtle_empirical(x, depth, 2.0, 0.1, 2048, s) for s in range(16)])
    m = ks.mean(0)
    se = ks.std(0, ddof=1) / math.sqrt(len(ks))
    assert np.all(np.abs(m - K) <= 4 * se + 4.0 / 2048 * np.abs(K))


# --------------------------------------------------------------------------
# Kernel ridge regression
# --------------------------------------------------------------------------

def test_krr_matches_dense_solve():
    rng = np.random.default_rng(3)
    a = rng.standard_normal((40, 60))
    K = a @ a.T / 60
    Kt = rng.standard_normal((7, 40))
    y = rng.standard_normal((40, 3))
    lam = 1e-3 * np.mean(np.diag(K))
    ref = Kt @ np.linalg.solve(K + lam * np.eye(40), y)
    got = oracle.krr_predict(K, Kt, y, 1e-3)
    assert np.max(np.abs(got - ref)) <= 1e-10 * np.abs(ref).max()


def test_krr_interpolates_training_set_at_tiny_ridge():
    rng = np.random.default_rng(4)
    a = rng.standard_normal((20, 50))
    K = a @ a.T / 50 + np.eye(20)
    y = rng.standard_normal((20, 2))
    got = oracle.krr_predict(K, K, y, 1e-12)
    assert np.max(np.abs(got - y)) < 1e-9


def test_krr_mse_cotangents_match_finite_differences():
    rng = np.random.default_rng(12)
    n, m, c = 9, 6, 3
    a = rng.standard_normal((n, n + 3))
    kss = a @ a.T / (n + 3)
    kts = rng.standard_normal((m, n))
    ys = rng.standard_normal((n, c))
    yt = rng.standard_normal((m, c))
    lam = 0.05
    dss, dts = oracle.krr_mse_cotangents(kss, kts, ys, yt, lam)
    h = 1e-6
    # K_ss is symmetric: perturb (i, j) and (j, i) together; the directional
    # derivative is dss[i, j] + dss[j, i] (dss[i, i] on the diagonal)
    for (i, j) in [(0, 0), (2, 5), (8, 1)]:
        e = np.zeros_like(kss)
        e[i, j] = e[j, i] = 1.0
        fd = (oracle.krr_mse_loss(kss + h * e, kts, ys, yt, lam) - oracle.krr_mse_loss(kss - h * e, kts, ys, yt, lam)) / (2 * h)
        ref = dss[i, j] + (dss[j, i] if i != j else 0.0)
        assert abs(fd - ref) <= 1e-7 * max(1.0, abs(dss).max())
    for (i, j) in [(0, 0), (5, 8), (3, 4)]:
        kp = kts.copy(); kp[i, j] += h
        km = kts.copy(); km[i, j] -= h
        fd = (oracle.krr_mse_loss(kss, kp, ys, yt, lam) - oracle.krr_mse_loss(kss, km, ys, yt, lam)) / (2 * h)
        assert abs(fd - dts[i, j]) <= 1e-7 * max(1.0, abs(dts).max())
