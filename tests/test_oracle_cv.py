"""Pins of the CNN-VEC (CV8) oracle: the displacement-0 loop of nk_oracle.c
against the independent joint-matrix form (flatten readout), Monte-Carlo
finite-width CNN-VEC networks, and invariances of the network."""
import numpy as np

import oracle
import synth
from oracle import matrix_form
from tests import mc_nets


def test_loop_matches_joint_matrix_form():
    for (h, w, depth, sb2, seed) in ((4, 4, 1, 0.0, 1), (4, 4, 3, 0.01, 2), (3, 5, 2, 0.1, 3), (2, 6, 4, 0.01, 4)):
        x = synth.iid_images(3, h, w, 3, seed)
        k = oracle.cv_gram(x, None, depth=depth, sigma_w2=2.0, sigma_b2=sb2)
        m = np.array([[matrix_form.cv_pair(x[a], x[b], depth, 2.0, sb2) for b in range(3)] for a in range(3)])
        assert np.max(np.abs(k - m) / np.abs(m)) < 1e-12, (h, w, depth)


def test_self_kernel_and_symmetry():
    x = synth.correlated_images(5, 8, 8, 3, 3.0, 5)
    k = oracle.cv_gram(x, None, depth=8)
    _, d = oracle.cv_self(x, 8)
    assert np.allclose(np.diag(k), d, rtol=1e-14)
    assert np.allclose(k, k.T, rtol=1e-14)
    assert np.min(np.linalg.eigvalsh(k)) > -1e-12 * np.max(np.abs(k))
    # Cauchy-Schwarz
    assert np.all(k ** 2 <= np.outer(d, d) * (1 + 1e-12))


def test_flip_and_homogeneity():
    x = synth.correlated_images(4, 8, 8, 3, 3.0, 6)
    k = oracle.cv_gram(x, None, depth=5)
    # mirroring both images (rows, then columns) maps the network onto itself
    for ax in (1, 2):
        xf = np.ascontiguousarray(np.flip(x, axis=ax))
        assert np.allclose(oracle.cv_gram(xf, None, depth=5), k, rtol=1e-13)
    # without biases every layer is positively homogeneous: K(c x, x') = c K(x, x')
    k0 = oracle.cv_gram(x[:2], x[2:], depth=5, sigma_b2=0.0)
    k3 = oracle.cv_gram(3.0 * x[:2], x[2:], depth=5, sigma_b2=0.0)
    assert np.allclose(k3, 3.0 * k0, rtol=1e-12)
    # sigma_w2 law without biases: K scales as sigma_w2^(depth + 1)
    k1 = oracle.cv_gram(x[:2], x[2:], depth=5, sigma_w2=1.0, sigma_b2=0.0)
    assert np.allclose(k0, 2.0 ** 6 * k1, rtol=1e-12)


def test_matches_finite_width_networks():
    """Monte-Carlo width-2048 CNN-VEC networks on 6x6x3 inputs, depth 3, with biases."""
    x = synth.correlated_images(4, 6, 6, 3, 2.0, 7)
    depth = 3
    ref = oracle.cv_gram(x, None, depth=depth, sigma_w2=2.0, sigma_b2=0.01)
    ks = np.array([mc_nets.cv_empirical(x, depth, 2.0, 0.01, 2048, s) for s in range(12)])
    mean = ks.mean(0)
    se = ks.std(0, ddof=1) / np.sqrt(len(ks))
    tol = 3 * se + 3.0 / 2048 * np.abs(ref)  # sampling error + O(depth / width) finite-width bias
    assert np.all(np.abs(mean - ref) <= tol)
    # and the estimate is tight enough to reject the same network without its biases
    nobias = oracle.cv_gram(x, None, depth=depth, sigma_w2=2.0, sigma_b2=0.0)
    assert np.any(np.abs(mean - nobias) > tol)
