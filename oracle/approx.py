"""FP64 CPU oracle for the approximate kernel-regression solvers the paper
compares with CG (Sec. 2, "Approximations to the linear system"): the
low-rank Nystrom and subset-of-regressors methods, the block-diagonal
approximation, and the Bayesian committee machine, in the forms of
Rasmussen and Williams, "Gaussian Processes for Machine Learning", ch. 8,
which the paper cites for them.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this module.  It shares no
code with the GPU library.

Notation: n training points, r the subset (inducing points) or partition
size, m test points, c targets; lam the ridge (the noise variance sigma^2 of
the GP reading), jitter the diagonal added to K_rr before it is inverted.
All kernel blocks are passed in (the paper picks the subset and the
partition uniformly at random; that draw is the caller's):

* Nystrom:   Kt = K_nr (K_rr + jitter I)^{-1} K_rn replaces the training
             kernel;  pred = K_mn (Kt + lam I)^{-1} Y.
* SoR:       pred = K_mr (K_rn K_nr + lam (K_rr + jitter I))^{-1} K_rn Y.
* Block-diagonal: K is replaced by blockdiag(K_11, ..., K_pp) over a
             partition;  alpha_i = (K_ii + lam I)^{-1} Y_i,
             pred = sum_i K_mi alpha_i.
* BCM:       per partition the GP posterior of the noise-free test values,
             mu_i = K_mi (K_ii + lam I)^{-1} Y_i,
             S_i = K_mm - K_mi (K_ii + lam I)^{-1} K_im;
             S^{-1} = sum_i S_i^{-1} - (p - 1) K_mm^{-1},
             pred = S sum_i S_i^{-1} mu_i   (transductive: the m test points
             are treated jointly).

The efficient forms below follow these definitions through the Woodbury
identity (Nystrom) or directly (the others); the pins in
tests/test_oracle_approx.py compare them with dense evaluations of the
definitions and with the cases where a method is exact.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def _f64(a):
    return np.asarray(a, dtype=np.float64)


def _chol_solve(a, b):
    return sla.cho_solve(sla.cho_factor(a, lower=True), b)


def nystrom_predict(k_nr, k_rr, k_mn, y, lam: float, jitter: float):
    """Nystrom: the training kernel replaced by K_nr (K_rr + jitter I)^{-1} K_rn.
    Woodbury: (Kt + lam I)^{-1} Y = (Y - K_nr A^{-1} K_rn Y) / lam with
    A = K_rn K_nr + lam (K_rr + jitter I)."""
    k_nr, k_rr, k_mn, y = _f64(k_nr), _f64(k_rr), _f64(k_mn), _f64(y)
    r = k_rr.shape[0]
    a = k_nr.T @ k_nr + lam * (k_rr + jitter * np.eye(r))
    v = _chol_solve(a, k_nr.T @ y)
    alpha = (y - k_nr @ v) / lam
    return k_mn @ alpha


def sor_predict(k_nr, k_rr, k_mr, y, lam: float, jitter: float):
    """Subset of regressors: K_mr (K_rn K_nr + lam (K_rr + jitter I))^{-1} K_rn Y."""
    k_nr, k_rr, k_mr, y = _f64(k_nr), _f64(k_rr), _f64(k_mr), _f64(y)
    r = k_rr.shape[0]
    a = k_nr.T @ k_nr + lam * (k_rr + jitter * np.eye(r))
    return k_mr @ _chol_solve(a, k_nr.T @ y)


def block_diag_predict(blocks, k_m_blocks, y_blocks, lam: float):
    """Block-diagonal approximation: one exact ridge solve per block.

    blocks: list of K_ii (b_i x b_i); k_m_blocks: list of K_mi (m x b_i);
    y_blocks: list of Y_i (b_i x c)."""
    pred = None
    for kii, kmi, yi in zip(blocks, k_m_blocks, y_blocks):
        kii = _f64(kii)
        alpha = _chol_solve(kii + lam * np.eye(len(kii)), _f64(yi))
        term = _f64(kmi) @ alpha
        pred = term if pred is None else pred + term
    return pred


def bcm_predict(blocks, k_m_blocks, y_blocks, k_mm, lam: float, jitter: float = 0.0):
    """Bayesian committee machine posterior mean of the m test points (jointly).

    k_mm: the test-test kernel (prior covariance of the noise-free test
    values); jitter is added to it and to every S_i before they are
    inverted."""
    k_mm = _f64(k_mm)
    m = k_mm.shape[0]
    eye = np.eye(m)
    prec = -(len(blocks) - 1) * _chol_solve(k_mm + jitter * eye, eye)
    rhs = 0.0
    for kii, kmi, yi in zip(blocks, k_m_blocks, y_blocks):
        kii, kmi = _f64(kii), _f64(kmi)
        cf = sla.cho_factor(kii + lam * np.eye(len(kii)), lower=True)
        mu = kmi @ sla.cho_solve(cf, _f64(yi))
        s = k_mm - kmi @ sla.cho_solve(cf, kmi.T)
        sinv = _chol_solve(s + jitter * eye, eye)
        prec = prec + sinv
        rhs = rhs + sinv @ mu
    return _chol_solve(prec, rhs)
