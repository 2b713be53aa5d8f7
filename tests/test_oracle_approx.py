"""Pins of the approximate-solver oracle (oracle/approx.py): each efficient
form against a dense evaluation of its definition, the cases where a method
is exact (the subset is the whole training set, a single block, a single
partition), and the committee machine's exactness when the partitions are
conditionally independent given the test values."""
import numpy as np
import scipy.linalg as sla

import oracle
import synth
from oracle import approx


def _data(n_train, n_test, seed, hw=8):
    x = synth.correlated_images(n_train + n_test, hw, hw, 3, 3.0, seed).reshape(n_train + n_test, -1)
    k = oracle.fc_nngp(x, x)
    y = synth.teacher_labels(x[:n_train].reshape(n_train, hw, hw, 3), 10, seed + 1).astype(np.float64)
    return k[:n_train, :n_train], k[n_train:, :n_train], k[n_train:, n_train:], y


def _krr(ktr, kte, y, lam):
    return kte @ sla.cho_solve(sla.cho_factor(ktr + lam * np.eye(len(ktr)), lower=True), y)


def test_nystrom_equals_its_dense_definition():
    ktr, kte, _, y = _data(150, 20, 11)
    rng = np.random.default_rng(12)
    sub = rng.choice(150, 30, replace=False)
    lam, jit = 1e-2, 1e-6
    got = approx.nystrom_predict(ktr[:, sub], ktr[np.ix_(sub, sub)], kte, y, lam, jit)
    kt = ktr[:, sub] @ np.linalg.solve(ktr[np.ix_(sub, sub)] + jit * np.eye(30), ktr[sub, :])
    ref = kte @ np.linalg.solve(kt + lam * np.eye(150), y)
    assert np.max(np.abs(got - ref)) <= 1e-8 * np.max(np.abs(ref))


def test_sor_equals_the_degenerate_gp_definition():
    ktr, kte, _, y = _data(150, 20, 13)
    rng = np.random.default_rng(14)
    sub = rng.choice(150, 25, replace=False)
    lam, jit = 1e-2, 1e-6
    krr_inv = np.linalg.inv(ktr[np.ix_(sub, sub)] + jit * np.eye(25))
    got = approx.sor_predict(ktr[:, sub], ktr[np.ix_(sub, sub)], kte[:, sub], y, lam, jit)
    kt = ktr[:, sub] @ krr_inv @ ktr[sub, :]
    kt_m = kte[:, sub] @ krr_inv @ ktr[sub, :]
    ref = kt_m @ np.linalg.solve(kt + lam * np.eye(150), y)
    assert np.max(np.abs(got - ref)) <= 1e-7 * np.max(np.abs(ref))


def test_full_subset_is_exact_krr():
    ktr, kte, _, y = _data(80, 15, 15)
    lam = 1e-2
    ref = _krr(ktr, kte, y, lam)
    ny = approx.nystrom_predict(ktr, ktr, kte, y, lam, 0.0)
    so = approx.sor_predict(ktr, ktr, kte, y, lam, 0.0)
    assert np.max(np.abs(ny - ref)) <= 1e-7 * np.max(np.abs(ref))
    assert np.max(np.abs(so - ref)) <= 1e-6 * np.max(np.abs(ref))


def test_block_diagonal_limits():
    ktr, kte, _, y = _data(60, 10, 16)
    lam = 1e-2
    one = approx.block_diag_predict([ktr], [kte], [y], lam)
    assert np.allclose(one, _krr(ktr, kte, y, lam), rtol=1e-10, atol=1e-12)
    singles = approx.block_diag_predict([ktr[i:i + 1, i:i + 1] for i in range(60)],
                                        [kte[:, i:i + 1] for i in range(60)], [y[i:i + 1] for i in range(60)], lam)
    ref = kte @ (y / (np.diag(ktr) + lam)[:, None])
    assert np.allclose(singles, ref, rtol=1e-12, atol=1e-14)


def test_bcm_single_partition_is_exact():
    ktr, kte, ktt, y = _data(70, 12, 17)
    lam = 1e-2
    got = approx.bcm_predict([ktr], [kte], [y], ktt, lam)
    assert np.allclose(got, _krr(ktr, kte, y, lam), rtol=1e-7, atol=1e-9)


def test_bcm_exact_for_conditionally_independent_partitions():
    """Every partition observes the test points themselves (with independent
    noise): given the test values the partitions are independent, and the
    committee machine equals the exact posterior mean on all data."""
    _, _, ktt, _ = _data(1, 9, 18)
    m, p, lam = 9, 4, 5e-2
    rng = np.random.default_rng(19)
    ys = [rng.standard_normal((m, 3)) for _ in range(p)]
    got = approx.bcm_predict([ktt] * p, [ktt] * p, ys, ktt, lam, jitter=0.0)
    kfull = np.kron(np.ones((p, p)), ktt)
    kmf = np.kron(np.ones((1, p)), ktt)
    ref = kmf @ np.linalg.solve(kfull + lam * np.eye(p * m), np.concatenate(ys, 0))
    assert np.max(np.abs(got - ref)) <= 1e-7 * np.max(np.abs(ref))


def test_more_subset_points_do_not_move_away_from_exact():
    ktr, kte, _, y = _data(200, 20, 20)
    lam = 1e-3
    ref = _krr(ktr, kte, y, lam)
    rng = np.random.default_rng(21)
    perm = rng.permutation(200)
    errs = [np.linalg.norm(approx.nystrom_predict(ktr[:, perm[:r]], ktr[np.ix_(perm[:r], perm[:r])], kte, y, lam,
                                                  1e-6) - ref) for r in (10, 50, 200)]
    assert errs[2] < errs[1] < errs[0]
