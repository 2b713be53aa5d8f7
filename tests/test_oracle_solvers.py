"""Pins of the solver oracle (partial pivoted Cholesky, Woodbury
preconditioner, preconditioned CG) to facts that do not come from the oracle
itself: the uniqueness of the Cholesky factor, exact low-rank recovery, a
brute-force Schur-complement pivot rule, the finite termination of CG on a
matrix with few distinct eigenvalues, the exact solve, and the monotone
A-norm error of CG."""
import numpy as np
import pytest
import scipy.linalg as sla

import oracle
import synth
from oracle import solvers


def _spd(n, seed, floor=1e-3):
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((n, n))
    return g @ g.T / n + floor * np.eye(n)


def test_full_rank_is_the_cholesky_of_the_permuted_matrix():
    k = _spd(40, 1)
    L, piv, d = solvers.pivoted_cholesky(k, 40)
    assert sorted(piv.tolist()) == list(range(40))
    lp = L[piv]
    # the permuted factor is lower triangular with a positive diagonal ...
    assert np.allclose(np.triu(lp, 1), 0.0, atol=1e-12)
    assert np.all(np.diag(lp) > 0)
    # ... so by uniqueness it is the Cholesky factor of the permuted matrix
    ref = np.linalg.cholesky(k[np.ix_(piv, piv)])
    assert np.allclose(lp, ref, rtol=1e-10, atol=1e-12)
    assert np.allclose(L @ L.T, k, atol=1e-12)
    assert np.allclose(d, 0.0, atol=1e-12)


def test_exact_low_rank_is_recovered_and_stops():
    rng = np.random.default_rng(2)
    g = rng.standard_normal((60, 5))
    k = g @ g.T
    L, piv, d = solvers.pivoted_cholesky(k, 20, pivot_tol=1e-10)
    assert solvers.rank_reached(piv) == 5
    assert np.all(piv[5:] == -1) and np.all(L[:, 5:] == 0.0)
    assert np.allclose(L @ L.T, k, atol=1e-10)


def test_pivots_follow_the_brute_force_schur_complement():
    k = oracle.fc_nngp(synth.correlated_images(50, 8, 8, 3, 3.0, 5).reshape(50, -1),
                       synth.correlated_images(50, 8, 8, 3, 3.0, 5).reshape(50, -1))
    L, piv, d = solvers.pivoted_cholesky(k, 12)
    picked = []
    for m in range(12):
        s = k - L[:, :m] @ L[:, :m].T  # explicit Schur complement (up to the permutation)
        diag = np.diag(s).copy()
        diag[picked] = -np.inf
        assert piv[m] == int(np.argmax(diag)), f"step {m}"
        picked.append(int(piv[m]))
    # residual diagonal = diag(K - L L^T) and the trace error decreases
    assert np.allclose(np.where(np.isin(np.arange(50), picked), 0.0, np.diag(k - L @ L.T)), d, atol=1e-10)
    tr = [np.trace(k - L[:, :m] @ L[:, :m].T) for m in range(13)]
    assert all(tr[m + 1] < tr[m] for m in range(12))


def test_diagonal_matrix_pivots_by_size_lowest_index_first():
    dg = np.array([1.0, 3.0, 2.0, 3.0, 0.5])
    L, piv, d = solvers.pivoted_cholesky(np.diag(dg), 5)
    assert piv.tolist() == [1, 3, 2, 0, 4]
    for m, p in enumerate(piv):
        e = np.zeros(5)
        e[p] = np.sqrt(dg[p])
        assert np.array_equal(L[:, m], e)


def test_woodbury_apply_equals_the_dense_inverse():
    k = _spd(30, 3)
    L, _, _ = solvers.pivoted_cholesky(k, 7)
    lam = 0.05
    v = np.random.default_rng(4).standard_normal((30, 3))
    got = solvers.WoodburyPreconditioner(L, lam).apply(v)
    ref = np.linalg.solve(L @ L.T + lam * np.eye(30), v)
    assert np.allclose(got, ref, rtol=1e-11, atol=1e-12)
    assert np.allclose(solvers.WoodburyPreconditioner(L[:, :0], lam).apply(v), v / lam)


def test_cg_terminates_in_as_many_steps_as_distinct_eigenvalues():
    rng = np.random.default_rng(6)
    q, _ = np.linalg.qr(rng.standard_normal((24, 24)))
    ev = np.repeat([0.5, 2.0, 7.0], 8)
    k = q @ np.diag(ev) @ q.T
    y = rng.standard_normal((24, 2))
    res = solvers.pcg(k, y, lam=0.1, rank=0, tol=1e-11, max_iter=50)
    assert np.all(res["iters"] <= 3)
    assert np.allclose(res["X"], np.linalg.solve(k + 0.1 * np.eye(24), y), rtol=1e-9, atol=1e-11)


def test_full_rank_preconditioner_converges_in_one_step():
    k = _spd(35, 7)
    y = np.random.default_rng(8).standard_normal((35, 3))
    res = solvers.pcg(k, y, lam=0.01, rank=35, tol=1e-9, max_iter=10)
    assert np.all(res["iters"] == 1)


def test_pcg_matches_the_direct_solve_and_preconditioning_helps():
    x = synth.correlated_images(300, 8, 8, 3, 3.0, 9).reshape(300, -1)
    k = oracle.fc_nngp(x, x)
    y = synth.teacher_labels(x.reshape(300, 8, 8, 3), 10, 10).astype(np.float64)
    lam = solvers.ridge_lambda(k, 1e-4, True)
    ref = sla.cho_solve(sla.cho_factor(k + lam * np.eye(300), lower=True), y)
    plain = solvers.pcg(k, y, lam, rank=0, tol=1e-10, max_iter=2000)
    pre = solvers.pcg(k, y, lam, rank=100, tol=1e-10, max_iter=2000)
    for res in (plain, pre):
        assert np.all(res["relres"] <= 1e-10)
        true = np.linalg.norm((k + lam * np.eye(300)) @ res["X"] - y, axis=0) / np.linalg.norm(y, axis=0)
        assert np.all(true <= 1e-8)
        assert np.allclose(res["X"], ref, rtol=1e-5, atol=1e-6 * np.abs(ref).max())
    assert pre["iters"].max() < plain["iters"].max() / 2


def test_a_norm_error_decreases_every_step():
    k = _spd(50, 11, floor=1e-2)
    y = np.random.default_rng(12).standard_normal(50)
    a = k + 0.01 * np.eye(50)
    xs = np.linalg.solve(a, y)
    res = solvers.pcg(k, y, 0.01, rank=5, tol=1e-13, max_iter=60, history=True)
    errs = [float((h[:, 0] - xs) @ a @ (h[:, 0] - xs)) for h in res["history"]]
    assert all(errs[i + 1] <= errs[i] * (1 + 1e-12) for i in range(len(errs) - 1))


def test_zero_target_column_and_frozen_columns():
    k = _spd(20, 13)
    y = np.random.default_rng(14).standard_normal((20, 3))
    y[:, 1] = 0.0
    res = solvers.pcg(k, y, 0.05, rank=3, tol=1e-8, max_iter=100)
    assert res["iters"][1] == 0 and np.all(res["X"][:, 1] == 0.0)
    # a column solved alone takes the same updates as inside the batch
    solo = solvers.pcg(k, y[:, 2:3], 0.05, rank=3, tol=1e-8, max_iter=100)
    assert solo["iters"][0] == res["iters"][2]
    # (BLAS may round a one-column product differently from a three-column one)
    assert np.allclose(solo["X"][:, 0], res["X"][:, 2], rtol=1e-6, atol=1e-9)
