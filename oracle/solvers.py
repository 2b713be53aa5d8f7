"""FP64 CPU oracle for the kernel-regression solvers: the partial pivoted
Cholesky factor, its preconditioner, and preconditioned conjugate gradients
(Sec. 2, "Iterative solvers"; Sec. 1, related work, for the preconditioner
and the need for high precision).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this module.  It shares no
code with the GPU library and never imports it.

The system is (K + lam I) X = Y with K symmetric positive semi-definite
(n x n), lam > 0 and Y (n x c): one column per regression target, solved
independently (the paper runs CG vectorised over tasks, App. B).

Partial pivoted Cholesky (the greedy diagonal-pivoting form of the
preconditioner the paper takes from its CG references): with d the diagonal
of the current Schur complement of K (d = diag K at the start), step m picks
the not-yet-picked index p with the largest d (lowest index on ties), stops
if d_p <= pivot_tol * max(diag K) or d_p <= 0, and otherwise appends the
column
    l(p) = sqrt(d_p),  l(i) = (K[p, i] - sum_{k<m} L[p, k] L[i, k]) / l(p)
for the indices not picked yet (0 at picked ones), then d_i -= l(i)^2 and p
leaves the candidate set.  After r steps K ~ L L^T with L n x r, and
diag(K - L L^T) = d.

Preconditioner  Ph = L L^T + lam I,  applied with the Woodbury identity
    Ph^{-1} v = (v - L (lam I_r + L^T L)^{-1} L^T v) / lam.
Rank 0 leaves Ph = lam I, i.e. plain CG.

PCG per column j, from x = 0 (the textbook recursion, Shewchuk's "method of
preconditioned conjugate gradients"):
    r = y, z = Ph^{-1} r, p = z, gamma = r.z
    repeat:  q = A p,  alpha = gamma / p.q,  x += alpha p,  r -= alpha q,
             stop the column once ||r|| <= tol ||y||,
             z = Ph^{-1} r,  gamma' = r.z,  p = z + (gamma'/gamma) p.
A stopped column keeps its x; its iteration count is the number of updates
it took.  A zero column of Y gives x = 0 after 0 iterations.
"""
from __future__ import annotations

import numpy as np


def pivoted_cholesky(k: np.ndarray, rank: int, pivot_tol: float = 0.0):
    """Greedy partial pivoted Cholesky of a PSD matrix (float64).

    Returns (L, piv, d): L (n x rank, columns past the rank reached are 0),
    piv (rank entries, -1 past the rank reached) and the final residual
    diagonal d (0 at picked indices)."""
    k = np.asarray(k, dtype=np.float64)
    n = k.shape[0]
    rank = int(min(max(rank, 0), n))
    L = np.zeros((n, rank))
    piv = np.full(rank, -1, dtype=np.int64)
    d = np.diag(k).copy()
    picked = np.zeros(n, dtype=bool)
    dmax0 = float(np.max(d)) if n else 0.0
    for m in range(rank):
        cand = np.where(picked, -np.inf, d)
        p = int(np.argmax(cand))  # first maximum: lowest index on ties
        dp = float(cand[p])
        if not dp > 0.0 or dp <= pivot_tol * dmax0:
            break
        lp = np.sqrt(dp)
        col = (k[p, :] - L[:, :m] @ L[p, :m]) / lp
        col[picked] = 0.0
        col[p] = lp
        L[:, m] = col
        rest = ~picked
        rest[p] = False
        d[rest] -= col[rest] ** 2
        d[p] = 0.0
        picked[p] = True
        piv[m] = p
    return L, piv, d


def rank_reached(piv: np.ndarray) -> int:
    return int(np.sum(np.asarray(piv) >= 0))


class WoodburyPreconditioner:
    """Ph = L L^T + lam I and its inverse by the Woodbury identity."""

    def __init__(self, L: np.ndarray, lam: float):
        import scipy.linalg as sla

        self.L = np.asarray(L, dtype=np.float64)
        self.lam = float(lam)
        r = self.L.shape[1]
        self.cf = sla.cho_factor(self.lam * np.eye(r) + self.L.T @ self.L, lower=True) if r else None

    def apply(self, v: np.ndarray) -> np.ndarray:
        import scipy.linalg as sla

        v = np.asarray(v, dtype=np.float64)
        if self.cf is None:
            return v / self.lam
        return (v - self.L @ sla.cho_solve(self.cf, self.L.T @ v)) / self.lam


def ridge_lambda(k: np.ndarray, ridge: float, relative: bool) -> float:
    """lam = ridge, or ridge * mean(diag K) when relative."""
    return float(ridge) * float(np.mean(np.diag(k))) if relative else float(ridge)


def pcg(k: np.ndarray, y: np.ndarray, lam: float, rank: int, tol: float, max_iter: int,
        pivot_tol: float = 0.0, history: bool = False):
    """Solve (K + lam I) X = Y column by column with preconditioned CG.

    Returns a dict with X (n x c), iters (c), relres (c, the recursive
    residual ||r|| / ||y|| at the column's last update), rank (of the
    preconditioner reached), piv, L, and, with history=True, the iterate X
    after every iteration."""
    k = np.asarray(k, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    squeeze = y.ndim == 1
    if squeeze:
        y = y[:, None]
    n, c = y.shape
    a = k + lam * np.eye(n)
    L, piv, _ = pivoted_cholesky(k, rank, pivot_tol)
    prec = WoodburyPreconditioner(L, lam)

    x = np.zeros((n, c))
    r = y.copy()
    z = prec.apply(r)
    p = z.copy()
    gamma = np.sum(r * z, axis=0)
    ynorm = np.linalg.norm(y, axis=0)
    active = ynorm > 0
    iters = np.zeros(c, dtype=np.int64)
    relres = np.zeros(c)
    relres[active] = 1.0
    hist = [x.copy()] if history else None
    for it in range(max_iter):
        if not active.any():
            break
        q = a @ p
        pq = np.sum(p * q, axis=0)
        alpha = np.where(active, gamma / np.where(active, pq, 1.0), 0.0)
        x += alpha * p
        r -= alpha * q
        rel = np.linalg.norm(r, axis=0) / np.where(active, ynorm, 1.0)
        relres[active] = rel[active]
        iters[active] = it + 1
        active = active & ~(rel <= tol)
        z = prec.apply(r)
        gnew = np.sum(r * z, axis=0)
        beta = np.where(active, gnew / np.where(active, gamma, 1.0), 0.0)
        gamma = np.where(active, gnew, gamma)
        p = z + beta * p
        if history:
            hist.append(x.copy())
    out = {"X": x[:, 0] if squeeze else x, "iters": iters, "relres": relres, "rank": rank_reached(piv),
           "piv": piv, "L": L}
    if history:
        out["history"] = hist
    return out
