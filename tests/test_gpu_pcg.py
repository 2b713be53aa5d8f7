"""GPU tests of the conjugate-gradient solver path (nk_pivoted_cholesky,
nk_gram_matvec, nk_krr_pcg) against the FP64 solver oracle on the same
float32 Gram matrices (promoted to float64 on both sides).

Tolerances.  Both sides run the same float64 recursions in different
summation orders, so values differ by rounding amplified by the condition
of the system: pivots must agree exactly wherever the two largest
candidates are separated by more than 1e-9 of the largest diagonal; L
within 1e-9 of sqrt(max diag K); the product within 1e-12 relative; PCG
iterates within 1e-6 relative, and every solution's true residual below
10 tol.  Iteration counts are decided partly by rounding: on these systems
the float64 residual plateaus near 4e-10 (the attainable accuracy of the
recursion), and a relative perturbation of K by 2e-16 already moves the
oracle's counts by up to 4 for plain CG at tol = 1e-8.  So each count must
not exceed the oracle's by more than 2 s + 1, s being the oracle's largest
spread between K and three such perturbed copies of K.  The bound is one
sided: the GPU, whose x and r updates are fused multiply-adds (one
rounding where numpy rounds twice), converges at or before the oracle on
nearly every column (up to five iterations earlier for plain CG, up to two
with a rank-30 preconditioner); its solutions are held to the oracle's by
the iterate and true-residual bars above."""
import sys

import numpy as np
import pytest
import torch

import oracle
import synth
from oracle import solvers

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def nk():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2303_05420_amd import ops
    return ops


def _gram32(n, seed, hw=16):
    """FP64 oracle FC-3 NNGP Gram of correlated images, rounded once to float32."""
    x = synth.correlated_images(n, hw, hw, 3, 3.0, seed).reshape(n, -1)
    return oracle.fc_nngp(x, x).astype(np.float32), x


def _pivot_margin_ok(k64, L, piv, m):
    """Whether step m's choice was separated from the runner-up by > 1e-9 max diag."""
    s = np.diag(k64 - L[:, :m] @ L[:, :m].T).copy()
    s[piv[:m]] = -np.inf
    top = np.sort(s)[-2:]
    return (top[1] - top[0]) > 1e-9 * np.max(np.diag(k64))


def test_pivoted_cholesky_matches_oracle(nk):
    k32, _ = _gram32(700, 31)  # 700 rows: two full 256-row blocks and a ragged one
    k64 = k32.astype(np.float64)
    _say("pivoted cholesky n=700 rank=64")
    L, piv, used = nk.pivoted_cholesky(torch.from_numpy(k32).cuda(), 64)
    L = L.cpu().numpy()
    piv = piv.cpu().numpy()
    Lr, pr, _ = solvers.pivoted_cholesky(k64, 64)
    assert used == 64 == solvers.rank_reached(pr)
    for m in range(64):
        if piv[m] != pr[m]:
            assert not _pivot_margin_ok(k64, Lr, pr, m), f"pivot {m}: {piv[m]} vs {pr[m]}"
            pytest.skip("near-tie pivot; later columns not comparable")
    scale = np.sqrt(np.max(np.diag(k64)))
    assert np.max(np.abs(L - Lr)) <= 1e-9 * scale
    # a column of picked rows is exactly zero above its own pivot
    for m in range(1, 64):
        assert np.all(L[piv[:m], m] == 0.0)


def test_pivoted_cholesky_stops_at_exact_rank(nk):
    rng = np.random.default_rng(32)
    g = rng.standard_normal((300, 6))
    k32 = (g @ g.T).astype(np.float32)
    k64 = k32.astype(np.float64)
    _say("pivoted cholesky low rank")
    L, piv, used = nk.pivoted_cholesky(torch.from_numpy(k32).cuda(), 40, pivot_tol=1e-5)
    Lr, pr, _ = solvers.pivoted_cholesky(k64, 40, pivot_tol=1e-5)
    assert used == solvers.rank_reached(pr)
    assert 6 <= used < 40
    assert np.array_equal(piv.cpu().numpy(), pr.astype(np.int32))
    L = L.cpu().numpy()
    assert np.all(L[:, used:] == 0.0)
    assert np.max(np.abs(L @ L.T - k64)) <= 1e-4 * np.max(np.diag(k64))


@pytest.mark.parametrize("n,c,pad", [(1000, 10, 0), (1000, 1, 0), (777, 16, 5), (1030, 3, 2), (64, 7, 0)])
def test_gram_matvec_matches_float64(nk, n, c, pad):
    rng = np.random.default_rng(n + c)
    a = rng.standard_normal((n, n)).astype(np.float32)
    k32 = ((a + a.T) / 2).astype(np.float32)
    kp = np.zeros((n, n + pad), dtype=np.float32)
    kp[:, :n] = k32
    p = rng.standard_normal((n, c))
    lam = 0.37
    _say(f"gram matvec n={n} c={c} ldk={n + pad}")
    kt = torch.from_numpy(kp).cuda()[:, :n]
    q = nk.gram_matvec(kt, torch.from_numpy(p).cuda(), lam).cpu().numpy()
    ref = k32.astype(np.float64) @ p + lam * p
    assert np.max(np.abs(q - ref)) <= 1e-12 * np.max(np.abs(ref))
    # bitwise reproducible
    q2 = nk.gram_matvec(kt, torch.from_numpy(p).cuda(), lam).cpu().numpy()
    assert np.array_equal(q, q2)


def _count_band(k64, y, lam, rank, tol, max_iter, ref):
    """2 s + 1, s = the oracle's largest count spread over three 2e-16 relative
    symmetric perturbations of K."""
    s = np.zeros_like(ref["iters"])
    for seed in (7, 8, 9):
        e = np.random.default_rng(seed).standard_normal(k64.shape)
        kp = k64 * (1.0 + 1e-16 * (e + e.T))
        alt = solvers.pcg(kp, y, lam, rank, tol, max_iter)
        s = np.maximum(s, np.abs(alt["iters"] - ref["iters"]))
    return 2 * s + 1


def _check_pcg(k32, y, got, ref, tol, band):
    x, iters, relres, stats = got
    x = x.cpu().numpy()
    k64 = k32.astype(np.float64)
    lam = stats["lambda"]
    assert abs(lam - solvers.ridge_lambda(k64, 1e-4, True)) <= 1e-12 * lam
    assert stats["rank"] == ref["rank"]
    assert np.all(iters.astype(np.int64) - ref["iters"] <= band), (iters, ref["iters"], band)
    conv = ref["iters"] > 0
    assert np.all(relres[conv] <= tol)
    a = k64 + lam * np.eye(len(k64))
    true = np.linalg.norm(a @ x - y, axis=0) / np.maximum(np.linalg.norm(y, axis=0), 1e-300)
    assert np.all(true[conv] <= 10 * tol), true
    assert np.max(np.abs(x - ref["X"])) <= 1e-6 * np.max(np.abs(ref["X"]))


@pytest.mark.parametrize("tol", [1e-8, 1e-10])
def test_krr_pcg_matches_oracle(nk, tol):
    k32, x = _gram32(1500, 33)
    y = synth.teacher_labels(x.reshape(1500, 16, 16, 3), 10, 34).astype(np.float64)
    _say(f"pcg n=1500 c=10 rank=100 tol={tol}")
    got = nk.krr_pcg(torch.from_numpy(k32).cuda(), torch.from_numpy(y).cuda(), 1e-4, True, rank=100, tol=tol,
                     max_iter=3000)
    k64 = k32.astype(np.float64)
    lam = solvers.ridge_lambda(k64, 1e-4, True)
    ref = solvers.pcg(k64, y, lam, 100, tol, 3000)
    band = _count_band(k64, y, lam, 100, tol, 3000, ref)
    _say(f"  iterations {got[1].tolist()} vs {ref['iters'].tolist()} (band {band.tolist()})")
    _check_pcg(k32, y, got, ref, tol, band)


def test_krr_pcg_4096_rank64_does_not_stall(nk):
    """n = 4096, rank 64: the case where a Woodbury matrix M = lam I + L^T L
    summed naively over the 4096 rows (about 3e-15 relative error instead
    of about 1e-16) made five of the ten columns stall near 1e-8 for some 50
    iterations; M is now accumulated with compensated sums."""
    m = 4096
    xs = synth.correlated_images(m, 16, 16, 3, 3.0, 77)
    y = synth.teacher_labels(xs, 10, 78).astype(np.float64)
    k32 = oracle.fc_nngp(xs.reshape(m, -1), xs.reshape(m, -1)).astype(np.float32)
    k64 = k32.astype(np.float64)
    lam = solvers.ridge_lambda(k64, 1e-4, True)
    _say("pcg n=4096 c=10 rank=64")
    got = nk.krr_pcg(torch.from_numpy(k32).cuda(), torch.from_numpy(y).cuda(), 1e-4, True, rank=64, tol=1e-8,
                     max_iter=3000)
    ref = solvers.pcg(k64, y, lam, 64, 1e-8, 3000)
    _say(f"  iterations {got[1].tolist()} vs {ref['iters'].tolist()}")
    _check_pcg(k32, y, got, ref, 1e-8, np.full(10, 3))


def test_krr_pcg_two_groups_zero_column_and_plain_cg(nk):
    k32, x = _gram32(600, 35, hw=8)
    rng = np.random.default_rng(36)
    y = rng.standard_normal((600, 20))
    y[:, 7] = 0.0
    k64 = k32.astype(np.float64)
    lam = solvers.ridge_lambda(k64, 1e-4, True)
    for rank in (0, 30):
        _say(f"pcg n=600 c=20 rank={rank}")
        got = nk.krr_pcg(torch.from_numpy(k32).cuda(), torch.from_numpy(y).cuda(), 1e-4, True, rank=rank, tol=1e-8,
                         max_iter=4000)
        ref = solvers.pcg(k64, y, lam, rank, 1e-8, 4000)
        band = _count_band(k64, y, lam, rank, 1e-8, 4000, ref)
        _say(f"  iterations {got[1].tolist()} vs {ref['iters'].tolist()} (band {band.tolist()})")
        assert got[1][7] == 0 and np.all(got[0].cpu().numpy()[:, 7] == 0.0)
        _check_pcg(k32, y, got, ref, 1e-8, band)


def test_krr_pcg_iteration_cap_and_absolute_ridge(nk):
    k32, x = _gram32(400, 37, hw=8)
    y = np.random.default_rng(38).standard_normal((400, 2))
    k64 = k32.astype(np.float64)
    _say("pcg iteration cap")
    xg, iters, relres, stats = nk.krr_pcg(torch.from_numpy(k32).cuda(), torch.from_numpy(y).cuda(), 1e-3, False,
                                          rank=10, tol=1e-14, max_iter=7)
    ref = solvers.pcg(k64, y, 1e-3, 10, 1e-14, 7)
    assert stats["lambda"] == 1e-3
    assert np.all(iters == 7) and np.all(ref["iters"] == 7)
    assert np.allclose(relres, ref["relres"], rtol=1e-6)
    assert np.max(np.abs(xg.cpu().numpy() - ref["X"])) <= 1e-8 * np.max(np.abs(ref["X"]))


def test_krr_pcg_full_size_sampled_residual(nk):
    """n = 32768 (a 4 GiB float32 Gram, FC-3 NNGP of 32x32x3 correlated
    images computed on the GPU), 10 targets, rank 512: the true residual of
    sampled rows, recomputed on the host in float64 from the same float32
    rows, and the recursive residuals."""
    n = 32768
    xs = synth.correlated_images(n, 32, 32, 3, 3.0, 39)
    y = synth.teacher_labels(xs, 10, 40).astype(np.float64)
    xt = torch.from_numpy(xs.reshape(n, -1)).cuda()
    _say("fc nngp 32768^2")
    k = nk.fc_nngp(xt, None, depth=3, sigma_w2=2.0, sigma_b2=0.01)
    del xt
    # the solver reads K by rows as its columns: make it exactly symmetric
    kt = k.t().contiguous()
    k.add_(kt).mul_(0.5)
    del kt
    tol = 1e-6
    _say("pcg n=32768 c=10 rank=512")
    x, iters, relres, stats = nk.krr_pcg(k, torch.from_numpy(y).cuda(), 1e-4, True, rank=512, tol=tol,
                                         max_iter=2000)
    _say(f"  rank {stats['rank']} iterations {iters.tolist()}")
    assert stats["rank"] == 512
    assert np.all(relres <= tol) and np.all(iters < 2000)
    rows = np.random.default_rng(41).choice(n, 16, replace=False)
    kr = k[torch.from_numpy(rows).cuda()].cpu().numpy().astype(np.float64)
    xh = x.cpu().numpy()
    res = kr @ xh + stats["lambda"] * xh[rows] - y[rows]
    # sampled rows of the residual: each is at most the whole residual norm
    assert np.all(np.abs(res) <= 10 * tol * np.linalg.norm(y, axis=0))
