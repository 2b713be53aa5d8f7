"""GPU tests of the approximate kernel-regression solvers (nk_krr_nystrom,
nk_krr_sor, nk_krr_block_diag, nk_krr_bcm) against the FP64 oracle on the
same float32 kernel blocks.  Both sides compute in float64 from the same
float32 inputs; the GPU rounds its predictions to float32 once, so the bar
is 1e-6 of the largest prediction (16x the float32 rounding of the output,
leaving room for float64 summation-order differences amplified by the
conditioning of each method's system)."""
import sys

import numpy as np
import pytest
import torch

import oracle
import synth
from oracle import approx

pytestmark = pytest.mark.gpu
TOL = 1e-6


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def nk():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2303_05420_amd import ops
    return ops


@pytest.fixture(scope="module")
def data():
    n, m = 700, 90
    x = synth.correlated_images(n + m, 16, 16, 3, 3.0, 8001).reshape(n + m, -1)
    k = oracle.fc_nngp(x, x).astype(np.float32)
    y = synth.teacher_labels(x[:n].reshape(n, 16, 16, 3), 10, 8002).astype(np.float32)
    lam = float(1e-4 * np.mean(np.diag(k[:n, :n].astype(np.float64))))
    return k[:n, :n], k[n:, :n], k[n:, n:], y, lam


def _g(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _close(got, ref):
    got = got.cpu().numpy()
    err = float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))
    _say(f"  max error / max |pred| = {err:.2e}")
    assert err <= TOL


@pytest.mark.parametrize("r,jitter", [(64, 1e-6), (333, 1e-4), (700, 0.0)])
def test_nystrom_and_sor(nk, data, r, jitter):
    ktr, kte, _, y, lam = data
    sub = np.random.default_rng(8003 + r).choice(len(ktr), r, replace=False)
    k_nr, k_rr, k_mr = ktr[:, sub], ktr[np.ix_(sub, sub)], kte[:, sub]
    k64 = [a.astype(np.float64) for a in (k_nr, k_rr, kte, k_mr, y)]
    _say(f"nystrom r={r} jitter={jitter}")
    got = nk.krr_nystrom(_g(k_nr), _g(k_rr), _g(kte), _g(y), lam, jitter)
    _close(got, approx.nystrom_predict(k64[0], k64[1], k64[2], k64[4], lam, jitter))
    _say(f"sor r={r}")
    got = nk.krr_sor(_g(k_nr), _g(k_rr), _g(k_mr), _g(y), lam, jitter)
    _close(got, approx.sor_predict(k64[0], k64[1], k64[3], k64[4], lam, jitter))


@pytest.mark.parametrize("sizes", [[700], [300, 250, 150], [100] * 7, [64, 1, 635]])
def test_block_diag_and_bcm(nk, data, sizes):
    ktr, kte, ktt, y, lam = data
    perm = np.random.default_rng(8010 + len(sizes)).permutation(len(ktr))
    kp, kmp, yp = ktr[np.ix_(perm, perm)], kte[:, perm], y[perm]
    offs = np.concatenate([[0], np.cumsum(sizes)])
    blocks = [np.ascontiguousarray(kp[offs[i]:offs[i + 1], offs[i]:offs[i + 1]]) for i in range(len(sizes))]
    kmb = [kmp[:, offs[i]:offs[i + 1]].astype(np.float64) for i in range(len(sizes))]
    yb = [yp[offs[i]:offs[i + 1]].astype(np.float64) for i in range(len(sizes))]
    _say(f"block diagonal {sizes}")
    got = nk.krr_block_diag([_g(b) for b in blocks], _g(kmp), _g(yp), lam)
    _close(got, approx.block_diag_predict([b.astype(np.float64) for b in blocks], kmb, yb, lam))
    _say(f"bcm {sizes}")
    got = nk.krr_bcm([_g(b) for b in blocks], _g(kmp), _g(ktt), _g(yp), lam, 1e-6)
    _close(got, approx.bcm_predict([b.astype(np.float64) for b in blocks], kmb, yb, ktt.astype(np.float64), lam,
                                   1e-6))
