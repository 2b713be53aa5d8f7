"""GPU tests of the CNN-VEC NNGP (nk_cv_nngp) against the FP64 oracle:
max |K_gpu - K_ref| / sqrt(K_ref(x,x) K_ref(x',x')) <= 2e-5 on full blocks
(symmetric and not, ragged pair counts, padded ldk) at every supported
resolution, CV8 at 32x32x3 on a 4096 x 4096 block by sampled entries."""
import sys

import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu
TOL = 2e-5


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def nk():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2303_05420_amd import ops
    return ops


def _err(got, ref, d1, d2):
    return float(np.max(np.abs(got - ref) / np.sqrt(np.outer(d1, d2))))


@pytest.mark.parametrize("hw,n1,n2,depth,sb2,sym", [
    (8, 128, 128, 8, 0.01, True),
    (32, 77, 53, 8, 0.01, False),
    (32, 40, 40, 8, 0.0, True),
    (16, 33, 65, 5, 0.01, False),
    (4, 50, 9, 3, 0.1, False),
    (2, 20, 20, 1, 0.01, True),
])
def test_cv_block_matches_oracle(nk, hw, n1, n2, depth, sb2, sym):
    xa = synth.correlated_images(n1, hw, hw, 3, 2.0, 100 + hw)
    xb = xa if sym else synth.correlated_images(n2, hw, hw, 3, 2.0, 200 + hw)
    _say(f"cv {hw}x{hw} depth {depth} {n1}x{n2} sym={sym}")
    ta = torch.from_numpy(xa).cuda()
    tb = ta if sym else torch.from_numpy(xb).cuda()
    got = nk.cv_nngp(ta, None if sym else tb, depth=depth, sigma_w2=2.0, sigma_b2=sb2).cpu().numpy()
    _, d1 = oracle.cv_self(xa, depth, 2.0, sb2)
    _, d2 = oracle.cv_self(xb, depth, 2.0, sb2)
    ref = oracle.cv_gram(xa, xb, depth, 2.0, sb2)
    err = _err(got, ref, d1, d2)
    _say(f"  max normalised error {err:.2e}")
    assert err <= TOL
    if sym:
        assert np.array_equal(got, got.T)


def test_cv_padded_ldk_and_channels(nk):
    x1 = synth.iid_images(30, 8, 8, 1, 301)
    x2 = synth.iid_images(17, 8, 8, 1, 302)
    out = torch.full((30, 25), float("nan"), device="cuda")
    nk.cv_nngp(torch.from_numpy(x1).cuda(), torch.from_numpy(x2).cuda(), depth=4, out=out[:, :17])
    torch.cuda.synchronize()
    o = out.cpu().numpy()
    assert np.isnan(o[:, 17:]).all()
    _, d1 = oracle.cv_self(x1, 4)
    _, d2 = oracle.cv_self(x2, 4)
    assert _err(o[:, :17], oracle.cv_gram(x1, x2, 4), d1, d2) <= TOL


def test_cv8_32x32_4096_sampled(nk):
    """CV8 at 32x32x3 (the benchmark block): 64 sampled entries vs the oracle."""
    n = 4096
    xa = synth.correlated_images(n, 32, 32, 3, 3.0, 7001)
    xb = synth.correlated_images(n, 32, 32, 3, 3.0, 7002)
    _say("cv8 32x32 4096x4096")
    got = nk.cv_nngp(torch.from_numpy(xa).cuda(), torch.from_numpy(xb).cuda(), depth=8).cpu().numpy()
    rng = np.random.default_rng(7003)
    r = rng.integers(0, n, 64)
    c = rng.integers(0, n, 64)
    q1, d1 = oracle.cv_self(xa[r], 8)
    q2, d2 = oracle.cv_self(xb[c], 8)
    ref = oracle.cv_pairs(xa[r], xb[c], np.stack([np.arange(64), np.arange(64)], 1), 8, q1=q1, q2=q2)
    err = float(np.max(np.abs(got[r, c] - ref) / np.sqrt(d1 * d2)))
    _say(f"  max normalised error {err:.2e}")
    assert err <= TOL
