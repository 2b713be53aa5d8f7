"""GPU parity at the sizes the measured workloads run at, and the cases where
the correlation of a pair reaches 1 exactly.

* The Myrtle-5 1024 x 1024 block at 32x32x3 (with its symmetric training
  block) by sampled cross and diagonal entries, then ridge regression on it.
* A symmetric Myrtle-10 4096 x 4096 block at 32x32x3 by sampled self and
  cross entries.
* The tangent kernel over several pair passes, and on two arrays holding
  the same images (displacement-0 correlation exactly 1).
* The adjoint with a cotangent on self entries only, on a symmetric block and
  on two arrays holding the same images.
* The torch.autograd.Function over the adjoint, and the one-call
  ridge-regression gradient against its parts.

Metric for kernels: |K_gpu - K_oracle| / sqrt(K(x,x) K(x',x')) <= 2e-5; for
gradients: max |g_gpu - g_ref| / max |g_ref| <= 1e-5 per output."""
import sys

import numpy as np
import pytest
import torch

import oracle
import synth
from oracle import grad as ograd

pytestmark = pytest.mark.gpu

TOL = 2e-5
GTOL = 1e-5


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def nk():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2303_05420_amd import ops
    return ops


def _gpu(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-30))


def test_c2_myrtle5_1024_sampled_then_krr(nk):
    """Myrtle-5 at 32x32x3 on the 1024 train + 1024 test images: >= 128 cross
    entries of K(test, train) and 32 diagonal entries of K(train, train)
    against the oracle, then ridge regression on the GPU blocks against the
    float64 solve of the same blocks."""
    w = synth.WORKLOADS["fc3_myrtle5_32x32_1024"]
    depth = w["depth"]
    xtr = synth.correlated_images(w["n1"], 32, 32, 3, w["length"], w["seeds"][0])
    xte = synth.correlated_images(w["n2"], 32, 32, 3, w["length"], w["seeds"][1])
    y = synth.teacher_labels(xtr, w["n_classes"], w["seeds"][2])
    g_tr, g_te = _gpu(xtr), _gpu(xte)
    _say("myrtle5 1024 train (symmetric) and 1024 x 1024 test blocks on GPU")
    ktr = nk.myrtle_nngp(g_tr, None, depth, w["sigma_w2"], w["sigma_b2"])
    kte = nk.myrtle_nngp(g_te, g_tr, depth, w["sigma_w2"], w["sigma_b2"])
    ktr_h, kte_h = ktr.cpu().numpy(), kte.cpu().numpy()
    assert np.array_equal(ktr_h, ktr_h.T)
    rng = np.random.default_rng(2101)
    cross = np.stack([rng.integers(0, w["n2"], 128), rng.integers(0, w["n1"], 128)], 1)
    diag = rng.choice(w["n1"], 32, replace=False)
    net = oracle.Myrtle(depth, w["sigma_w2"], w["sigma_b2"])
    _say("oracle: 128 cross entries, 32 diagonal entries")
    te_idx = np.unique(cross[:, 0])
    tr_idx = np.unique(np.concatenate([cross[:, 1], diag]))
    q_te, d_te = oracle.myrtle_self(xte[te_idx], net)
    q_tr, d_tr = oracle.myrtle_self(xtr[tr_idx], net)
    pos_te = {int(v): i for i, v in enumerate(te_idx)}
    pos_tr = {int(v): i for i, v in enumerate(tr_idx)}
    loc = np.array([[pos_te[int(a)], pos_tr[int(b)]] for a, b in cross])
    kr = oracle.myrtle_pairs(xte[te_idx], xtr[tr_idx], loc, net, q_te, q_tr)
    err_c = float(np.max(np.abs(kte_h[cross[:, 0], cross[:, 1]] - kr) / np.sqrt(d_te[loc[:, 0]] * d_tr[loc[:, 1]])))
    dref = d_tr[[pos_tr[int(v)] for v in diag]]
    err_d = float(np.max(np.abs(ktr_h[diag, diag] - dref) / dref))
    _say(f"  normalised error cross {err_c:.3e} diagonal {err_d:.3e}")
    assert err_c <= TOL and err_d <= TOL
    _say("krr on the GPU blocks")
    pred = nk.krr_predict(ktr, kte, _gpu(y), w["ridge_rel"]).cpu().numpy()
    ref = oracle.krr_predict(ktr_h, kte_h, y, w["ridge_rel"])
    rel = _rel(pred, ref)
    _say(f"  krr max rel error {rel:.3e}")
    assert rel <= 1e-5


def test_c3_symmetric_myrtle10_4096_sampled(nk):
    """Symmetric Myrtle-10 block of the 4096 images of the headline's first
    set: 16 self entries and 64 cross entries against the oracle, and the
    block exactly symmetric."""
    w = synth.WORKLOADS["myrtle10_32x32_4096"]
    n = w["n1"]
    x = synth.correlated_images(n, 32, 32, 3, w["length"], w["seeds"][0])
    _say(f"myrtle10 symmetric {n} x {n} at 32x32 on GPU")
    k = nk.myrtle_nngp(_gpu(x), None, w["depth"], w["sigma_w2"], w["sigma_b2"]).cpu().numpy()
    rng = np.random.default_rng(3101)
    selfs = rng.choice(n, 16, replace=False)
    cross = rng.integers(0, n, (64, 2))
    cross = cross[cross[:, 0] != cross[:, 1]]
    assert len(cross) >= 60
    idx = np.unique(np.concatenate([selfs, cross.ravel()]))
    pos = {int(v): i for i, v in enumerate(idx)}
    net = oracle.Myrtle(w["depth"], w["sigma_w2"], w["sigma_b2"])
    _say(f"oracle: {len(idx)} self recursions, {len(cross)} cross entries")
    q, d = oracle.myrtle_self(x[idx], net)
    loc = np.array([[pos[int(a)], pos[int(b)]] for a, b in cross])
    kr = oracle.myrtle_pairs(x[idx], x[idx], loc, net, q, q)
    err_c = float(np.max(np.abs(k[cross[:, 0], cross[:, 1]] - kr) / np.sqrt(d[loc[:, 0]] * d[loc[:, 1]])))
    ds = d[[pos[int(v)] for v in selfs]]
    err_s = float(np.max(np.abs(k[selfs, selfs] - ds) / ds))
    _say(f"  normalised error cross {err_c:.3e} self {err_s:.3e}")
    assert err_c <= TOL and err_s <= TOL
    sub = k[np.ix_(idx, idx)]
    assert np.array_equal(sub, sub.T)


def test_ntk_several_passes_sampled(nk):
    """Myrtle-10 tangent kernel on a 256 x 256 block at 32x32x3 (65536 pairs:
    four passes of 16384 pairs): four sampled entries from each pass's range
    of rows against the oracle."""
    w = synth.WORKLOADS["myrtle10_32x32_4096"]
    n = 256
    x1 = synth.correlated_images(n, 32, 32, 3, w["length"], w["seeds"][0])
    x2 = synth.correlated_images(n, 32, 32, 3, w["length"], w["seeds"][1])
    _say("ntk myrtle10 256 x 256 at 32x32 on GPU")
    th, kk = nk.myrtle_ntk(_gpu(x1), _gpu(x2), w["depth"], w["sigma_w2"], w["sigma_b2"], with_nngp=True)
    th, kk = th.cpu().numpy(), kk.cpu().numpy()
    rng = np.random.default_rng(3201)
    # pairs run in 16 x 16 image tiles, tile rows in order: rows [64 p, 64 p + 64) are pass p
    rows = np.concatenate([rng.integers(64 * p, 64 * p + 64, 4) for p in range(4)])
    cols = rng.integers(0, n, 16)
    pairs = np.stack([rows, cols], 1)
    net = oracle.Myrtle(w["depth"], w["sigma_w2"], w["sigma_b2"])
    _say("oracle on 16 sampled pairs")
    rn, rt = oracle.myrtle_ntk_pairs(x1, x2, pairs, net)
    d1n, d1t = oracle.myrtle_ntk_pairs(x1, x1, np.stack([rows] * 2, 1), net)
    d2n, d2t = oracle.myrtle_ntk_pairs(x2, x2, np.stack([cols] * 2, 1), net)
    et = float(np.max(np.abs(th[rows, cols] - rt) / np.sqrt(d1t * d2t)))
    en = float(np.max(np.abs(kk[rows, cols] - rn) / np.sqrt(d1n * d2n)))
    _say(f"  normalised error NTK {et:.3e} NNGP {en:.3e}")
    assert et <= TOL and en <= TOL


@pytest.mark.parametrize("hw,depth", [(32, (3, 3, 3)), (8, (2, 1, 1))])
def test_ntk_identical_images_as_two_arrays(nk, hw, depth):
    """Theta(x, x') with x' a copy of x in another array: every entry,
    diagonal included, within the bar (the displacement-0 correlation of a
    diagonal pair is 1 exactly and must not be taken from a rounded value);
    the result equals the symmetric block's on the diagonal."""
    x = synth.correlated_images(6, hw, hw, 3, 3.0, 3301)
    net = oracle.Myrtle(depth, 2.0, 0.0)
    _say(f"ntk x vs copy of x, 6 images at {hw}x{hw}, depth {depth}")
    gx = _gpu(x)
    th = nk.myrtle_ntk(gx, gx.clone(), depth).cpu().numpy()
    ths = nk.myrtle_ntk(gx, None, depth).cpu().numpy()
    a, b = np.meshgrid(np.arange(6), np.arange(6), indexing="ij")
    pairs = np.stack([a.ravel(), b.ravel()], 1)
    _, rt = oracle.myrtle_ntk_pairs(x, x.copy(), pairs, net)
    rt = rt.reshape(6, 6)
    d = np.diag(rt)
    err = float(np.max(np.abs(th - rt) / np.sqrt(np.outer(d, d))))
    err_diag = float(np.max(np.abs(np.diag(th) - d) / d))
    _say(f"  normalised error all {err:.3e} diagonal {err_diag:.3e}; sym diagonal vs copy diagonal "
         f"{float(np.max(np.abs(np.diag(ths) - np.diag(th)) / d)):.3e}")
    assert err <= TOL and err_diag <= TOL
    assert np.max(np.abs(np.diag(ths) - np.diag(th)) / d) <= 1e-6


@pytest.mark.parametrize("two_arrays", [False, True])
def test_vjp_identity_cotangent_32x32(nk, two_arrays):
    """Adjoint of a Myrtle-5 32x32 block of 3 images with dK = I (cotangent on
    self entries only, where the correlation of the displacement-0 tile is 1
    exactly): the symmetric block, and the same images passed as two arrays,
    against the float64 autograd oracle."""
    x = synth.correlated_images(3, 32, 32, 3, 3.0, 3401)
    depth = (2, 1, 1)
    gk = np.eye(3, dtype=np.float32)
    _say(f"vjp dK = I, 3 images at 32x32, two arrays: {two_arrays}")
    gx = _gpu(x)
    if two_arrays:
        dx1, dx2, ds = nk.myrtle_nngp_backward(gx, gx.clone(), _gpu(gk), depth, 2.0, 0.0)
        g = dx1.cpu().numpy().astype(np.float64) + dx2.cpu().numpy()
    else:
        dx1, dx2, ds = nk.myrtle_nngp_backward(gx, None, _gpu(gk), depth, 2.0, 0.0)
        assert dx2 is None
        g = dx1.cpu().numpy().astype(np.float64)
    pairs = np.stack([np.arange(3)] * 2, 1)
    r, _, rs, _ = ograd.myrtle_vjp(x, None, pairs, np.ones(3), depth, 2.0, 0.0)
    e = _rel(g, r)
    es = np.abs(ds.cpu().numpy() - rs) / np.abs(rs)
    _say(f"  rel err dx {e:.2e} dsigma {es}")
    assert e <= GTOL and np.all(es <= GTOL)


def test_vjp_without_x2_gradient_32x32(nk):
    """The adjoint without x2's seed gradients (dx2 not asked for; at 32x32 a
    kernel variant that keeps no j-side image sums) gives the same dx1 and
    dsigma as the full adjoint, up to float64 summation order."""
    depth = (2, 1, 1)
    x1 = _gpu(synth.correlated_images(5, 32, 32, 3, 3.0, 3701))
    x2 = _gpu(synth.correlated_images(7, 32, 32, 3, 3.0, 3702))
    g = _gpu(np.random.default_rng(3703).standard_normal((5, 7)).astype(np.float32))
    _say("vjp 5 x 7 at 32x32 with and without dx2")
    a1, a2, sa = nk.myrtle_nngp_backward(x1, x2, g, depth, 2.0, 0.02)
    a1, a2, sa = a1.clone(), a2.clone(), sa.clone()
    b1, b2, sb = nk.myrtle_nngp_backward(x1, x2, g, depth, 2.0, 0.02, need_dx2=False)
    assert b2 is None and a2 is not None
    e = float((a1 - b1).abs().max() / a1.abs().max())
    es = float(((sa - sb).abs() / sa.abs()).max())
    _say(f"  dx1 {e:.2e} dsigma {es:.2e}")
    assert e <= 1e-6 and es <= 1e-6


@pytest.mark.parametrize("mode", ["x2_none", "x2_is_x1", "distinct", "distinct_x2_fixed"])
def test_autograd_function(nk, mode):
    """torch.autograd through MyrtleNNGP: gradients of sum(K * G) with respect
    to the images and to both sigmas (given as tensors) against the float64
    autograd oracle."""
    from paper_2303_05420_amd import autograd

    depth = (2, 1, 1)
    x1 = synth.correlated_images(3, 8, 8, 3, 2.0, 3501)
    x2 = synth.correlated_images(4, 8, 8, 3, 2.0, 3502)
    t1 = _gpu(x1).requires_grad_(True)
    t2 = _gpu(x2).requires_grad_(mode != "distinct_x2_fixed")
    sw = torch.tensor(2.0, dtype=torch.float64, requires_grad=True)
    sb = torch.tensor(0.03, dtype=torch.float64, requires_grad=True)
    if mode == "x2_none":
        k = autograd.myrtle_nngp(t1, None, sw, sb, depth)
    elif mode == "x2_is_x1":
        k = autograd.MyrtleNNGP.apply(t1, t1, sw, sb, depth)
    else:
        k = autograd.MyrtleNNGP.apply(t1, t2, sw, sb, depth)
    rng = np.random.default_rng(3503)
    g = rng.standard_normal(tuple(k.shape)).astype(np.float32)
    (k * _gpu(g)).sum().backward()
    n1, n2 = k.shape
    a, b = np.meshgrid(np.arange(n1), np.arange(n2), indexing="ij")
    pairs = np.stack([a.ravel(), b.ravel()], 1)
    if mode == "distinct":
        r1, r2, rs, _ = ograd.myrtle_vjp(x1, x2, pairs, g.ravel().astype(np.float64), depth, 2.0, 0.03)
        assert _rel(t2.grad.cpu().numpy(), r2) <= GTOL
    elif mode == "distinct_x2_fixed":
        r1, _, rs, _ = ograd.myrtle_vjp(x1, x2, pairs, g.ravel().astype(np.float64), depth, 2.0, 0.03)
        assert t2.grad is None
    else:
        r1, _, rs, _ = ograd.myrtle_vjp(x1, None, pairs, g.ravel().astype(np.float64), depth, 2.0, 0.03)
        assert t2.grad is None
    e1 = _rel(t1.grad.cpu().numpy(), r1)
    es = np.abs(np.array([sw.grad.item(), sb.grad.item()]) - rs) / np.abs(rs)
    _say(f"  {mode}: rel err dx1 {e1:.2e} dsigma {es}")
    assert e1 <= GTOL and np.all(es <= GTOL)
    assert sw.grad.dtype == torch.float64 and sw.grad.device.type == "cpu"


@pytest.mark.parametrize("hw,ns,nt,keep", [(16, 24, 40, False), (32, 6, 10, False), (16, 24, 40, True),
                                           (32, 6, 10, True),
                                           # several passes of 16384 pairs in both blocks
                                           (16, 200, 300, False), (16, 200, 300, True)])
def test_krr_mse_grad_equals_its_parts(nk, hw, ns, nt, keep):
    """nk_krr_mse_grad (one call) against the same step assembled from the
    separate entry points (two blocks, ridge cotangents, two adjoints summed
    on the host): equal up to the float64 summation order of the per-image
    sums.  The one call runs the cross block's adjoint as (support, targets)
    with its cotangent read transposed and, at 32x32, without the targets'
    seed gradients; the parts run it as (targets, support) with all sums.
    keep: the call keeps the first-stage outputs from its forward pass (its
    cross block then runs forward as (support, targets) too, transposed into
    K_ts, so the parts take K_ts from that block)."""
    w = synth.WORKLOADS["myrtle5_krr_grad"]
    depth = w["depth"]
    xs = _gpu(synth.correlated_images(ns, hw, hw, 3, 2.0, 3601))
    xt = _gpu(synth.correlated_images(nt, hw, hw, 3, 2.0, 3602))
    ys = _gpu(synth.balanced_labels(ns, 10))
    yt = _gpu(synth.teacher_labels(xt.cpu().numpy(), 10, 3603))
    _say(f"krr_mse_grad at {hw}x{hw}, {ns} support, {nt} targets, kept checkpoints: {keep}")
    loss, dx, ds, lam = nk.krr_mse_grad(xs, ys, xt, yt, depth, 2.0, 0.01, 1e-3, keep_checkpoints=keep)
    kss = nk.myrtle_nngp(xs, None, depth, 2.0, 0.01).clone()
    if keep:
        kts = nk.myrtle_nngp(xs, xt, depth, 2.0, 0.01).t().contiguous()
    else:
        kts = nk.myrtle_nngp(xt, xs, depth, 2.0, 0.01).clone()
    dss, dts, loss2, lam2 = nk.krr_mse_backward(kss, kts, ys, yt, 1e-3, relative=True)
    d1, _, s1 = nk.myrtle_nngp_backward(xs, None, dss, depth, 2.0, 0.01)
    d1, s1 = d1.clone(), s1.clone()
    _, d2, s2 = nk.myrtle_nngp_backward(xt, xs, dts, depth, 2.0, 0.01)
    ref_dx = (d1.double() + d2.double()).cpu().numpy()
    ref_ds = (s1.double() + s2.double()).cpu().numpy()
    assert loss == loss2 and lam == lam2
    # the one call sums the two blocks' contributions in float64 and rounds
    # once; the parts are each rounded to float32 first, and they partly
    # cancel, so the difference is measured against the larger part.  The
    # sigma sums also differ by the order of their float32 per-tile partial
    # sums (the one call runs the cross block in the other orientation), and
    # they add terms of both signs over every entry of every pair: at 80,000
    # pairs that reaches about 1.3e-6 of the larger part, hence 5e-6 there
    # (half the bar against the float64 oracle).
    scale = max(float(d1.abs().max()), float(d2.abs().max()))
    e = float(np.max(np.abs(dx.cpu().numpy() - ref_dx))) / scale
    sscale = np.maximum(np.abs(s1.double().cpu().numpy()), np.abs(s2.double().cpu().numpy()))
    es = np.abs(ds.cpu().numpy() - ref_ds) / sscale
    _say(f"  one call vs parts: dx {e:.2e} dsigma {es} (relative to the larger part)")
    assert e <= 1e-6 and np.all(es <= 5e-6)
