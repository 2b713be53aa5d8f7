"""Kernel ridge regression of learnable support images onto target images
through the Myrtle-5 NNGP: GPU cotangents of the ridge solve, end-to-end
gradients against central finite differences of the FP64 oracle loss, and
the full-size (256 support, 2048 targets, 32x32x3) kernel VJP on sparse
cotangents against the FP64 autograd oracle."""
import numpy as np
import pytest
import torch

import oracle
import synth
from oracle import grad as ograd

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nk():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2303_05420_amd import krr_grad, ops
    return ops, krr_grad


def _gpu(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()


def test_krr_mse_backward_matches_oracle(nk):
    ops, _ = nk
    rng = np.random.default_rng(21)
    n, m, c = 40, 70, 10
    a = rng.standard_normal((n, n + 8))
    kss = (a @ a.T / (n + 8)).astype(np.float32)
    kts = rng.standard_normal((m, n)).astype(np.float32)
    ys = synth.balanced_labels(n, c)
    yt = rng.standard_normal((m, c)).astype(np.float32)
    dss, dts, loss, lam = ops.krr_mse_backward(_gpu(kss), _gpu(kts), _gpu(ys), _gpu(yt), 1e-2, relative=True)
    lam_ref = 1e-2 * np.mean(np.diag(kss.astype(np.float64)))
    assert abs(lam - lam_ref) <= 1e-12 * lam_ref
    rss, rts = oracle.krr_mse_cotangents(kss, kts, ys, yt, lam_ref)
    assert abs(loss - oracle.krr_mse_loss(kss, kts, ys, yt, lam_ref)) <= 1e-10 * loss
    assert np.max(np.abs(dss.cpu().numpy() - rss)) <= 1e-5 * np.abs(rss).max()
    assert np.max(np.abs(dts.cpu().numpy() - rts)) <= 1e-5 * np.abs(rts).max()


def _oracle_loss(xs, ys, xt, yt, depth, sw2, sb2, lam):
    net = oracle.Myrtle(depth, sw2, sb2)
    kss = oracle.myrtle_gram(xs, None, net)
    kts = oracle.myrtle_gram(xt, xs, net)
    return oracle.krr_mse_loss(kss, kts, ys, yt, lam)


@pytest.mark.parametrize("ns,nt,hw,sb2,npix", [(16, 48, 8, 0.0, 8), (12, 30, 8, 0.01, 6), (3, 6, 32, 0.0, 0)])
def test_end_to_end_gradient_matches_finite_differences(nk, ns, nt, hw, sb2, npix):
    _, krr_grad = nk
    w = synth.WORKLOADS["myrtle5_krr_grad"]
    depth = w["depth"]
    xs = synth.correlated_images(ns, hw, hw, 3, w["length"], w["seeds"][0]).astype(np.float64)
    xt = synth.correlated_images(nt, hw, hw, 3, w["length"], w["seeds"][1])
    ys = synth.balanced_labels(ns, 10)
    yt = synth.teacher_labels(xt, 10, w["seeds"][2])
    print(f"end-to-end {ns} support {nt} targets at {hw}", flush=True)
    loss, dxs, ds, lam = krr_grad.krr_mse_loss_and_grad(_gpu(xs), _gpu(ys), _gpu(xt), _gpu(yt), depth,
                                                        w["sigma_w2"], sb2, w["ridge_rel"])
    dxs = dxs.cpu().numpy().astype(np.float64)
    ds = ds.cpu().numpy().astype(np.float64)
    h = w["fd_h"]          # pixel step
    hs = 1e-4              # sigma step (sigma_b2 may be as small as 0.01)
    base = _oracle_loss(xs.astype(np.float32), ys, xt, yt, depth, w["sigma_w2"], sb2, lam)
    assert abs(loss - base) <= 1e-4 * base
    fds, gs = [], []
    fw = (_oracle_loss(xs.astype(np.float32), ys, xt, yt, depth, w["sigma_w2"] + hs, sb2, lam)
          - _oracle_loss(xs.astype(np.float32), ys, xt, yt, depth, w["sigma_w2"] - hs, sb2, lam)) / (2 * hs)
    if sb2 >= hs:
        fb = (_oracle_loss(xs.astype(np.float32), ys, xt, yt, depth, w["sigma_w2"], sb2 + hs, lam)
              - _oracle_loss(xs.astype(np.float32), ys, xt, yt, depth, w["sigma_w2"], sb2 - hs, lam)) / (2 * hs)
    else:
        # sigma_b2 cannot go below 0: second-order one-sided difference.  At
        # sigma_b2 = 0 the loss has large higher derivatives in sigma_b2 (the
        # one-sided estimate moves by 1e-2 between steps 1e-4 and 1e-5), so the
        # step is much smaller here; the loss is float64, so 1e-6 is still
        # far above its rounding noise.
        h1 = 1e-6
        f0, f1, f2 = (_oracle_loss(xs.astype(np.float32), ys, xt, yt, depth, w["sigma_w2"], sb2 + k * h1, lam)
                      for k in (0, 1, 2))
        fb = (-3 * f0 + 4 * f1 - f2) / (2 * h1)
    fds += [fw, fb]
    gs += [ds[0], ds[1]]
    rng = np.random.default_rng(w["seeds"][3])
    for _ in range(npix):
        idx = tuple(int(rng.integers(0, s)) for s in xs.shape)
        xp = xs.copy(); xp[idx] += h
        xm = xs.copy(); xm[idx] -= h
        fd = (_oracle_loss(xp.astype(np.float32), ys, xt, yt, depth, w["sigma_w2"], sb2, lam)
              - _oracle_loss(xm.astype(np.float32), ys, xt, yt, depth, w["sigma_w2"], sb2, lam)) / (2 * h)
        fds.append(fd)
        gs.append(dxs[idx])
    # one random direction through all support pixels
    u = rng.standard_normal(xs.shape)
    u /= np.linalg.norm(u)
    fdu = (_oracle_loss((xs + h * u).astype(np.float32), ys, xt, yt, depth, w["sigma_w2"], sb2, lam)
           - _oracle_loss((xs - h * u).astype(np.float32), ys, xt, yt, depth, w["sigma_w2"], sb2, lam)) / (2 * h)
    fds.append(fdu)
    gs.append(float((dxs * u).sum()))
    fds, gs = np.array(fds), np.array(gs)
    err = np.max(np.abs(fds - gs)) / np.max(np.abs(fds))
    print(f"  fd {fds}\n  gpu {gs}\n  rel err {err:.2e}", flush=True)
    assert err <= 1e-3


def test_full_size_kernel_vjp_sparse_cotangent(nk):
    """256 support x 2048 targets at 32x32x3 (the full workload): the GPU
    adjoint of the full K_ts and K_ss blocks with cotangents nonzero on 24 + 8
    seeded entries, against the oracle's summed per-pair VJPs."""
    ops, _ = nk
    w = synth.WORKLOADS["myrtle5_krr_grad"]
    depth = w["depth"]
    xs = synth.correlated_images(w["n_support"], 32, 32, 3, w["length"], w["seeds"][0])
    xt = synth.correlated_images(w["n_target"], 32, 32, 3, w["length"], w["seeds"][1])
    rng = np.random.default_rng(w["seeds"][3])
    pts = np.stack([rng.integers(0, w["n_target"], 24), rng.integers(0, w["n_support"], 24)], 1)
    pss = np.stack([rng.integers(0, w["n_support"], 8), rng.integers(0, w["n_support"], 8)], 1)
    gts = rng.standard_normal(24)
    gss = rng.standard_normal(8)
    dts = np.zeros((w["n_target"], w["n_support"]), np.float32)
    dss = np.zeros((w["n_support"], w["n_support"]), np.float32)
    for (a, b), g in zip(pts, gts):
        dts[a, b] += g
    for (a, b), g in zip(pss, gss):
        dss[a, b] += g
    print("full-size sparse VJP on GPU", flush=True)
    _, dxs_ts, ds_ts = ops.myrtle_nngp_backward(_gpu(xt), _gpu(xs), _gpu(dts), depth, w["sigma_w2"], w["sigma_b2"])
    dxs_ts = dxs_ts.cpu().numpy()
    ds_ts = ds_ts.cpu().numpy()
    dxs_ss, _, ds_ss = ops.myrtle_nngp_backward(_gpu(xs), None, _gpu(dss), depth, w["sigma_w2"], w["sigma_b2"])
    g_gpu = dxs_ts.astype(np.float64) + dxs_ss.cpu().numpy()
    s_gpu = ds_ts.astype(np.float64) + ds_ss.cpu().numpy()
    print("oracle VJPs", flush=True)
    _, r2, rs1, _ = ograd.myrtle_vjp(xt, xs, pts, gts, depth, w["sigma_w2"], w["sigma_b2"])
    r3, _, rs2, _ = ograd.myrtle_vjp(xs, None, pss, gss, depth, w["sigma_w2"], w["sigma_b2"])
    g_ref = r2 + r3
    s_ref = rs1 + rs2
    err = np.max(np.abs(g_gpu - g_ref)) / np.max(np.abs(g_ref))
    es = np.abs(s_gpu - s_ref) / np.abs(s_ref)
    print(f"  rel err dx {err:.2e} dsigma {es}", flush=True)
    assert err <= 1e-5 and np.all(es <= 1e-5)
