"""Pins of the float64 gradient oracle (oracle.grad): finite differences,
the sigma_w^2 power law, Euler's theorem for homogeneous functions, and the
closed-form partials of the ReLU map.  CPU only."""
import math

import numpy as np
import pytest
import torch

import oracle
import synth
from oracle import grad as ograd

torch.set_num_threads(8)


def _F(s, q1, q2):
    return oracle.relu_map(s, q1, q2)


@pytest.mark.parametrize("s,q1,q2", [(0.3, 1.0, 2.0), (-0.6, 1.4, 0.9), (0.95, 1.0, 1.1)])
def test_relu_partials_closed_form_vs_fd(s, q1, q2):
    h = 1e-6
    th = math.acos(s / math.sqrt(q1 * q2))
    ds = (math.pi - th) / (2 * math.pi)
    dq1 = math.sin(th) * math.sqrt(q2 / q1) / (4 * math.pi)
    dq2 = math.sin(th) * math.sqrt(q1 / q2) / (4 * math.pi)
    fd_s = (_F(s + h, q1, q2) - _F(s - h, q1, q2)) / (2 * h)
    fd_1 = (_F(s, q1 + h, q2) - _F(s, q1 - h, q2)) / (2 * h)
    fd_2 = (_F(s, q1, q2 + h) - _F(s, q1, q2 - h)) / (2 * h)
    assert abs(fd_s - ds) < 1e-8 and abs(fd_1 - dq1) < 1e-8 and abs(fd_2 - dq2) < 1e-8
    # and the autograd function uses exactly these partials
    ts = torch.tensor(s, dtype=torch.float64, requires_grad=True)
    t1 = torch.tensor(q1, dtype=torch.float64, requires_grad=True)
    t2 = torch.tensor(q2, dtype=torch.float64, requires_grad=True)
    ograd.relu_map(ts, t1, t2).backward()
    assert abs(ts.grad.item() - ds) < 1e-14 and abs(t1.grad.item() - dq1) < 1e-14
    assert abs(t2.grad.item() - dq2) < 1e-14


def test_torch_forward_equals_c_oracle():
    x = synth.correlated_images(4, 8, 8, 3, 3.0, 81)
    for depth, sb2 in [((2, 1, 1), 0.0), ((1, 2, 1), 0.03)]:
        net = oracle.Myrtle(depth, 2.0, sb2)
        K = oracle.myrtle_gram(x, None, net)
        t = torch.tensor(x.astype(np.float64))
        kt = ograd.myrtle_pair_kernel(t[[0, 1, 2, 3, 0]], t[[1, 2, 3, 0, 0]], depth,
                                      torch.tensor(2.0, dtype=torch.float64), torch.tensor(sb2, dtype=torch.float64))
        ref = np.array([K[0, 1], K[1, 2], K[2, 3], K[3, 0], K[0, 0]])
        assert np.max(np.abs(kt.detach().numpy() - ref)) <= 1e-13 * ref.max()


def _kfun(x1, x2, depth, sw2, sb2):
    t1 = torch.tensor(x1[None].astype(np.float64))
    t2 = torch.tensor(x2[None].astype(np.float64))
    return ograd.myrtle_pair_kernel(t1, t2, depth, torch.tensor(sw2, dtype=torch.float64),
                                    torch.tensor(sb2, dtype=torch.float64)).item()


@pytest.mark.parametrize("sb2", [0.0, 0.05])
def test_vjp_matches_central_differences(sb2):
    x = synth.correlated_images(2, 8, 8, 3, 3.0, 91).astype(np.float64)
    depth = (2, 1, 1)
    dx1, dx2, ds, k = ograd.myrtle_vjp(x[:1], x[1:], np.array([[0, 0]]), np.array([1.0]), depth, 2.0, sb2)
    rng = np.random.default_rng(0)
    h = 1e-5
    for _ in range(6):
        y, xx, c = rng.integers(0, 8), rng.integers(0, 8), rng.integers(0, 3)
        for which, g in ((0, dx1), (1, dx2)):
            xp = x.copy()
            xm = x.copy()
            xp[which, y, xx, c] += h
            xm[which, y, xx, c] -= h
            fd = (_kfun(xp[0], xp[1], depth, 2.0, sb2) - _kfun(xm[0], xm[1], depth, 2.0, sb2)) / (2 * h)
            assert abs(fd - g[0, y, xx, c]) <= 1e-7 * max(1.0, np.abs(g).max())
    fdw = (_kfun(x[0], x[1], depth, 2.0 + h, sb2) - _kfun(x[0], x[1], depth, 2.0 - h, sb2)) / (2 * h)
    fdb = (_kfun(x[0], x[1], depth, 2.0, sb2 + h) - _kfun(x[0], x[1], depth, 2.0, sb2 - h)) / (2 * h)
    assert abs(fdw - ds[0]) <= 1e-8 * abs(ds[0])
    assert abs(fdb - ds[1]) <= 1e-7 * max(1.0, abs(ds[1]))


def test_vjp_sigma_law_and_euler():
    """sb2 = 0: dK/dsw2 = n_aff K / sw2; K is 1-homogeneous in each argument,
    so sum_p x_p dK/dx_p = K (cross entry) and 2 K (self entry)."""
    x = synth.correlated_images(3, 8, 8, 3, 3.0, 101).astype(np.float64)
    depth = (2, 1, 1)
    n_aff = sum(depth) + 1
    dx1, dx2, ds, k = ograd.myrtle_vjp(x[:1], x[1:2], np.array([[0, 0]]), np.array([1.0]), depth, 2.0, 0.0)
    assert abs(ds[0] - n_aff * k[0] / 2.0) <= 1e-13 * abs(ds[0])
    assert abs((dx1 * x[:1]).sum() - k[0]) <= 1e-12 * k[0]
    assert abs((dx2 * x[1:2]).sum() - k[0]) <= 1e-12 * k[0]
    dxs, _, _, ks = ograd.myrtle_vjp(x[2:3], None, np.array([[0, 0]]), np.array([1.0]), depth, 2.0, 0.0)
    assert abs((dxs * x[2:3]).sum() - 2 * ks[0]) <= 1e-12 * ks[0]
