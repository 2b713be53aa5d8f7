"""GPU adjoint of the Myrtle NNGP against the float64 autograd oracle
(oracle.grad): kernel-level vector-Jacobian products, relative max error
<= 1e-5 per output (dx1, dx2, dsigma_w2, dsigma_b2)."""
import numpy as np
import pytest
import torch

import synth
from oracle import grad as ograd

pytestmark = pytest.mark.gpu

TOL = 1e-5


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


@pytest.mark.parametrize("n1,n2,hw,depth,sb2", [
    (4, 3, 8, (2, 1, 1), 0.0),
    (3, 5, 8, (1, 2, 1), 0.05),
    (3, 2, 16, (2, 1, 1), 0.0),
    (2, 2, 32, (2, 1, 1), 0.0),
    (2, 3, 8, (2, 1, 1), 0.05),   # pair slots past the chunk end share waves with live ones
    (1, 1, 4, (1,), 0.1),
    (3, 2, 8, (2, 0, 1), 0.0),
])
def test_vjp_block(nk, n1, n2, hw, depth, sb2):
    x1 = synth.correlated_images(n1, hw, hw, 3, 3.0, 700 + n1)
    x2 = synth.correlated_images(n2, hw, hw, 3, 3.0, 800 + n2)
    rng = np.random.default_rng(5)
    gk = rng.standard_normal((n1, n2)).astype(np.float32)
    print(f"vjp block {n1}x{n2} at {hw} depth {depth} sb2 {sb2}", flush=True)
    dx1, dx2, ds = nk.myrtle_nngp_backward(_gpu(x1), _gpu(x2), _gpu(gk), depth, 2.0, sb2)
    torch.cuda.synchronize()
    a, b = np.meshgrid(np.arange(n1), np.arange(n2), indexing="ij")
    pairs = np.stack([a.ravel(), b.ravel()], 1)
    r1, r2, rs, _ = ograd.myrtle_vjp(x1, x2, pairs, gk.ravel().astype(np.float64), depth, 2.0, sb2)
    e1 = _rel(dx1.cpu().numpy(), r1)
    e2 = _rel(dx2.cpu().numpy(), r2)
    es = np.abs(ds.cpu().numpy() - rs) / np.maximum(np.abs(rs), 1e-30)
    print(f"  rel err dx1 {e1:.2e} dx2 {e2:.2e} dsw2 {es[0]:.2e} dsb2 {es[1]:.2e}  ref dsigma {rs}", flush=True)
    assert e1 <= TOL and e2 <= TOL
    assert es[0] <= TOL and es[1] <= TOL


@pytest.mark.parametrize("depth,C,need_dx2,sb2", [
    ((1, 1, 1), 1, True, 0.02),    # 512-thread workgroup, j-side seed sums kept
    ((1, 1, 1), 3, False, 0.02),   # 512 threads
    ((2, 1, 1), 1, True, 0.02),    # 512 threads
    ((2, 1, 1), 2, False, 0.02),   # 512 threads
    ((3, 1, 1), 1, False, 0.02),   # 512 threads
    ((3, 1, 1), 3, False, 0.02),   # 256 threads (registers above 256)
    ((2, 1, 1), 3, True, 0.02),    # 256 threads
    ((2, 1, 1), 3, False, 0.0),    # 512 threads, the sigma_b2 = 0 variant (the ridge gradient's cross block)
    ((1, 1, 1), 2, True, 0.0),     # 512 threads, sigma_b2 = 0
])
def test_vjp_32x32_workgroup_shapes(nk, depth, C, need_dx2, sb2):
    """First-stage adjoints at 32x32 in both workgroup shapes (eight
    four-column segments per pair where the registers fit two waves per SIMD,
    else four of eight), over channel counts, depths and both bias variants,
    against the float64 autograd oracle."""
    x1 = synth.correlated_images(2, 32, 32, C, 3.0, 1100 + C)
    x2 = synth.correlated_images(2, 32, 32, C, 3.0, 1200 + C)
    gk = np.random.default_rng(7).standard_normal((2, 2)).astype(np.float32)
    print(f"vjp 2x2 at 32x32 depth {depth} C {C} dx2 {need_dx2} sb2 {sb2}", flush=True)
    dx1, dx2, ds = nk.myrtle_nngp_backward(_gpu(x1), _gpu(x2), _gpu(gk), depth, 2.0, sb2, need_dx2=need_dx2)
    torch.cuda.synchronize()
    pairs = np.array([[0, 0], [0, 1], [1, 0], [1, 1]])
    r1, r2, rs, _ = ograd.myrtle_vjp(x1, x2, pairs, gk.ravel().astype(np.float64), depth, 2.0, sb2)
    e1 = _rel(dx1.cpu().numpy(), r1)
    e2 = _rel(dx2.cpu().numpy(), r2) if need_dx2 else 0.0
    es = np.abs(ds.cpu().numpy() - rs) / np.maximum(np.abs(rs), 1e-30)
    print(f"  rel err dx1 {e1:.2e} dx2 {e2:.2e} dsigma {es}", flush=True)
    assert (dx2 is not None) == need_dx2
    assert e1 <= TOL and e2 <= TOL and np.all(es <= TOL)


@pytest.mark.parametrize("C,sb2", [(2, 0.0), (1, 0.02)])
def test_vjp_symmetric_32x32_two_waves(nk, C, sb2):
    """A symmetric 32x32 block (x2 None: self pairs included, their
    displacement-0 tile at rho = 1 exactly) through a first-stage adjoint that
    keeps the second image's seed sums and still fits two waves per SIMD
    (depth 1, one or two channels), cotangent on every entry including the
    diagonal, against the float64 autograd oracle."""
    x = synth.correlated_images(3, 32, 32, C, 3.0, 1300 + C)
    gk = np.random.default_rng(8).standard_normal((3, 3)).astype(np.float32) + 2 * np.eye(3, dtype=np.float32)
    depth = (1, 1, 1)
    print(f"vjp symmetric 3x3 at 32x32 C {C} sb2 {sb2}", flush=True)
    dx, dx2, ds = nk.myrtle_nngp_backward(_gpu(x), None, _gpu(gk), depth, 2.0, sb2)
    torch.cuda.synchronize()
    assert dx2 is None
    a, b = np.meshgrid(np.arange(3), np.arange(3), indexing="ij")
    pairs = np.stack([a.ravel(), b.ravel()], 1)
    r, _, rs, _ = ograd.myrtle_vjp(x, None, pairs, gk.ravel().astype(np.float64), depth, 2.0, sb2)
    e = _rel(dx.cpu().numpy(), r)
    es = np.abs(ds.cpu().numpy() - rs) / np.maximum(np.abs(rs), 1e-30)
    print(f"  sym rel err dx {e:.2e} dsigma {es}", flush=True)
    assert e <= TOL and np.all(es <= TOL)


def test_vjp_symmetric(nk):
    x = synth.correlated_images(4, 8, 8, 3, 3.0, 901)
    rng = np.random.default_rng(6)
    gk = rng.standard_normal((4, 4)).astype(np.float32)
    depth = (2, 1, 1)
    dx, dx2, ds = nk.myrtle_nngp_backward(_gpu(x), None, _gpu(gk), depth, 2.0, 0.02)
    assert dx2 is None
    a, b = np.meshgrid(np.arange(4), np.arange(4), indexing="ij")
    pairs = np.stack([a.ravel(), b.ravel()], 1)
    r, _, rs, _ = ograd.myrtle_vjp(x, None, pairs, gk.ravel().astype(np.float64), depth, 2.0, 0.02)
    e = _rel(dx.cpu().numpy(), r)
    es = np.abs(ds.cpu().numpy() - rs) / np.abs(rs)
    print(f"  sym rel err dx {e:.2e} dsigma {es}", flush=True)
    assert e <= TOL and np.all(es <= TOL)
