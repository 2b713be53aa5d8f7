"""GPU parity of the FC NNGP (MFMA first layer) and of float64 kernel ridge
regression against the oracle."""
import sys

import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nk():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2303_05420_amd import ops
    return ops


def _gpu(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


@pytest.mark.parametrize("n1,n2,hw", [(1024, 1024, 32), (37, 51, 8), (1, 3, 5), (300, 260, 7), (1100, 700, 16)])
def test_fc3_matches_oracle(nk, n1, n2, hw):
    w = synth.WORKLOADS["fc3_myrtle5_32x32_1024"]
    x1 = synth.correlated_images(n1, hw, hw, 3, 3.0, w["seeds"][0])
    x2 = synth.correlated_images(n2, hw, hw, 3, 3.0, w["seeds"][1])
    print(f"fc3 {n1} x {n2} at {hw}x{hw}", flush=True)
    kg = nk.fc_nngp(_gpu(x1), _gpu(x2), 3, 2.0, 0.01).cpu().numpy()
    kr = oracle.fc_nngp(x1, x2, 3, 2.0, 0.01)
    d1 = np.diag(oracle.fc_nngp(x1, x1, 3, 2.0, 0.01))
    d2 = np.diag(oracle.fc_nngp(x2, x2, 3, 2.0, 0.01))
    err = np.max(np.abs(kg - kr) / np.sqrt(np.outer(d1, d2)))
    print(f"  normalised error {err:.3e}", flush=True)
    assert err <= 2e-5


@pytest.mark.parametrize("n,hw,pad", [(1, 5, 0), (37, 7, 3), (300, 7, 0), (1100, 16, 5), (1024, 32, 0)])
def test_fc3_symmetric_block(nk, n, hw, pad):
    """A symmetric FC-3 block (x2 the same images): the tiles on and above the
    diagonal run and the others are their mirror, into a row stride padded
    by `pad` (unaligned rows take the scalar mirror stores); against the
    float64 oracle and symmetric within float32 rounding."""
    w = synth.WORKLOADS["fc3_myrtle5_32x32_1024"]
    x = synth.correlated_images(n, hw, hw, 3, 3.0, w["seeds"][0])
    print(f"fc3 symmetric {n} x {n} at {hw}x{hw}, ldk {n + pad}", flush=True)
    big = torch.full((n, n + pad), float("nan"), dtype=torch.float32, device="cuda")
    out = big[:, :n]
    nk.fc_nngp(_gpu(x), None, 3, 2.0, 0.01, out=out)
    torch.cuda.synchronize()
    kg = out.cpu().numpy()
    kr = oracle.fc_nngp(x, x, 3, 2.0, 0.01)
    d = np.sqrt(np.diag(kr))
    err = np.max(np.abs(kg - kr) / np.outer(d, d))
    asym = np.max(np.abs(kg - kg.T) / np.outer(d, d))
    print(f"  normalised error {err:.3e}, asymmetry {asym:.3e}", flush=True)
    assert err <= 2e-5 and asym <= 1e-6
    if pad:
        assert torch.isnan(big[:, n:]).all()  # nothing written past the block


def test_krr_predict_matches_oracle(nk):
    w = synth.WORKLOADS["fc3_myrtle5_32x32_1024"]
    x1 = synth.correlated_images(1024, 32, 32, 3, 3.0, w["seeds"][0])
    x2 = synth.correlated_images(1024, 32, 32, 3, 3.0, w["seeds"][1])
    y = synth.teacher_labels(x1, 10, w["seeds"][2])
    g1, g2 = _gpu(x1), _gpu(x2)
    ktr = nk.fc_nngp(g1, None, 3, 2.0, 0.01)
    kte = nk.fc_nngp(g2, g1, 3, 2.0, 0.01)
    print("krr 1024 train, 1024 test", flush=True)
    pred = nk.krr_predict(ktr, kte, _gpu(y), w["ridge_rel"]).cpu().numpy()
    ref = oracle.krr_predict(ktr.cpu().numpy(), kte.cpu().numpy(), y, w["ridge_rel"])
    rel = np.max(np.abs(pred - ref)) / np.max(np.abs(ref))
    print(f"  max rel error {rel:.3e}", flush=True)
    assert rel <= 1e-5


def test_krr_small_and_not_pd(nk):
    from paper_2303_05420_amd import _lib
    rng = np.random.default_rng(9)
    for n, m, c in [(1, 1, 1), (70, 5, 3), (130, 9, 10)]:
        a = rng.standard_normal((n, n + 5))
        K = (a @ a.T / (n + 5)).astype(np.float32)
        Kt = rng.standard_normal((m, n)).astype(np.float32)
        y = rng.standard_normal((n, c)).astype(np.float32)
        pred = nk.krr_predict(_gpu(K), _gpu(Kt), _gpu(y), 1e-3).cpu().numpy()
        ref = oracle.krr_predict(K, Kt, y, 1e-3)
        assert np.max(np.abs(pred - ref)) <= 1e-5 * max(1.0, np.abs(ref).max())
    K = -np.eye(8, dtype=np.float32)
    with pytest.raises(_lib.NKError) as e:
        nk.krr_predict(_gpu(K), _gpu(K), _gpu(np.ones((8, 1), np.float32)), 0.0)
    assert e.value.code == _lib.NK_ENOTPD
