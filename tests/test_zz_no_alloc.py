"""The allocation-free FC NNGP entry point (nk_fc_nngp_static) against the
workspace entry point (nk_fc_nngp), called through the C ABI: two calls in a
row on the same device, the second with a smaller input, each bitwise equal
to nk_fc_nngp on the same inputs (same kernels, same arithmetic) and within
the parity bar of the float64 oracle; sizes beyond the static scratch are
rejected."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2303_05420_amd import _lib
    return _lib


def _call_static(_lib, a, b, out, cfg):
    stream = torch.cuda.current_stream().cuda_stream
    return _lib.lib().nk_fc_nngp_static(a.data_ptr(), a.shape[0], b.data_ptr(), b.shape[0], ctypes.byref(cfg),
                                        out.data_ptr(), out.stride(0), stream)


def _call_ws(_lib, a, b, out, cfg):
    need = _lib.lib().nk_workspace_size(_lib.NK_OP_FC, ctypes.byref(cfg), a.shape[0], b.shape[0])
    ws = torch.empty(int(need), dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    return _lib.lib().nk_fc_nngp(a.data_ptr(), a.shape[0], b.data_ptr(), b.shape[0], ctypes.byref(cfg),
                                 out.data_ptr(), out.stride(0), ws.data_ptr(), ws.numel(), stream)


def test_static_entry_point_matches_workspace_entry_point(lib):
    w = synth.WORKLOADS["fc3_myrtle5_32x32_1024"]
    cfg = lib.FcCfg(3072, 3, 2.0, 0.01)
    xa = synth.correlated_images(700, 32, 32, 3, 3.0, w["seeds"][0]).reshape(700, -1)
    xb = synth.correlated_images(900, 32, 32, 3, 3.0, w["seeds"][1]).reshape(900, -1)
    for n1, n2 in ((700, 900), (37, 5)):  # second call smaller: stale scratch must not leak in
        a = torch.from_numpy(np.ascontiguousarray(xa[:n1])).cuda()
        b = torch.from_numpy(np.ascontiguousarray(xb[:n2])).cuda()
        k_static = torch.full((n1, n2 + 3), float("nan"), device="cuda")
        k_ws = torch.full((n1, n2 + 3), float("nan"), device="cuda")
        print(f"fc static {n1} x {n2}", flush=True)
        assert _call_static(lib, a, b, k_static, cfg) == 0, lib.lib().nk_last_error()
        assert _call_ws(lib, a, b, k_ws, cfg) == 0, lib.lib().nk_last_error()
        torch.cuda.synchronize()
        assert torch.equal(k_static[:, :n2], k_ws[:, :n2])
        assert torch.isnan(k_static[:, n2:]).all()
        ref = oracle.fc_nngp(xa[:n1], xb[:n2], 3, 2.0, 0.01)
        d1 = np.diag(oracle.fc_nngp(xa[:n1], xa[:n1], 3, 2.0, 0.01))
        d2 = np.diag(oracle.fc_nngp(xb[:n2], xb[:n2], 3, 2.0, 0.01))
        err = float(np.max(np.abs(k_static[:, :n2].cpu().numpy() - ref) / np.sqrt(np.outer(d1, d2))))
        print(f"  normalised error vs oracle {err:.2e}", flush=True)
        assert err <= 2e-5


def test_static_entry_point_rejects_oversize(lib):
    cfg = lib.FcCfg(4, 3, 2.0, 0.01)
    big = (1 << 21) // 2 + 1
    a = torch.zeros((big, 4), dtype=torch.float32, device="cuda")
    out = torch.empty((1, 1), dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    rc = lib.lib().nk_fc_nngp_static(a.data_ptr(), big, a.data_ptr(), big, ctypes.byref(cfg), out.data_ptr(),
                                     big, stream)
    assert rc == lib.NK_EINVAL
    assert b"static scratch" in lib.lib().nk_last_error()
