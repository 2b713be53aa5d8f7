"""The C ABI library loads and exports every function include/nk.h declares;
argument validation returns the documented codes without touching the GPU."""
import ctypes

import pytest

from paper_2303_05420_amd import _lib


def test_library_exports_header_functions():
    L = _lib.lib()
    names = _lib.header_functions()
    assert "nk_myrtle_nngp" in names and "nk_fc_nngp" in names and "nk_krr_predict" in names
    assert "nk_myrtle_nngp_backward" in names
    for n in names:
        assert hasattr(L, n), n
    assert L.nk_version().decode().startswith("libnk")


def _cfg(**kw):
    d = dict(hw=8, c=3, depth=(2, 1, 1), sigma_w2=2.0, sigma_b2=0.0)
    d.update(kw)
    return _lib.myrtle_cfg(**d)


def test_workspace_size_queries():
    L = _lib.lib()
    cfg = _cfg()
    a = L.nk_workspace_size(_lib.NK_OP_MYRTLE, ctypes.byref(cfg), 16, 16)
    b = L.nk_workspace_size(_lib.NK_OP_MYRTLE, ctypes.byref(cfg), 64, 64)
    assert 0 < a < b
    bad = _cfg(hw=12)
    assert L.nk_workspace_size(_lib.NK_OP_MYRTLE, ctypes.byref(bad), 16, 16) == 0
    assert L.nk_workspace_size(_lib.NK_OP_KRR, None, 100, 10) >= 100 * 100 * 8
    assert L.nk_workspace_size(_lib.NK_OP_FC, None, 10, 10) > 0
    assert L.nk_workspace_size(99, None, 10, 10) == 0


def test_krr_grad_keep_workspace():
    """The workspace that keeps the first-stage outputs between the passes
    holds (n (n + 1) / 2 + n m) (H/2)^4 floats for them in place of one chunk
    buffer of that stage (all within the 256-byte alignment of each region);
    a one-stage network has nothing to keep."""
    L = _lib.lib()
    for hw, n, m in ((32, 256, 2048), (16, 24, 40), (8, 5, 7)):
        cfg = _cfg(hw=hw)
        base = L.nk_krr_mse_grad_workspace(ctypes.byref(cfg), n, m, 10)
        keep = L.nk_krr_mse_grad_workspace_keep(ctypes.byref(cfg), n, m, 10)
        q4 = (hw // 2) ** 4
        pairs = n * (n + 1) // 2 + n * m
        chunk = min(max(n * (n + 1) // 2, n * m), 16384)
        expect = base + 4 * q4 * (pairs - chunk)
        assert abs(keep - expect) <= 512, (hw, keep, expect)
    # the kept variant refuses a workspace that only fits the default (no device work)
    cfg = _cfg(hw=16)
    base = L.nk_krr_mse_grad_workspace(ctypes.byref(cfg), 24, 40, 10)
    keep = L.nk_krr_mse_grad_workspace_keep(ctypes.byref(cfg), 24, 40, 10)
    p, q = ctypes.c_void_p(256), ctypes.c_void_p(512)
    loss = ctypes.c_double(0.0)
    assert L.nk_krr_mse_grad_kept(p, 24, q, 40, p, q, 10, ctypes.byref(cfg), 1e-3, 1, p, p, ctypes.byref(loss),
                                  None, p, keep - 1, None) == _lib.NK_EINVAL
    assert "keep" in L.nk_last_error().decode() and base < keep
    one = _cfg(hw=8, depth=(2,))
    assert (L.nk_krr_mse_grad_workspace_keep(ctypes.byref(one), 5, 7, 10)
            == L.nk_krr_mse_grad_workspace(ctypes.byref(one), 5, 7, 10) > 0)
    assert L.nk_krr_mse_grad_workspace_keep(ctypes.byref(_cfg(hw=12)), 5, 7, 10) == 0


@pytest.mark.parametrize("kw,code", [
    (dict(hw=12), _lib.NK_EUNSUPPORTED),           # not a power of two
    (dict(hw=128), _lib.NK_EUNSUPPORTED),          # above the supported sizes
    (dict(hw=64, depth=(3, 1, 1)), _lib.NK_EUNSUPPORTED),  # 64x64 first stage with 3 layers
    (dict(hw=64, depth=(2,)), _lib.NK_EUNSUPPORTED),  # 64x64 single stage (no pool)
    (dict(c=5), _lib.NK_EUNSUPPORTED),             # > 4 channels
    (dict(depth=(0, 1, 1)), _lib.NK_EUNSUPPORTED),  # first stage without a conv
    (dict(depth=(1, 1, 1, 1, 1)), None),           # too many stages (python side)
    (dict(sigma_w2=0.0), _lib.NK_EINVAL),
    (dict(sigma_b2=-1.0), _lib.NK_EINVAL),
    (dict(depth=(2, 5, 1)), _lib.NK_EUNSUPPORTED),
    (dict(hw=8, depth=(1, 1, 1, 1)), _lib.NK_EUNSUPPORTED),  # last stage 1 x 1
    (dict(hw=32, depth=(4, 1, 1)), _lib.NK_EUNSUPPORTED),  # first-stage tables + images exceed LDS
])
def test_myrtle_config_validation(kw, code):
    L = _lib.lib()
    if code is None:
        with pytest.raises(ValueError):
            _cfg(**kw)
        return
    cfg = _cfg(**kw)
    rc = L.nk_myrtle_nngp(ctypes.c_void_p(16), 4, ctypes.c_void_p(16), 4, ctypes.byref(cfg), ctypes.c_void_p(16), 4,
                          ctypes.c_void_p(16), 1 << 20, None)
    assert rc == code, L.nk_last_error()
    assert L.nk_last_error().decode() != ""


def test_depth4_first_stage_fits_below_32():
    L = _lib.lib()
    cfg = _cfg(hw=16, depth=(4, 1, 1))
    assert L.nk_workspace_size(_lib.NK_OP_MYRTLE, ctypes.byref(cfg), 8, 8) > 0
    cfg = _cfg(hw=32, depth=(3, 3, 3))
    assert L.nk_workspace_size(_lib.NK_OP_MYRTLE, ctypes.byref(cfg), 8, 8) > 0
    cfg = _cfg(hw=32, depth=(4, 1, 1))
    assert L.nk_workspace_size(_lib.NK_OP_MYRTLE, ctypes.byref(cfg), 8, 8) == 0


def test_64x64_only_for_the_nngp_block():
    """64x64 inputs: accepted by the NNGP block and its workspace query,
    refused by the tangent kernel, the adjoint and the batched pass."""
    L = _lib.lib()
    cfg = _cfg(hw=64, depth=(2, 2, 2))
    need = L.nk_workspace_size(_lib.NK_OP_MYRTLE, ctypes.byref(cfg), 256, 256)
    assert need > 1024 * (32 ** 4 + 16 ** 4) * 4  # 1024 pairs per pass: their pooled stage inputs
    assert L.nk_workspace_size(_lib.NK_OP_MYRTLE_NTK, ctypes.byref(cfg), 8, 8) == 0
    assert L.nk_workspace_size(_lib.NK_OP_MYRTLE_BWD, ctypes.byref(cfg), 8, 8) == 0
    p = ctypes.c_void_p(256)
    # a valid 64x64 call that stops at the workspace check (no device work)
    assert L.nk_myrtle_nngp(p, 4, p, 4, ctypes.byref(cfg), p, 4, p, 16, None) == _lib.NK_EINVAL
    assert "workspace" in L.nk_last_error().decode()
    assert L.nk_myrtle_ntk(p, 4, p, 4, ctypes.byref(cfg), p, p, 4, p, 1 << 30, None) == _lib.NK_EUNSUPPORTED
    assert L.nk_myrtle_nngp_backward(p, 4, p, 4, ctypes.byref(cfg), p, 4, p, p, p, p, 1 << 30,
                                     None) == _lib.NK_EUNSUPPORTED
    tiles = (_lib.Tile * 1)()
    tiles[0].x1 = tiles[0].x2 = tiles[0].K = 256
    tiles[0].n1, tiles[0].n2, tiles[0].ldk = 5, 7, 7
    assert L.nk_myrtle_nngp_batched_workspace(tiles, 1, ctypes.byref(cfg)) == 0
    assert L.nk_myrtle_nngp_batched(tiles, 1, ctypes.byref(cfg), p, 1 << 30, None, 0) == _lib.NK_EUNSUPPORTED


def test_myrtle_argument_validation():
    L = _lib.lib()
    cfg = _cfg()
    p = ctypes.c_void_p(256)
    # null image / output
    assert L.nk_myrtle_nngp(None, 4, p, 4, ctypes.byref(cfg), p, 4, p, 1 << 30, None) == _lib.NK_EINVAL
    assert L.nk_myrtle_nngp(p, 4, p, 4, ctypes.byref(cfg), None, 4, p, 1 << 30, None) == _lib.NK_EINVAL
    # sizes
    assert L.nk_myrtle_nngp(p, 0, p, 4, ctypes.byref(cfg), p, 4, p, 1 << 30, None) == _lib.NK_EINVAL
    assert L.nk_myrtle_nngp(p, 4, p, 4, ctypes.byref(cfg), p, 3, p, 1 << 30, None) == _lib.NK_EINVAL  # ldk < n2
    # workspace too small
    assert L.nk_myrtle_nngp(p, 4, p, 4, ctypes.byref(cfg), p, 4, p, 16, None) == _lib.NK_EINVAL
    assert "workspace" in L.nk_last_error().decode()
    assert L.nk_myrtle_nngp(p, 4, p, 4, None, p, 4, p, 1 << 30, None) == _lib.NK_EINVAL


def test_fc_and_krr_validation():
    L = _lib.lib()
    p = ctypes.c_void_p(256)
    fc = _lib.FcCfg(3072, 3, 2.0, 0.01)
    assert L.nk_fc_nngp(p, 4, p, 4, ctypes.byref(fc), p, 3, p, 1 << 20, None) == _lib.NK_EINVAL
    bad = _lib.FcCfg(0, 3, 2.0, 0.01)
    assert L.nk_fc_nngp(p, 4, p, 4, ctypes.byref(bad), p, 4, p, 1 << 20, None) == _lib.NK_EINVAL
    assert L.nk_krr_predict(p, 0, p, 4, p, 10, 1e-4, p, p, 1 << 30, None) == _lib.NK_EINVAL
    assert L.nk_krr_predict(p, 10, p, 4, p, 10, -1.0, p, p, 1 << 30, None) == _lib.NK_EINVAL
    assert L.nk_krr_predict(p, 10, p, 4, p, 10, 1e-4, p, p, 64, None) == _lib.NK_EINVAL


def test_batched_validation():
    L = _lib.lib()
    cfg = _cfg()
    p = ctypes.c_void_p(256)
    tiles = (_lib.Tile * 2)()
    for t in tiles:
        t.x1 = t.x2 = t.K = 256
        t.n1, t.n2, t.ldk = 5, 7, 7
    need = L.nk_myrtle_nngp_batched_workspace(tiles, 2, ctypes.byref(cfg))
    assert need > 0
    assert L.nk_myrtle_nngp_batched_workspace(tiles, 0, ctypes.byref(cfg)) == 0
    assert L.nk_myrtle_nngp_batched(None, 2, ctypes.byref(cfg), p, need, None, 0) == _lib.NK_EINVAL
    assert L.nk_myrtle_nngp_batched(tiles, 0, ctypes.byref(cfg), p, need, None, 0) == _lib.NK_EINVAL
    assert L.nk_myrtle_nngp_batched(tiles, 2, ctypes.byref(cfg), None, need, None, 0) == _lib.NK_EINVAL
    assert L.nk_myrtle_nngp_batched(tiles, 2, ctypes.byref(cfg), p, 64, None, 0) == _lib.NK_EINVAL
    assert "workspace" in L.nk_last_error().decode()
    tiles[1].ldk = 6  # < n2
    assert L.nk_myrtle_nngp_batched(tiles, 2, ctypes.byref(cfg), p, need, None, 0) == _lib.NK_EINVAL
    tiles[1].ldk = 7
    tiles[0].n1 = 0
    assert L.nk_myrtle_nngp_batched(tiles, 2, ctypes.byref(cfg), p, need, None, 0) == _lib.NK_EINVAL
    tiles[0].n1 = 5
    tiles[0].K = None
    assert L.nk_myrtle_nngp_batched(tiles, 2, ctypes.byref(cfg), p, need, None, 0) == _lib.NK_EINVAL
    # no pass has been tuned in this process
    out = (_lib.BatchedCandidate * 4)()
    assert L.nk_myrtle_batched_tuning(ctypes.byref(cfg), out, 4, None) == _lib.NK_EINVAL


def test_batched_set_schedule_validation():
    # a configuration no other test tunes
    L = _lib.lib()
    cfg = _lib.myrtle_cfg(8, 2, (1, 3, 1), 1.7, 0.05)
    ch = _lib.BatchedCandidate()
    ch.chunk, ch.pair_tile, ch.persistent, ch.wg_pairs_mult = 4096, 16, 1, 2
    assert L.nk_myrtle_batched_set_schedule(ctypes.byref(cfg), None) == _lib.NK_EINVAL
    for field, bad in (("chunk", 0), ("chunk", 32769), ("pair_tile", 0), ("pair_tile", 257), ("persistent", 2),
                       ("wg_pairs_mult", 3), ("wg_pairs_mult", 0)):
        b = _lib.BatchedCandidate()
        ctypes.memmove(ctypes.byref(b), ctypes.byref(ch), ctypes.sizeof(ch))
        setattr(b, field, bad)
        assert L.nk_myrtle_batched_set_schedule(ctypes.byref(cfg), ctypes.byref(b)) == _lib.NK_EINVAL, field
    assert L.nk_myrtle_batched_set_schedule(ctypes.byref(cfg), ctypes.byref(ch)) == _lib.NK_OK
    out = (_lib.BatchedCandidate * 4)()
    chosen = _lib.BatchedCandidate()
    assert L.nk_myrtle_batched_tuning(ctypes.byref(cfg), out, 4, ctypes.byref(chosen)) == 0
    assert (chosen.chunk, chosen.pair_tile, chosen.persistent, chosen.wg_pairs_mult) == (4096, 16, 1, 2)


def test_solver_workspace_and_validation():
    L = _lib.lib()
    p = ctypes.c_void_p(256)
    cfg = _lib.PcgCfg(64, 100, 1e-8, 0.0)
    a = L.nk_workspace_size(_lib.NK_OP_PCG, ctypes.byref(cfg), 1000, 10)
    cfg0 = _lib.PcgCfg(0, 100, 1e-8, 0.0)
    b = L.nk_workspace_size(_lib.NK_OP_PCG, ctypes.byref(cfg0), 1000, 10)
    assert a > b > 0 and a - b >= 2 * 1000 * 64 * 8  # two copies of L
    assert L.nk_workspace_size(_lib.NK_OP_PCG, None, 1000, 10) == 0
    assert L.nk_workspace_size(_lib.NK_OP_PIVOTED_CHOL, None, 1000, 64) > 1000 * 8
    assert L.nk_workspace_size(_lib.NK_OP_GRAM_MATVEC, None, 1000, 10) > 0
    need = L.nk_workspace_size(_lib.NK_OP_PIVOTED_CHOL, None, 100, 10)
    used = ctypes.c_int32(-7)
    assert L.nk_pivoted_cholesky(None, 100, 100, 10, 0.0, p, p, ctypes.byref(used), p, need, None) == _lib.NK_EINVAL
    assert L.nk_pivoted_cholesky(p, 100, 99, 10, 0.0, p, p, None, p, need, None) == _lib.NK_EINVAL
    assert L.nk_pivoted_cholesky(p, 100, 100, 101, 0.0, p, p, None, p, need, None) == _lib.NK_EINVAL
    assert L.nk_pivoted_cholesky(p, 100, 100, 10, -1.0, p, p, None, p, need, None) == _lib.NK_EINVAL
    assert L.nk_pivoted_cholesky(p, 100, 100, 10, 0.0, p, p, None, p, 64, None) == _lib.NK_EINVAL
    assert "workspace" in L.nk_last_error().decode()
    assert L.nk_pivoted_cholesky(p, 100, 100, 0, 0.0, None, None, ctypes.byref(used), None, 0, None) == _lib.NK_OK
    assert used.value == 0
    mv = L.nk_workspace_size(_lib.NK_OP_GRAM_MATVEC, None, 100, 16)
    assert L.nk_gram_matvec(p, 100, 100, p, 17, 0.0, p, p, mv, None) == _lib.NK_EUNSUPPORTED
    assert L.nk_gram_matvec(p, 100, 100, p, 0, 0.0, p, p, mv, None) == _lib.NK_EUNSUPPORTED
    assert L.nk_gram_matvec(p, 100, 100, p, 4, 0.0, p, p, 8, None) == _lib.NK_EINVAL
    ws = L.nk_workspace_size(_lib.NK_OP_PCG, ctypes.byref(cfg), 100, 10)
    st = _lib.PcgStats()
    assert L.nk_krr_pcg(p, 100, 100, p, 10, 1e-3, 0, None, p, None, None, None, p, ws, None) == _lib.NK_EINVAL
    bad = _lib.PcgCfg(64, 0, 1e-8, 0.0)
    assert L.nk_krr_pcg(p, 100, 100, p, 10, 1e-3, 0, ctypes.byref(bad), p, None, None, None, p, ws,
                        None) == _lib.NK_EINVAL
    bad = _lib.PcgCfg(64, 10, -1.0, 0.0)
    assert L.nk_krr_pcg(p, 100, 100, p, 10, 1e-3, 0, ctypes.byref(bad), p, None, None, None, p, ws,
                        None) == _lib.NK_EINVAL
    assert L.nk_krr_pcg(p, 100, 100, p, 10, 1e-3, 0, ctypes.byref(cfg), p, None, None, ctypes.byref(st), p, 64,
                        None) == _lib.NK_EINVAL
    # lambda = 0 is rejected before any device work
    assert L.nk_krr_pcg(p, 100, 100, p, 10, 0.0, 0, ctypes.byref(cfg), p, None, None, ctypes.byref(st), p, ws,
                        None) == _lib.NK_EINVAL
    assert "lambda" in L.nk_last_error().decode()


def test_cv_validation():
    L = _lib.lib()
    p = ctypes.c_void_p(256)
    cfg = _lib.CvCfg(32, 32, 3, 8, 2.0, 0.01)
    need = L.nk_workspace_size(_lib.NK_OP_CV, ctypes.byref(cfg), 100, 50)
    sym = L.nk_workspace_size(_lib.NK_OP_CV, ctypes.byref(cfg), 100, 0)
    assert need > sym >= 100 * 8 * 32 * 32 * 8
    for bad, code in ((_lib.CvCfg(64, 64, 3, 8, 2.0, 0.01), _lib.NK_EUNSUPPORTED),
                      (_lib.CvCfg(12, 12, 3, 8, 2.0, 0.01), _lib.NK_EUNSUPPORTED),
                      (_lib.CvCfg(32, 16, 3, 8, 2.0, 0.01), _lib.NK_EUNSUPPORTED),
                      (_lib.CvCfg(32, 32, 5, 8, 2.0, 0.01), _lib.NK_EUNSUPPORTED),
                      (_lib.CvCfg(32, 32, 3, 17, 2.0, 0.01), _lib.NK_EUNSUPPORTED),
                      (_lib.CvCfg(32, 32, 3, 0, 2.0, 0.01), _lib.NK_EINVAL),
                      (_lib.CvCfg(32, 32, 3, 8, 0.0, 0.01), _lib.NK_EINVAL),
                      (_lib.CvCfg(32, 32, 3, 8, 2.0, -1.0), _lib.NK_EINVAL)):
        assert L.nk_cv_nngp(p, 4, p, 4, ctypes.byref(bad), p, 4, p, need, None) == code
        assert L.nk_workspace_size(_lib.NK_OP_CV, ctypes.byref(bad), 4, 4) == 0
    assert L.nk_cv_nngp(p, 4, p, 5, ctypes.byref(cfg), p, 4, p, need, None) == _lib.NK_EINVAL  # ldk < n2
    assert L.nk_cv_nngp(p, 0, p, 5, ctypes.byref(cfg), p, 5, p, need, None) == _lib.NK_EINVAL
    assert L.nk_cv_nngp(p, 4, p, 5, ctypes.byref(cfg), p, 5, p, 64, None) == _lib.NK_EINVAL
    assert "workspace" in L.nk_last_error().decode()
    assert L.nk_cv_nngp(None, 4, p, 5, ctypes.byref(cfg), p, 5, p, need, None) == _lib.NK_EINVAL


def test_approx_validation():
    L = _lib.lib()
    p = ctypes.c_void_p(256)
    d = _lib.ApproxDims(100, 10, 20, 3, 0)
    need = L.nk_workspace_size(_lib.NK_OP_APPROX, ctypes.byref(d), 0, 0)
    assert need > 100 * 3 * 8
    bad = _lib.ApproxDims(0, 10, 20, 3, 0)
    assert L.nk_workspace_size(_lib.NK_OP_APPROX, ctypes.byref(bad), 0, 0) == 0
    assert L.nk_krr_nystrom(p, 100, 10, 9, p, 10, p, 20, 100, p, 3, 1e-3, 1e-6, p, p, need, None) == _lib.NK_EINVAL
    assert L.nk_krr_nystrom(p, 100, 101, 101, p, 101, p, 20, 100, p, 3, 1e-3, 1e-6, p, p, need,
                            None) == _lib.NK_EINVAL
    assert L.nk_krr_nystrom(p, 100, 10, 10, p, 10, p, 20, 100, p, 3, 0.0, 1e-6, p, p, need, None) == _lib.NK_EINVAL
    assert L.nk_krr_sor(p, 100, 10, 10, p, 10, p, 20, 9, p, 3, 1e-3, 1e-6, p, p, need, None) == _lib.NK_EINVAL
    assert L.nk_krr_sor(p, 100, 10, 10, p, 10, p, 20, 10, p, 3, 1e-3, -1.0, p, p, need, None) == _lib.NK_EINVAL
    assert L.nk_krr_sor(p, 100, 10, 10, p, 10, p, 20, 10, p, 3, 1e-3, 1e-6, p, p, 64, None) == _lib.NK_EINVAL
    blocks = (ctypes.c_void_p * 2)(256, 256)
    sizes = (ctypes.c_int64 * 2)(60, 40)
    assert L.nk_krr_block_diag(0, blocks, sizes, p, 20, 100, p, 3, 1e-3, p, p, need, None) == _lib.NK_EINVAL
    assert L.nk_krr_block_diag(2, blocks, sizes, p, 20, 99, p, 3, 1e-3, p, p, need, None) == _lib.NK_EINVAL
    sizes[1] = 0
    assert L.nk_krr_block_diag(2, blocks, sizes, p, 20, 100, p, 3, 1e-3, p, p, need, None) == _lib.NK_EINVAL
    sizes[1] = 40
    assert L.nk_krr_bcm(2, blocks, sizes, p, 20, 100, p, 19, p, 3, 1e-3, 0.0, p, p, need, None) == _lib.NK_EINVAL
    assert L.nk_krr_bcm(2, blocks, sizes, p, 20, 100, p, 20, p, 3, 1e-3, 0.0, p, p, 64, None) == _lib.NK_EINVAL
    sizes[0] = 10000
    assert L.nk_krr_bcm(2, blocks, sizes, p, 20, 10040, p, 20, p, 3, 1e-3, 0.0, p, p, need,
                        None) == _lib.NK_EUNSUPPORTED
