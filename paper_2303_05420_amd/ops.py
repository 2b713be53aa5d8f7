"""Python entry points over libnk (include/nk.h).  Tensors must be CUDA
(HIP) float32 and contiguous; torch provides the device memory and the
stream, libnk does all of the computation.  Names match the C ABI."""
from __future__ import annotations

import ctypes
from typing import Sequence

import torch

from . import _lib

_ws_cache: dict = {}


def _stream(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _check_images(x: torch.Tensor, name: str):
    if not isinstance(x, torch.Tensor) or not x.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    if x.dtype != torch.float32 or not x.is_contiguous() or x.dim() != 4:
        raise TypeError(f"{name} must be a contiguous float32 (n, H, W, C) tensor")


def workspace(nbytes: int, device) -> torch.Tensor:
    """A cached uint8 device buffer of at least nbytes (grows, never shrinks)."""
    key = (str(device),)
    buf = _ws_cache.get(key)
    if buf is None or buf.numel() < nbytes:
        buf = None
        _ws_cache.pop(key, None)
        buf = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)
        _ws_cache[key] = buf
    return buf


def release_workspace():
    _ws_cache.clear()


def workspace_size(op: int, cfg, n1: int, n2: int) -> int:
    ptr = ctypes.byref(cfg) if cfg is not None else None
    return int(_lib.lib().nk_workspace_size(op, ptr, int(n1), int(n2)))


def myrtle_nngp(x1: torch.Tensor, x2: torch.Tensor | None, depth: Sequence[int], sigma_w2: float = 2.0,
                sigma_b2: float = 0.0, out: torch.Tensor | None = None, ws: torch.Tensor | None = None,
                ldk: int | None = None) -> torch.Tensor:
    """Myrtle NNGP block K[a, b] = k(x1[a], x2[b]); x2=None means x1 x x1
    (upper triangle computed once and mirrored)."""
    _check_images(x1, "x1")
    sym = x2 is None
    if sym:
        x2 = x1
    else:
        _check_images(x2, "x2")
    n1, h, w, c = x1.shape
    n2 = x2.shape[0]
    if x2.shape[1:] != x1.shape[1:]:
        raise ValueError("x1 and x2 image shapes differ")
    cfg = _lib.myrtle_cfg(h, c, depth, sigma_w2, sigma_b2)
    if out is None:
        ld = n2 if ldk is None else ldk
        out = torch.empty((n1, ld), dtype=torch.float32, device=x1.device)
    ld = out.stride(0) if ldk is None else ldk
    if ws is None:
        need = workspace_size(_lib.NK_OP_MYRTLE, cfg, n1, n2)
        if need == 0:
            _lib.check(_lib.lib().nk_myrtle_nngp(None, 0, None, 0, ctypes.byref(cfg), None, 0, None, 0, None))
        ws = workspace(need, x1.device)
    rc = _lib.lib().nk_myrtle_nngp(x1.data_ptr(), n1, x2.data_ptr(), n2, ctypes.byref(cfg), out.data_ptr(), ld,
                                   ws.data_ptr(), ws.numel(), _stream(x1.device))
    _lib.check(rc)
    return out[:, :n2] if out.shape[1] != n2 else out


def myrtle_ntk(x1: torch.Tensor, x2: torch.Tensor | None, depth: Sequence[int], sigma_w2: float = 2.0,
               sigma_b2: float = 0.0, with_nngp: bool = False, ws: torch.Tensor | None = None):
    """Myrtle neural tangent kernel block Theta[a, b] (x2=None: x1 x x1).  With
    with_nngp=True returns (Theta, K) where K is the NNGP of the same pass."""
    _check_images(x1, "x1")
    sym = x2 is None
    if sym:
        x2 = x1
    else:
        _check_images(x2, "x2")
    if x2.shape[1:] != x1.shape[1:]:
        raise ValueError("x1 and x2 image shapes differ")
    n1, h, w, c = x1.shape
    n2 = x2.shape[0]
    cfg = _lib.myrtle_cfg(h, c, depth, sigma_w2, sigma_b2)
    th = torch.empty((n1, n2), dtype=torch.float32, device=x1.device)
    k = torch.empty((n1, n2), dtype=torch.float32, device=x1.device) if with_nngp else None
    if ws is None:
        need = workspace_size(_lib.NK_OP_MYRTLE_NTK, cfg, n1, n2)
        if need == 0:
            _lib.check(_lib.lib().nk_myrtle_ntk(None, 0, None, 0, ctypes.byref(cfg), None, None, 0, None, 0, None))
        ws = workspace(need, x1.device)
    rc = _lib.lib().nk_myrtle_ntk(x1.data_ptr(), n1, x2.data_ptr(), n2, ctypes.byref(cfg), th.data_ptr(),
                                  None if k is None else k.data_ptr(), n2, ws.data_ptr(), ws.numel(),
                                  _stream(x1.device))
    _lib.check(rc)
    return (th, k) if with_nngp else th


def fc_nngp(x1: torch.Tensor, x2: torch.Tensor | None, depth: int = 3, sigma_w2: float = 2.0,
            sigma_b2: float = 0.01, out: torch.Tensor | None = None) -> torch.Tensor:
    """FC NNGP block on the flattened inputs."""
    if x2 is None:
        x2 = x1
    a = x1.reshape(x1.shape[0], -1)
    b = x2.reshape(x2.shape[0], -1)
    for t, nm in ((a, "x1"), (b, "x2")):
        if not t.is_cuda or t.dtype != torch.float32 or not t.is_contiguous():
            raise TypeError(f"{nm} must be a contiguous float32 CUDA tensor")
    if a.shape[1] != b.shape[1]:
        raise ValueError("feature sizes differ")
    cfg = _lib.FcCfg(int(a.shape[1]), int(depth), float(sigma_w2), float(sigma_b2))
    if out is None:
        out = torch.empty((a.shape[0], b.shape[0]), dtype=torch.float32, device=a.device)
    ws = workspace(workspace_size(_lib.NK_OP_FC, cfg, a.shape[0], b.shape[0]), a.device)
    rc = _lib.lib().nk_fc_nngp(a.data_ptr(), a.shape[0], b.data_ptr(), b.shape[0], ctypes.byref(cfg),
                               out.data_ptr(), out.stride(0), ws.data_ptr(), ws.numel(), _stream(a.device))
    _lib.check(rc)
    return out


def fc_nngp_static(x1: torch.Tensor, x2: torch.Tensor | None, out: torch.Tensor, depth: int = 3,
                   sigma_w2: float = 2.0, sigma_b2: float = 0.01) -> torch.Tensor:
    """nk_fc_nngp_static: the FC NNGP block into the caller's `out` with no
    allocation at all (the library's static scratch holds the diagonals)."""
    if x2 is None:
        x2 = x1
    a = x1.reshape(x1.shape[0], -1)
    b = x2.reshape(x2.shape[0], -1)
    for t, nm in ((a, "x1"), (b, "x2")):
        if not t.is_cuda or t.dtype != torch.float32 or not t.is_contiguous():
            raise TypeError(f"{nm} must be a contiguous float32 CUDA tensor")
    if a.shape[1] != b.shape[1] or out.shape[0] < a.shape[0] or out.shape[1] < b.shape[0]:
        raise ValueError("shape mismatch")
    cfg = _lib.FcCfg(int(a.shape[1]), int(depth), float(sigma_w2), float(sigma_b2))
    rc = _lib.lib().nk_fc_nngp_static(a.data_ptr(), a.shape[0], b.data_ptr(), b.shape[0], ctypes.byref(cfg),
                                      out.data_ptr(), out.stride(0), _stream(a.device))
    _lib.check(rc)
    return out


def krr_predict(k_train: torch.Tensor, k_test: torch.Tensor, y: torch.Tensor, ridge_rel: float) -> torch.Tensor:
    """pred = K_test (K_train + lambda I)^{-1} Y with lambda = ridge_rel mean diag (float64 inside)."""
    for t, nm in ((k_train, "k_train"), (k_test, "k_test"), (y, "y")):
        if not t.is_cuda or t.dtype != torch.float32 or not t.is_contiguous():
            raise TypeError(f"{nm} must be a contiguous float32 CUDA tensor")
    n = k_train.shape[0]
    m = k_test.shape[0]
    c = y.shape[1]
    if k_train.shape != (n, n) or k_test.shape[1] != n or y.shape[0] != n:
        raise ValueError("shape mismatch")
    pred = torch.empty((m, c), dtype=torch.float32, device=k_train.device)
    ws = workspace(workspace_size(_lib.NK_OP_KRR, None, n, max(m, c)), k_train.device)
    rc = _lib.lib().nk_krr_predict(k_train.data_ptr(), n, k_test.data_ptr(), m, y.data_ptr(), c, float(ridge_rel),
                                   pred.data_ptr(), ws.data_ptr(), ws.numel(), _stream(k_train.device))
    _lib.check(rc)
    return pred


def myrtle_nngp_backward(x1: torch.Tensor, x2: torch.Tensor | None, dK: torch.Tensor, depth: Sequence[int],
                         sigma_w2: float = 2.0, sigma_b2: float = 0.0, need_dx: bool = True,
                         ws: torch.Tensor | None = None, need_dx2: bool | None = None):
    """Adjoint of myrtle_nngp: returns (dx1, dx2, dsigma[2]) for cotangent dK.
    For x2=None (symmetric block) dx2 is None and dx1 holds the whole gradient.
    need_dx2=False (default: need_dx) leaves dx2 None and spares the library
    the second image set's seed gradients.
    An x2 that shares x1's memory (same start, same count) asks for the two
    partial gradients separately, so it is passed as a copy: the library reads
    an aliased pair of arguments as one symmetric block."""
    _check_images(x1, "x1")
    sym = x2 is None
    if sym:
        x2 = x1
    else:
        _check_images(x2, "x2")
        if x2.data_ptr() == x1.data_ptr() and x2.shape[0] == x1.shape[0]:
            x2 = x2.clone()
    n1, h, w, c = x1.shape
    n2 = x2.shape[0]
    if dK.shape != (n1, n2) or dK.dtype != torch.float32 or not dK.is_cuda:
        raise ValueError("dK must be a float32 CUDA tensor of shape (n1, n2)")
    dK = dK.contiguous()
    cfg = _lib.myrtle_cfg(h, c, depth, sigma_w2, sigma_b2)
    dx1 = torch.empty_like(x1) if need_dx else None
    if need_dx2 is None:
        need_dx2 = need_dx
    dx2 = None if sym or not need_dx2 else torch.empty_like(x2)
    ds = torch.empty(2, dtype=torch.float32, device=x1.device)
    if ws is None:
        need = workspace_size(_lib.NK_OP_MYRTLE_BWD, cfg, n1, n2)
        if need == 0:
            _lib.check(_lib.lib().nk_myrtle_nngp_backward(None, 0, None, 0, ctypes.byref(cfg), None, 0, None, None,
                                                          None, None, 0, None))
        ws = workspace(need, x1.device)
    rc = _lib.lib().nk_myrtle_nngp_backward(
        x1.data_ptr(), n1, x2.data_ptr(), n2, ctypes.byref(cfg), dK.data_ptr(), dK.stride(0),
        None if dx1 is None else dx1.data_ptr(), None if dx2 is None else dx2.data_ptr(), ds.data_ptr(),
        ws.data_ptr(), ws.numel(), _stream(x1.device))
    _lib.check(rc)
    return dx1, dx2, ds


def krr_mse_grad(x_s: torch.Tensor, y_s: torch.Tensor, x_t: torch.Tensor, y_t: torch.Tensor, depth: Sequence[int],
                 sigma_w2: float = 2.0, sigma_b2: float = 0.0, ridge: float = 1e-4, relative: bool = True,
                 ws: torch.Tensor | None = None, keep_checkpoints: bool = False):
    """nk_krr_mse_grad: (loss, dL/dx_s, dL/d[sigma_w2, sigma_b2], lambda) of the
    held-out squared error of kernel ridge regression of the support images
    x_s (labels y_s) onto the targets x_t (labels y_t); lambda = ridge (times
    mean diag K_ss when relative) is held fixed.  keep_checkpoints: every
    pair's first-stage output is kept between the forward and the adjoint
    pass (nk_krr_mse_grad_kept, nk_krr_mse_grad_workspace_keep bytes of
    workspace) instead of being recomputed."""
    _check_images(x_s, "x_s")
    _check_images(x_t, "x_t")
    for t, nm in ((y_s, "y_s"), (y_t, "y_t")):
        if not t.is_cuda or t.dtype != torch.float32 or not t.is_contiguous() or t.dim() != 2:
            raise TypeError(f"{nm} must be a contiguous float32 CUDA matrix")
    n, h, w, c = x_s.shape
    m = x_t.shape[0]
    k = y_s.shape[1]
    if x_t.shape[1:] != x_s.shape[1:] or y_s.shape[0] != n or y_t.shape != (m, k):
        raise ValueError("shape mismatch")
    if x_t.data_ptr() == x_s.data_ptr():
        x_t = x_t.clone()
    cfg = _lib.myrtle_cfg(h, c, depth, sigma_w2, sigma_b2)
    if ws is None:
        size_fn = _lib.lib().nk_krr_mse_grad_workspace_keep if keep_checkpoints else _lib.lib().nk_krr_mse_grad_workspace
        need = int(size_fn(ctypes.byref(cfg), n, m, k))
        if need == 0:
            raise ValueError("invalid network or sizes for nk_krr_mse_grad")
        ws = workspace(need, x_s.device)
    dx = torch.empty_like(x_s)
    ds = torch.empty(2, dtype=torch.float32, device=x_s.device)
    loss = ctypes.c_double(0.0)
    lam = ctypes.c_double(0.0)
    fn = _lib.lib().nk_krr_mse_grad_kept if keep_checkpoints else _lib.lib().nk_krr_mse_grad
    rc = fn(x_s.data_ptr(), n, x_t.data_ptr(), m, y_s.data_ptr(), y_t.data_ptr(), k, ctypes.byref(cfg), float(ridge),
            1 if relative else 0, dx.data_ptr(), ds.data_ptr(), ctypes.byref(loss), ctypes.byref(lam), ws.data_ptr(),
            ws.numel(), _stream(x_s.device))
    _lib.check(rc)
    return loss.value, dx, ds, lam.value


def cv_nngp(x1: torch.Tensor, x2: torch.Tensor | None, depth: int = 8, sigma_w2: float = 2.0,
            sigma_b2: float = 0.01, out: torch.Tensor | None = None) -> torch.Tensor:
    """CNN-VEC (CV8 for depth 8) NNGP block of NHWC images; x2 None or x1
    gives the symmetric block."""
    if x2 is None:
        x2 = x1
    _check_images(x1, "x1")
    _check_images(x2, "x2")
    if x1.shape[1:] != x2.shape[1:]:
        raise ValueError("image shapes differ")
    n1, h, w, c = (int(v) for v in x1.shape)
    n2 = int(x2.shape[0])
    cfg = _lib.CvCfg(h, w, c, int(depth), float(sigma_w2), float(sigma_b2))
    sym = x1.data_ptr() == x2.data_ptr() and n1 == n2
    if out is None:
        out = torch.empty((n1, n2), dtype=torch.float32, device=x1.device)
    ws = workspace(workspace_size(_lib.NK_OP_CV, cfg, n1, 0 if sym else n2), x1.device)
    rc = _lib.lib().nk_cv_nngp(x1.data_ptr(), n1, x2.data_ptr(), n2, ctypes.byref(cfg), out.data_ptr(),
                               out.stride(0), ws.data_ptr(), ws.numel(), _stream(x1.device))
    _lib.check(rc)
    return out


def _f32_rows(t: torch.Tensor, name: str):
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float32 or t.dim() != 2 \
            or t.stride(1) != 1:
        raise TypeError(f"{name} must be a 2-D float32 CUDA tensor with contiguous rows")
    return int(t.shape[0]), int(t.shape[1]), int(t.stride(0))


def _approx_ws(n, r, m, c, maxb, device):
    d = _lib.ApproxDims(int(n), int(r), int(m), int(c), int(maxb))
    return workspace(workspace_size(_lib.NK_OP_APPROX, d, 0, 0), device)


def krr_nystrom(k_nr, k_rr, k_mn, y, lam: float, jitter: float = 1e-6) -> torch.Tensor:
    """Nystrom kernel ridge regression prediction (float32 m x c)."""
    n, r, ldnr = _f32_rows(k_nr, "k_nr")
    _, _, ldrr = _f32_rows(k_rr, "k_rr")
    m, _, ldmn = _f32_rows(k_mn, "k_mn")
    _, c, _ = _f32_rows(y, "y")
    pred = torch.empty((m, c), dtype=torch.float32, device=y.device)
    ws = _approx_ws(n, r, m, c, 0, y.device)
    rc = _lib.lib().nk_krr_nystrom(k_nr.data_ptr(), n, r, ldnr, k_rr.data_ptr(), ldrr, k_mn.data_ptr(), m, ldmn,
                                   y.contiguous().data_ptr(), c, float(lam), float(jitter), pred.data_ptr(),
                                   ws.data_ptr(), ws.numel(), _stream(y.device))
    _lib.check(rc)
    return pred


def krr_sor(k_nr, k_rr, k_mr, y, lam: float, jitter: float = 1e-6) -> torch.Tensor:
    """Subset-of-regressors prediction (float32 m x c)."""
    n, r, ldnr = _f32_rows(k_nr, "k_nr")
    _, _, ldrr = _f32_rows(k_rr, "k_rr")
    m, _, ldmr = _f32_rows(k_mr, "k_mr")
    _, c, _ = _f32_rows(y, "y")
    pred = torch.empty((m, c), dtype=torch.float32, device=y.device)
    ws = _approx_ws(n, r, m, c, 0, y.device)
    rc = _lib.lib().nk_krr_sor(k_nr.data_ptr(), n, r, ldnr, k_rr.data_ptr(), ldrr, k_mr.data_ptr(), m, ldmr,
                               y.contiguous().data_ptr(), c, float(lam), float(jitter), pred.data_ptr(),
                               ws.data_ptr(), ws.numel(), _stream(y.device))
    _lib.check(rc)
    return pred


def _blocks(blocks):
    ptrs = (ctypes.c_void_p * len(blocks))(*[b.data_ptr() for b in blocks])
    sizes = (ctypes.c_int64 * len(blocks))(*[int(b.shape[0]) for b in blocks])
    for b in blocks:
        if not b.is_cuda or b.dtype != torch.float32 or not b.is_contiguous() or b.shape[0] != b.shape[1]:
            raise TypeError("blocks must be square contiguous float32 CUDA tensors")
    return ptrs, sizes, sum(int(b.shape[0]) for b in blocks), max(int(b.shape[0]) for b in blocks)


def krr_block_diag(blocks, k_mn, y, lam: float) -> torch.Tensor:
    """Block-diagonal approximation; training points ordered block by block."""
    ptrs, sizes, n, maxb = _blocks(blocks)
    m, _, ldmn = _f32_rows(k_mn, "k_mn")
    _, c, _ = _f32_rows(y, "y")
    pred = torch.empty((m, c), dtype=torch.float32, device=y.device)
    ws = _approx_ws(n, 0, m, c, maxb, y.device)
    rc = _lib.lib().nk_krr_block_diag(len(blocks), ptrs, sizes, k_mn.data_ptr(), m, ldmn, y.contiguous().data_ptr(),
                                      c, float(lam), pred.data_ptr(), ws.data_ptr(), ws.numel(), _stream(y.device))
    _lib.check(rc)
    return pred


def krr_bcm(blocks, k_mn, k_mm, y, lam: float, jitter: float = 0.0) -> torch.Tensor:
    """Bayesian committee machine posterior mean of the test points (jointly)."""
    ptrs, sizes, n, maxb = _blocks(blocks)
    m, _, ldmn = _f32_rows(k_mn, "k_mn")
    _, _, ldmm = _f32_rows(k_mm, "k_mm")
    _, c, _ = _f32_rows(y, "y")
    pred = torch.empty((m, c), dtype=torch.float32, device=y.device)
    ws = _approx_ws(n, 0, m, c, maxb, y.device)
    rc = _lib.lib().nk_krr_bcm(len(blocks), ptrs, sizes, k_mn.data_ptr(), m, ldmn, k_mm.data_ptr(), ldmm,
                               y.contiguous().data_ptr(), c, float(lam), float(jitter), pred.data_ptr(),
                               ws.data_ptr(), ws.numel(), _stream(y.device))
    _lib.check(rc)
    return pred


def _check_gram(k: torch.Tensor) -> tuple[int, int]:
    """(n, ldk) of a float32 CUDA n x n matrix with unit column stride."""
    if not isinstance(k, torch.Tensor) or not k.is_cuda or k.dtype != torch.float32:
        raise TypeError("k must be a float32 CUDA tensor")
    if k.dim() != 2 or k.shape[0] != k.shape[1] or k.stride(1) != 1 or k.stride(0) < k.shape[0]:
        raise ValueError("k must be square with rows contiguous")
    return int(k.shape[0]), int(k.stride(0))


def pivoted_cholesky(k: torch.Tensor, rank: int, pivot_tol: float = 0.0):
    """Greedy partial pivoted Cholesky K ~ L L^T (float64): returns (L as an
    n x rank view of the column-major factor, piv (int32, -1 past the rank
    reached), rank reached)."""
    n, ldk = _check_gram(k)
    rank = int(rank)
    lcm = torch.zeros((max(rank, 0), n), dtype=torch.float64, device=k.device)
    piv = torch.full((max(rank, 0),), -1, dtype=torch.int32, device=k.device)
    used = ctypes.c_int32(0)
    ws = workspace(workspace_size(_lib.NK_OP_PIVOTED_CHOL, None, n, max(rank, 0)), k.device)
    rc = _lib.lib().nk_pivoted_cholesky(k.data_ptr(), n, ldk, rank, float(pivot_tol), lcm.data_ptr(),
                                        piv.data_ptr(), ctypes.byref(used), ws.data_ptr(), ws.numel(),
                                        _stream(k.device))
    _lib.check(rc)
    return lcm.t(), piv, int(used.value)


def gram_matvec(k: torch.Tensor, p: torch.Tensor, lam: float = 0.0) -> torch.Tensor:
    """Q = (K + lam I) P for a symmetric float32 K and float64 P (n x c, c <= 16)."""
    n, ldk = _check_gram(k)
    if not p.is_cuda or p.dtype != torch.float64 or not p.is_contiguous() or p.dim() != 2 or p.shape[0] != n:
        raise TypeError("p must be a contiguous float64 CUDA (n, c) tensor")
    c = int(p.shape[1])
    q = torch.empty_like(p)
    ws = workspace(workspace_size(_lib.NK_OP_GRAM_MATVEC, None, n, c), k.device)
    rc = _lib.lib().nk_gram_matvec(k.data_ptr(), n, ldk, p.data_ptr(), c, float(lam), q.data_ptr(), ws.data_ptr(),
                                   ws.numel(), _stream(k.device))
    _lib.check(rc)
    return q


def krr_pcg(k: torch.Tensor, y: torch.Tensor, ridge: float, relative: bool = True, rank: int = 100,
            tol: float = 1e-8, max_iter: int = 1000, pivot_tol: float = 0.0):
    """Solve (K + lam I) X = Y by preconditioned CG in float64 (lam = ridge,
    or ridge * mean diag K if relative).  Returns (X, iters, relres, stats)
    with iters/relres numpy arrays and stats = {rank, iterations, lambda}."""
    import numpy as np

    n, ldk = _check_gram(k)
    if not y.is_cuda or y.dtype != torch.float64 or not y.is_contiguous() or y.dim() != 2 or y.shape[0] != n:
        raise TypeError("y must be a contiguous float64 CUDA (n, c) tensor")
    c = int(y.shape[1])
    cfg = _lib.PcgCfg()
    cfg.rank = int(rank)
    cfg.max_iter = int(max_iter)
    cfg.tol = float(tol)
    cfg.pivot_tol = float(pivot_tol)
    x = torch.empty_like(y)
    iters = np.zeros(c, dtype=np.int32)
    relres = np.zeros(c, dtype=np.float64)
    st = _lib.PcgStats()
    ws = workspace(workspace_size(_lib.NK_OP_PCG, cfg, n, c), k.device)
    rc = _lib.lib().nk_krr_pcg(k.data_ptr(), n, ldk, y.data_ptr(), c, float(ridge), 1 if relative else 0,
                               ctypes.byref(cfg), x.data_ptr(), iters.ctypes.data, relres.ctypes.data,
                               ctypes.byref(st), ws.data_ptr(), ws.numel(), _stream(k.device))
    _lib.check(rc)
    return x, iters, relres, {"rank": int(st.rank), "iterations": int(st.iterations), "lambda": float(st.lambda_)}


def krr_mse_backward(k_ss: torch.Tensor, k_ts: torch.Tensor, y_s: torch.Tensor, y_t: torch.Tensor, ridge: float,
                     relative: bool = False):
    """Cotangents of L = mean((K_ts (K_ss + lam I)^{-1} Y_s - Y_t)^2) with lam
    held fixed (lam = ridge, or ridge * mean diag K_ss if relative):
    returns (dK_ss, dK_ts, L, lam)."""
    for t, nm in ((k_ss, "k_ss"), (k_ts, "k_ts"), (y_s, "y_s"), (y_t, "y_t")):
        if not t.is_cuda or t.dtype != torch.float32 or not t.is_contiguous():
            raise TypeError(f"{nm} must be a contiguous float32 CUDA tensor")
    n = k_ss.shape[0]
    m = k_ts.shape[0]
    c = y_s.shape[1]
    if k_ss.shape != (n, n) or k_ts.shape != (m, n) or y_s.shape != (n, c) or y_t.shape != (m, c):
        raise ValueError("shape mismatch")
    dss = torch.empty_like(k_ss)
    dts = torch.empty_like(k_ts)
    loss = ctypes.c_double(0.0)
    lam = ctypes.c_double(0.0)
    ws = workspace(workspace_size(_lib.NK_OP_KRR, None, n, max(m, c)), k_ss.device)
    rc = _lib.lib().nk_krr_mse_backward(k_ss.data_ptr(), n, k_ts.data_ptr(), m, y_s.data_ptr(), y_t.data_ptr(), c,
                                        float(ridge), 1 if relative else 0, dss.data_ptr(), dts.data_ptr(),
                                        ctypes.byref(loss), ctypes.byref(lam), ws.data_ptr(), ws.numel(),
                                        _stream(k_ss.device))
    _lib.check(rc)
    return dss, dts, float(loss.value), float(lam.value)


def myrtle_nngp_batched(tiles, depth: Sequence[int], sigma_w2: float = 2.0, sigma_b2: float = 0.0,
                        graph: bool = False, ws: torch.Tensor | None = None):
    """Many Myrtle Gram tiles in one scheduled pass.  `tiles` is a list of
    (x1, x2_or_None, out) with out a float32 (n1, >= n2) CUDA tensor whose
    rows receive K[a, b] = k(x1[a], x2[b]) (x2 None: the symmetric x1 x x1
    tile).  Tiles passing the same x tensor share its variance tables."""
    if not tiles:
        raise ValueError("no tiles")
    arr = (_lib.Tile * len(tiles))()
    hw = c = None
    dev = None
    for i, (x1, x2, out) in enumerate(tiles):
        _check_images(x1, "x1")
        if x2 is None:
            x2 = x1
        else:
            _check_images(x2, "x2")
        if x2.shape[1:] != x1.shape[1:] or (hw is not None and (x1.shape[1], x1.shape[3]) != (hw, c)):
            raise ValueError("all tiles must use images of one shape")
        hw, c = x1.shape[1], x1.shape[3]
        dev = x1.device
        if out.dtype != torch.float32 or not out.is_cuda or out.dim() != 2 or out.stride(1) != 1:
            raise TypeError("out must be a row-major float32 CUDA matrix")
        if out.shape[0] < x1.shape[0] or out.shape[1] < x2.shape[0]:
            raise ValueError("out is smaller than the tile")
        arr[i].x1 = x1.data_ptr()
        arr[i].x2 = x2.data_ptr()
        arr[i].n1 = x1.shape[0]
        arr[i].n2 = x2.shape[0]
        arr[i].K = out.data_ptr()
        arr[i].ldk = out.stride(0)
    cfg = _lib.myrtle_cfg(hw, c, depth, sigma_w2, sigma_b2)
    L = _lib.lib()
    if ws is None:
        need = int(L.nk_myrtle_nngp_batched_workspace(arr, len(tiles), ctypes.byref(cfg)))
        if need == 0:
            _lib.check(L.nk_myrtle_nngp_batched(arr, len(tiles), ctypes.byref(cfg), None, 0, None, 0))
        ws = workspace(need, dev)
    rc = L.nk_myrtle_nngp_batched(arr, len(tiles), ctypes.byref(cfg), ws.data_ptr(), ws.numel(), _stream(dev),
                                  1 if graph else 0)
    _lib.check(rc)


def batched_workspace_size(tiles, depth: Sequence[int], sigma_w2: float = 2.0, sigma_b2: float = 0.0) -> int:
    arr = (_lib.Tile * len(tiles))()
    for i, (x1, x2, out) in enumerate(tiles):
        x2 = x1 if x2 is None else x2
        arr[i].x1, arr[i].x2 = x1.data_ptr(), x2.data_ptr()
        arr[i].n1, arr[i].n2 = x1.shape[0], x2.shape[0]
        arr[i].K, arr[i].ldk = out.data_ptr(), out.stride(0)
    x1 = tiles[0][0]
    cfg = _lib.myrtle_cfg(x1.shape[1], x1.shape[3], depth, sigma_w2, sigma_b2)
    return int(_lib.lib().nk_myrtle_nngp_batched_workspace(arr, len(tiles), ctypes.byref(cfg)))


def batched_tuning(hw: int, c: int, depth: Sequence[int], sigma_w2: float = 2.0, sigma_b2: float = 0.0):
    """(candidates, chosen) of the batched schedule tuned for this network, as
    lists of dicts; raises if no batched pass has run for it yet."""
    cfg = _lib.myrtle_cfg(hw, c, depth, sigma_w2, sigma_b2)
    buf = (_lib.BatchedCandidate * 64)()
    ch = _lib.BatchedCandidate()
    n = _lib.lib().nk_myrtle_batched_tuning(ctypes.byref(cfg), buf, 64, ctypes.byref(ch))
    if n < 0:
        _lib.check(n)

    def d(x):
        return {"chunk": int(x.chunk), "pair_tile": int(x.pair_tile), "persistent": int(x.persistent),
                "us_per_pair": float(x.us_per_pair), "kind": "shape" if x.kind else "schedule",
                "wg_pairs_mult": int(x.wg_pairs_mult)}
    return [d(buf[i]) for i in range(min(n, 64))], d(ch)


def batched_set_schedule(hw: int, c: int, depth: Sequence[int], sigma_w2: float = 2.0, sigma_b2: float = 0.0, *,
                         chunk: int, pair_tile: int, persistent: int, wg_pairs_mult: int):
    """Fixes the batched pass's schedule and kernel shape for this network for
    the rest of the process, in place of tuning (nk_myrtle_batched_set_schedule)."""
    cfg = _lib.myrtle_cfg(hw, c, depth, sigma_w2, sigma_b2)
    ch = _lib.BatchedCandidate()
    ch.chunk, ch.pair_tile, ch.persistent, ch.wg_pairs_mult = chunk, pair_tile, persistent, wg_pairs_mult
    _lib.check(_lib.lib().nk_myrtle_batched_set_schedule(ctypes.byref(cfg), ctypes.byref(ch)))
