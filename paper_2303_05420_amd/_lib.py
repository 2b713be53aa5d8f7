"""ctypes view of libnk.so (include/nk.h).  Marshalling only: every step of
the computation runs in the library's HIP kernels.  Loading fails loudly if
the library has not been built."""
from __future__ import annotations

import ctypes
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnk.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "nk.h")

NK_OK = 0
NK_EINVAL = -1
NK_EUNSUPPORTED = -2
NK_EHIP = -3
NK_ENOMEM = -4
NK_ENOTPD = -5

NK_OP_FC = 0
NK_OP_MYRTLE = 1
NK_OP_MYRTLE_BWD = 2
NK_OP_KRR = 3
NK_OP_MYRTLE_BATCHED = 4
NK_OP_MYRTLE_NTK = 5
NK_OP_PCG = 6
NK_OP_PIVOTED_CHOL = 7
NK_OP_GRAM_MATVEC = 8
NK_OP_CV = 9
NK_OP_APPROX = 10


class MyrtleCfg(ctypes.Structure):
    _fields_ = [("H", ctypes.c_int32), ("W", ctypes.c_int32), ("C", ctypes.c_int32), ("n_stages", ctypes.c_int32),
                ("depth", ctypes.c_int32 * 4), ("filter", ctypes.c_int32), ("sigma_w2", ctypes.c_float),
                ("sigma_b2", ctypes.c_float)]


class FcCfg(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int32), ("depth", ctypes.c_int32), ("sigma_w2", ctypes.c_float),
                ("sigma_b2", ctypes.c_float)]


class Tile(ctypes.Structure):
    _fields_ = [("x1", ctypes.c_void_p), ("x2", ctypes.c_void_p), ("n1", ctypes.c_int64), ("n2", ctypes.c_int64),
                ("K", ctypes.c_void_p), ("ldk", ctypes.c_int64)]


class BatchedCandidate(ctypes.Structure):
    _fields_ = [("chunk", ctypes.c_int64), ("pair_tile", ctypes.c_int32), ("persistent", ctypes.c_int32),
                ("us_per_pair", ctypes.c_double), ("kind", ctypes.c_int32), ("wg_pairs_mult", ctypes.c_int32)]


class CvCfg(ctypes.Structure):
    _fields_ = [("H", ctypes.c_int32), ("W", ctypes.c_int32), ("C", ctypes.c_int32), ("depth", ctypes.c_int32),
                ("sigma_w2", ctypes.c_float), ("sigma_b2", ctypes.c_float)]


class ApproxDims(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("r", ctypes.c_int64), ("m", ctypes.c_int64), ("c", ctypes.c_int64),
                ("max_block", ctypes.c_int64)]


class PcgCfg(ctypes.Structure):
    _fields_ = [("rank", ctypes.c_int32), ("max_iter", ctypes.c_int32), ("tol", ctypes.c_double),
                ("pivot_tol", ctypes.c_double)]


class PcgStats(ctypes.Structure):
    _fields_ = [("rank", ctypes.c_int32), ("iterations", ctypes.c_int32), ("lambda_", ctypes.c_double)]


class ProfileEntry(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 48), ("launches", ctypes.c_int64), ("total_ms", ctypes.c_double)]


class NKError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libnk error {code}: {msg}")
        self.code = code


_lib = None


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2303_05420_amd.build` "
                           "(there is no fallback implementation)")
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    i64 = ctypes.c_int64
    i32 = ctypes.c_int32
    ci = ctypes.c_int
    sz = ctypes.c_size_t
    L.nk_workspace_size.argtypes = [ci, P, i64, i64]
    L.nk_workspace_size.restype = sz
    L.nk_fc_nngp.argtypes = [P, i64, P, i64, ctypes.POINTER(FcCfg), P, i64, P, sz, P]
    L.nk_fc_nngp.restype = ci
    L.nk_fc_nngp_static.argtypes = [P, i64, P, i64, ctypes.POINTER(FcCfg), P, i64, P]
    L.nk_fc_nngp_static.restype = ci
    L.nk_myrtle_nngp.argtypes = [P, i64, P, i64, ctypes.POINTER(MyrtleCfg), P, i64, P, sz, P]
    L.nk_myrtle_nngp.restype = ci
    L.nk_myrtle_ntk.argtypes = [P, i64, P, i64, ctypes.POINTER(MyrtleCfg), P, P, i64, P, sz, P]
    L.nk_myrtle_ntk.restype = ci
    L.nk_myrtle_nngp_backward.argtypes = [P, i64, P, i64, ctypes.POINTER(MyrtleCfg), P, i64, P, P, P, P, sz, P]
    L.nk_myrtle_nngp_backward.restype = ci
    L.nk_krr_predict.argtypes = [P, i64, P, i64, P, i64, ctypes.c_double, P, P, sz, P]
    L.nk_krr_predict.restype = ci
    L.nk_krr_mse_backward.argtypes = [P, i64, P, i64, P, P, i64, ctypes.c_double, ci, P, P,
                                      ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double), P, sz, P]
    L.nk_krr_mse_backward.restype = ci
    L.nk_krr_mse_grad.argtypes = [P, i64, P, i64, P, P, i64, ctypes.POINTER(MyrtleCfg), ctypes.c_double, ci, P, P,
                                  ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double), P, sz, P]
    L.nk_krr_mse_grad.restype = ci
    L.nk_krr_mse_grad_workspace.argtypes = [ctypes.POINTER(MyrtleCfg), i64, i64, i64]
    L.nk_krr_mse_grad_workspace.restype = sz
    L.nk_krr_mse_grad_kept.argtypes = L.nk_krr_mse_grad.argtypes
    L.nk_krr_mse_grad_kept.restype = ci
    L.nk_krr_mse_grad_workspace_keep.argtypes = [ctypes.POINTER(MyrtleCfg), i64, i64, i64]
    L.nk_krr_mse_grad_workspace_keep.restype = sz
    L.nk_myrtle_nngp_batched.argtypes = [ctypes.POINTER(Tile), i32, ctypes.POINTER(MyrtleCfg), P, sz, P, i32]
    L.nk_myrtle_nngp_batched.restype = ci
    L.nk_myrtle_nngp_batched_workspace.argtypes = [ctypes.POINTER(Tile), i32, ctypes.POINTER(MyrtleCfg)]
    L.nk_myrtle_nngp_batched_workspace.restype = sz
    L.nk_myrtle_batched_tuning.argtypes = [ctypes.POINTER(MyrtleCfg), ctypes.POINTER(BatchedCandidate), ci,
                                           ctypes.POINTER(BatchedCandidate)]
    L.nk_myrtle_batched_tuning.restype = ci
    L.nk_myrtle_batched_set_schedule.argtypes = [ctypes.POINTER(MyrtleCfg), ctypes.POINTER(BatchedCandidate)]
    L.nk_myrtle_batched_set_schedule.restype = ci
    dbl = ctypes.c_double
    L.nk_cv_nngp.argtypes = [P, i64, P, i64, ctypes.POINTER(CvCfg), P, i64, P, sz, P]
    L.nk_cv_nngp.restype = ci
    L.nk_krr_nystrom.argtypes = [P, i64, i64, i64, P, i64, P, i64, i64, P, i64, dbl, dbl, P, P, sz, P]
    L.nk_krr_nystrom.restype = ci
    L.nk_krr_sor.argtypes = [P, i64, i64, i64, P, i64, P, i64, i64, P, i64, dbl, dbl, P, P, sz, P]
    L.nk_krr_sor.restype = ci
    L.nk_krr_block_diag.argtypes = [i32, P, P, P, i64, i64, P, i64, dbl, P, P, sz, P]
    L.nk_krr_block_diag.restype = ci
    L.nk_krr_bcm.argtypes = [i32, P, P, P, i64, i64, P, i64, P, i64, dbl, dbl, P, P, sz, P]
    L.nk_krr_bcm.restype = ci
    L.nk_pivoted_cholesky.argtypes = [P, i64, i64, i32, dbl, P, P, ctypes.POINTER(i32), P, sz, P]
    L.nk_pivoted_cholesky.restype = ci
    L.nk_gram_matvec.argtypes = [P, i64, i64, P, i64, dbl, P, P, sz, P]
    L.nk_gram_matvec.restype = ci
    L.nk_krr_pcg.argtypes = [P, i64, i64, P, i64, dbl, ci, ctypes.POINTER(PcgCfg), P, P, P,
                             ctypes.POINTER(PcgStats), P, sz, P]
    L.nk_krr_pcg.restype = ci
    L.nk_profile_enable.argtypes = [ci]
    L.nk_profile_enable.restype = ci
    L.nk_profile_read.argtypes = [ctypes.POINTER(ProfileEntry), ci, ci]
    L.nk_profile_read.restype = ci
    L.nk_last_error.argtypes = []
    L.nk_last_error.restype = ctypes.c_char_p
    L.nk_version.argtypes = []
    L.nk_version.restype = ctypes.c_char_p
    _lib = L
    return L


def check(rc: int):
    if rc != NK_OK:
        raise NKError(rc, lib().nk_last_error().decode())


def header_functions() -> list[str]:
    """Names of every function declared in include/nk.h."""
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(nk_[a-z0-9_]+)\s*\(", txt)))


def myrtle_cfg(hw: int, c: int, depth, sigma_w2: float, sigma_b2: float) -> MyrtleCfg:
    d = list(depth)
    if len(d) > 4:
        raise ValueError("at most 4 stages")
    cfg = MyrtleCfg()
    cfg.H = cfg.W = int(hw)
    cfg.C = int(c)
    cfg.n_stages = len(d)
    for i in range(4):
        cfg.depth[i] = int(d[i]) if i < len(d) else 0
    cfg.filter = 3
    cfg.sigma_w2 = float(sigma_w2)
    cfg.sigma_b2 = float(sigma_b2)
    return cfg


def profile_enable(on: bool = True):
    check(lib().nk_profile_enable(1 if on else 0))


def profile_read(reset: bool = True) -> dict:
    """{kernel kind: (launches, total_ms)} of the launches recorded so far."""
    buf = (ProfileEntry * 64)()
    n = lib().nk_profile_read(buf, 64, 1 if reset else 0)
    if n < 0:
        check(n)
    return {buf[i].name.decode(): (int(buf[i].launches), float(buf[i].total_ms)) for i in range(min(n, 64))}
