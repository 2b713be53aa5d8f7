"""FP64 CPU oracle for the NNGP kernels and kernel ridge regression.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package.  It shares no
code with the GPU library ``paper_2303_05420_amd`` and never imports it.

Contents
--------
* ``myrtle_self`` / ``myrtle_pairs`` / ``myrtle_gram`` -- the Myrtle NNGP
  (App. A, Myrtle listing) as the plain float64 loop recursion in
  ``nk_oracle.c``.
* ``myrtle_ntk_pairs`` / ``myrtle_ntk_gram`` -- the Myrtle neural tangent
  kernel (the kernel of the paper's large-scale runs) with its NNGP, same C
  file.
* ``fc_nngp`` -- the FC3 NNGP (App. A, FC listing), same C file.
* ``cv_self`` / ``cv_pairs`` / ``cv_gram`` -- the CNN-VEC (CV8) NNGP
  (App. A, CNN-VEC listing: full-resolution convs, Flatten readout), same C
  file.
* ``krr_predict`` -- kernel ridge regression, the linear system that the
  paper's conjugate-gradient solver targets (Sec. 2, iterative solvers),
  solved exactly with a float64 Cholesky factorisation.
* ``grad`` (submodule) -- float64 PyTorch autograd over a tensor form of the
  same recursion, used as the reference for kernel gradients.
* ``matrix_form`` (submodule) -- joint-covariance-matrix form of the Myrtle
  recursion for tiny images, used to pin the C loop nest.
* ``solvers`` (submodule) -- the partial pivoted Cholesky preconditioner and
  preconditioned conjugate gradients in float64 (Sec. 2, iterative solvers).
* ``approx`` (submodule) -- Nystrom, subset of regressors, block-diagonal and
  Bayesian-committee-machine predictions in float64 (Sec. 2, approximations
  to the linear system).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass
from typing import Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "nk_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libnk_oracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (float64, OpenMP)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.c_void_p
    i64 = ctypes.c_int64
    ci = ctypes.c_int
    cd = ctypes.c_double
    lib.nko_myrtle_self.argtypes = [P, i64, ci, ci, ci, ci, P, cd, cd, P, P, ci]
    lib.nko_myrtle_self.restype = ci
    lib.nko_myrtle_pairs.argtypes = [P, P, P, P, ci, ci, ci, ci, P, cd, cd, P, i64, P, ci]
    lib.nko_myrtle_pairs.restype = ci
    lib.nko_myrtle_qmaps_len.argtypes = [ci, ci, ci, P]
    lib.nko_myrtle_qmaps_len.restype = ctypes.c_size_t
    lib.nko_fc_nngp.argtypes = [P, i64, P, i64, ci, ci, cd, cd, P, ci]
    lib.nko_fc_nngp.restype = ci
    lib.nko_relu_map.argtypes = [cd, cd, cd]
    lib.nko_relu_map.restype = cd
    lib.nko_relu_dot.argtypes = [cd, cd, cd]
    lib.nko_relu_dot.restype = cd
    lib.nko_myrtle_ntk_pairs.argtypes = [P, P, P, P, ci, ci, ci, ci, P, cd, cd, P, i64, P, P, ci]
    lib.nko_myrtle_ntk_pairs.restype = ci
    lib.nko_cv_self.argtypes = [P, i64, ci, ci, ci, ci, cd, cd, P, P, ci]
    lib.nko_cv_self.restype = ci
    lib.nko_cv_pairs.argtypes = [P, P, P, P, ci, ci, ci, ci, cd, cd, P, i64, P, ci]
    lib.nko_cv_pairs.restype = ci
    lib.nko_num_threads.argtypes = []
    lib.nko_num_threads.restype = ci
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def default_threads() -> int:
    return max(1, len(os.sched_getaffinity(0)))


@dataclass(frozen=True)
class Myrtle:
    """Myrtle network: ``depth[s]`` [conv3x3, ReLU] blocks at stage s, 2x2
    average pools between stages, global average pool and Dense readout."""

    depth: Sequence[int]
    sigma_w2: float = 2.0
    sigma_b2: float = 0.0

    @property
    def n_stages(self) -> int:
        return len(self.depth)


def relu_map(s: float, q1: float, q2: float) -> float:
    """E[relu(u) relu(v)], (u, v) ~ N(0, [[q1, s], [s, q2]])."""
    return float(_load().nko_relu_map(float(s), float(q1), float(q2)))


def relu_dot(s: float, q1: float, q2: float) -> float:
    """E[relu'(u) relu'(v)], (u, v) ~ N(0, [[q1, s], [s, q2]])."""
    return float(_load().nko_relu_dot(float(s), float(q1), float(q2)))


def _check_images(x: np.ndarray) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float32)
    if x.ndim != 4:
        raise ValueError("images must be (n, H, W, C)")
    return x


def myrtle_qmaps_len(h: int, w: int, net: Myrtle) -> int:
    d = np.ascontiguousarray(net.depth, dtype=np.int32)
    return int(_load().nko_myrtle_qmaps_len(h, w, net.n_stages, _ptr(d)))


def myrtle_self(x: np.ndarray, net: Myrtle, threads: int | None = None):
    """Variance maps (n, qlen) and self kernel K(x, x) (n,) of each image."""
    x = _check_images(x)
    n, h, w, c = x.shape
    d = np.ascontiguousarray(net.depth, dtype=np.int32)
    qlen = myrtle_qmaps_len(h, w, net)
    q = np.zeros((n, qlen), dtype=np.float64)
    k = np.zeros(n, dtype=np.float64)
    rc = _load().nko_myrtle_self(_ptr(x), n, h, w, c, net.n_stages, _ptr(d), net.sigma_w2, net.sigma_b2,
                                 _ptr(q), _ptr(k), threads or default_threads())
    if rc != 0:
        raise ValueError(f"oracle nko_myrtle_self failed ({rc})")
    return q, k


def myrtle_pairs(x1: np.ndarray, x2: np.ndarray, pairs: np.ndarray, net: Myrtle, q1=None, q2=None,
                 threads: int | None = None) -> np.ndarray:
    """K(x1[a], x2[b]) for each row (a, b) of ``pairs`` (float64)."""
    x1 = _check_images(x1)
    x2 = _check_images(x2)
    n1, h, w, c = x1.shape
    if x2.shape[1:] != (h, w, c):
        raise ValueError("image shapes differ")
    pairs = np.ascontiguousarray(pairs, dtype=np.int64).reshape(-1, 2)
    if pairs.size and (pairs[:, 0].min() < 0 or pairs[:, 0].max() >= n1 or pairs[:, 1].min() < 0
                       or pairs[:, 1].max() >= x2.shape[0]):
        raise IndexError("pair index out of range")
    thr = threads or default_threads()
    # self recursions only for the images the pairs touch
    ua, ia = np.unique(pairs[:, 0], return_inverse=True)
    ub, ib = np.unique(pairs[:, 1], return_inverse=True)
    if q1 is None:
        q1s, _ = myrtle_self(x1[ua], net, thr)
    else:
        q1s = np.ascontiguousarray(q1[ua])
    if q2 is None:
        q2s, _ = myrtle_self(x2[ub], net, thr)
    else:
        q2s = np.ascontiguousarray(q2[ub])
    xs1 = np.ascontiguousarray(x1[ua])
    xs2 = np.ascontiguousarray(x2[ub])
    local = np.ascontiguousarray(np.stack([ia, ib], axis=1).astype(np.int64))
    out = np.zeros(len(local), dtype=np.float64)
    d = np.ascontiguousarray(net.depth, dtype=np.int32)
    rc = _load().nko_myrtle_pairs(_ptr(xs1), _ptr(q1s), _ptr(xs2), _ptr(q2s), h, w, c, net.n_stages, _ptr(d),
                                  net.sigma_w2, net.sigma_b2, _ptr(local), len(local), _ptr(out), thr)
    if rc != 0:
        raise ValueError(f"oracle nko_myrtle_pairs failed ({rc})")
    return out


def myrtle_gram(x1: np.ndarray, x2: np.ndarray | None, net: Myrtle, threads: int | None = None) -> np.ndarray:
    """Full Gram block (float64).  ``x2 is None`` means the symmetric x1 x x1 block."""
    if x2 is None:
        n = x1.shape[0]
        iu = np.triu_indices(n)
        pairs = np.stack(iu, axis=1)
        v = myrtle_pairs(x1, x1, pairs, net, threads=threads)
        K = np.zeros((n, n))
        K[iu] = v
        K[(iu[1], iu[0])] = v
        return K
    n1, n2 = x1.shape[0], x2.shape[0]
    a, b = np.meshgrid(np.arange(n1), np.arange(n2), indexing="ij")
    pairs = np.stack([a.ravel(), b.ravel()], axis=1)
    return myrtle_pairs(x1, x2, pairs, net, threads=threads).reshape(n1, n2)


def myrtle_ntk_pairs(x1: np.ndarray, x2: np.ndarray, pairs: np.ndarray, net: Myrtle, q1=None, q2=None,
                     threads: int | None = None):
    """(NNGP, NTK) of (x1[a], x2[b]) for each row (a, b) of ``pairs`` (float64)."""
    x1 = _check_images(x1)
    x2 = _check_images(x2)
    n1, h, w, c = x1.shape
    if x2.shape[1:] != (h, w, c):
        raise ValueError("image shapes differ")
    pairs = np.ascontiguousarray(pairs, dtype=np.int64).reshape(-1, 2)
    if pairs.size and (pairs[:, 0].min() < 0 or pairs[:, 0].max() >= n1 or pairs[:, 1].min() < 0
                       or pairs[:, 1].max() >= x2.shape[0]):
        raise IndexError("pair index out of range")
    thr = threads or default_threads()
    ua, ia = np.unique(pairs[:, 0], return_inverse=True)
    ub, ib = np.unique(pairs[:, 1], return_inverse=True)
    q1s = myrtle_self(x1[ua], net, thr)[0] if q1 is None else np.ascontiguousarray(q1[ua])
    q2s = myrtle_self(x2[ub], net, thr)[0] if q2 is None else np.ascontiguousarray(q2[ub])
    xs1 = np.ascontiguousarray(x1[ua])
    xs2 = np.ascontiguousarray(x2[ub])
    local = np.ascontiguousarray(np.stack([ia, ib], axis=1).astype(np.int64))
    kn = np.zeros(len(local), dtype=np.float64)
    kt = np.zeros(len(local), dtype=np.float64)
    d = np.ascontiguousarray(net.depth, dtype=np.int32)
    rc = _load().nko_myrtle_ntk_pairs(_ptr(xs1), _ptr(q1s), _ptr(xs2), _ptr(q2s), h, w, c, net.n_stages, _ptr(d),
                                      net.sigma_w2, net.sigma_b2, _ptr(local), len(local), _ptr(kn), _ptr(kt), thr)
    if rc != 0:
        raise ValueError(f"oracle nko_myrtle_ntk_pairs failed ({rc})")
    return kn, kt


def myrtle_ntk_gram(x1: np.ndarray, x2: np.ndarray | None, net: Myrtle, threads: int | None = None):
    """(NNGP, NTK) Gram blocks (float64); ``x2 is None`` means x1 x x1."""
    if x2 is None:
        n = x1.shape[0]
        iu = np.triu_indices(n)
        kn, kt = myrtle_ntk_pairs(x1, x1, np.stack(iu, axis=1), net, threads=threads)
        out = []
        for v in (kn, kt):
            K = np.zeros((n, n))
            K[iu] = v
            K[(iu[1], iu[0])] = v
            out.append(K)
        return out[0], out[1]
    n1, n2 = x1.shape[0], x2.shape[0]
    a, b = np.meshgrid(np.arange(n1), np.arange(n2), indexing="ij")
    kn, kt = myrtle_ntk_pairs(x1, x2, np.stack([a.ravel(), b.ravel()], axis=1), net, threads=threads)
    return kn.reshape(n1, n2), kt.reshape(n1, n2)


def fc_nngp(x1: np.ndarray, x2: np.ndarray, depth: int = 3, sigma_w2: float = 2.0, sigma_b2: float = 0.01,
            threads: int | None = None) -> np.ndarray:
    """FC NNGP Gram block on flattened inputs (float64)."""
    a = np.ascontiguousarray(np.asarray(x1, dtype=np.float32).reshape(x1.shape[0], -1))
    b = np.ascontiguousarray(np.asarray(x2, dtype=np.float32).reshape(x2.shape[0], -1))
    if a.shape[1] != b.shape[1]:
        raise ValueError("feature sizes differ")
    K = np.zeros((a.shape[0], b.shape[0]), dtype=np.float64)
    rc = _load().nko_fc_nngp(_ptr(a), a.shape[0], _ptr(b), b.shape[0], a.shape[1], depth, sigma_w2, sigma_b2,
                             _ptr(K), threads or default_threads())
    if rc != 0:
        raise ValueError(f"oracle nko_fc_nngp failed ({rc})")
    return K


def cv_self(x: np.ndarray, depth: int = 8, sigma_w2: float = 2.0, sigma_b2: float = 0.01,
            threads: int | None = None):
    """CNN-VEC variance maps (n, depth, h*w) and self kernels K(x, x) (n,)."""
    x = _check_images(x)
    n, h, w, c = x.shape
    q = np.zeros((n, depth, h * w), dtype=np.float64)
    k = np.zeros(n, dtype=np.float64)
    rc = _load().nko_cv_self(_ptr(x), n, h, w, c, depth, sigma_w2, sigma_b2, _ptr(q), _ptr(k),
                             threads or default_threads())
    if rc != 0:
        raise ValueError(f"oracle nko_cv_self failed ({rc})")
    return q, k


def cv_pairs(x1: np.ndarray, x2: np.ndarray, pairs: np.ndarray, depth: int = 8, sigma_w2: float = 2.0,
             sigma_b2: float = 0.01, q1=None, q2=None, threads: int | None = None) -> np.ndarray:
    """CNN-VEC NNGP K(x1[a], x2[b]) for each row (a, b) of ``pairs`` (float64)."""
    x1 = _check_images(x1)
    x2 = _check_images(x2)
    n1, h, w, c = x1.shape
    if x2.shape[1:] != (h, w, c):
        raise ValueError("image shapes differ")
    pairs = np.ascontiguousarray(pairs, dtype=np.int64).reshape(-1, 2)
    if pairs.size and (pairs[:, 0].min() < 0 or pairs[:, 0].max() >= n1 or pairs[:, 1].min() < 0
                       or pairs[:, 1].max() >= x2.shape[0]):
        raise IndexError("pair index out of range")
    if q1 is None:
        q1, _ = cv_self(x1, depth, sigma_w2, sigma_b2, threads)
    if q2 is None:
        q2, _ = cv_self(x2, depth, sigma_w2, sigma_b2, threads)
    q1 = np.ascontiguousarray(q1, dtype=np.float64)
    q2 = np.ascontiguousarray(q2, dtype=np.float64)
    out = np.zeros(pairs.shape[0], dtype=np.float64)
    rc = _load().nko_cv_pairs(_ptr(x1), _ptr(q1), _ptr(x2), _ptr(q2), h, w, c, depth, sigma_w2, sigma_b2,
                              _ptr(pairs), pairs.shape[0], _ptr(out), threads or default_threads())
    if rc != 0:
        raise ValueError(f"oracle nko_cv_pairs failed ({rc})")
    return out


def cv_gram(x1: np.ndarray, x2: np.ndarray | None, depth: int = 8, sigma_w2: float = 2.0, sigma_b2: float = 0.01,
            threads: int | None = None) -> np.ndarray:
    """Full CNN-VEC NNGP block (n1, n2), float64."""
    x2 = x1 if x2 is None else x2
    a, b = np.meshgrid(np.arange(len(x1)), np.arange(len(x2)), indexing="ij")
    pairs = np.stack([a.ravel(), b.ravel()], 1)
    return cv_pairs(x1, x2, pairs, depth, sigma_w2, sigma_b2, threads=threads).reshape(len(x1), len(x2))


def krr_ridge(k_train: np.ndarray, ridge_rel: float) -> float:
    """Ridge lambda = ridge_rel * mean(diag K_train)."""
    return float(ridge_rel) * float(np.mean(np.diag(np.asarray(k_train, dtype=np.float64))))


def krr_predict(k_train: np.ndarray, k_test: np.ndarray, y: np.ndarray, ridge_rel: float) -> np.ndarray:
    """pred = K_test (K_train + lambda I)^{-1} Y, float64 Cholesky solve."""
    import scipy.linalg as sla

    kt = np.asarray(k_train, dtype=np.float64)
    lam = krr_ridge(kt, ridge_rel)
    a = kt + lam * np.eye(kt.shape[0])
    cf = sla.cho_factor(a, lower=True)
    alpha = sla.cho_solve(cf, np.asarray(y, dtype=np.float64))
    return np.asarray(k_test, dtype=np.float64) @ alpha


def krr_mse_loss(k_ss, k_ts, y_s, y_t, lam: float) -> float:
    """Held-out squared error of kernel ridge regression with ridge lam:
    mean((K_ts (K_ss + lam I)^{-1} Y_s - Y_t)^2), float64 Cholesky solve."""
    import scipy.linalg as sla

    a = np.asarray(k_ss, dtype=np.float64) + lam * np.eye(len(k_ss))
    alpha = sla.cho_solve(sla.cho_factor(a, lower=True), np.asarray(y_s, dtype=np.float64))
    r = np.asarray(k_ts, dtype=np.float64) @ alpha - np.asarray(y_t, dtype=np.float64)
    return float(np.mean(r * r))


def krr_mse_cotangents(k_ss, k_ts, y_s, y_t, lam: float):
    """d loss / d K_ss and d loss / d K_ts of krr_mse_loss with lam held fixed
    (reverse mode of the solve: alpha = A^{-1} Y, pred = K_ts alpha)."""
    import scipy.linalg as sla

    a = np.asarray(k_ss, dtype=np.float64) + lam * np.eye(len(k_ss))
    cf = sla.cho_factor(a, lower=True)
    alpha = sla.cho_solve(cf, np.asarray(y_s, dtype=np.float64))
    kts = np.asarray(k_ts, dtype=np.float64)
    r = kts @ alpha - np.asarray(y_t, dtype=np.float64)
    g = 2.0 * r / r.size
    d_ts = g @ alpha.T
    z = sla.cho_solve(cf, kts.T @ g)
    d_ss = -z @ alpha.T
    return d_ss, d_ts
