"""Generates the float32 coefficients of the ReLU arc-cosine map used by the
HIP kernels (nk_common.h: NK_J1_C0..NK_J1_C4 of the degree-4 fit,
NK_J1D3_C0..NK_J1D3_C3 of the degree-3 fit, NK_ACOSD5_C0..C5 and
NK_ACOSD4_C0..C4 of the angle).

For cos t = rho in [0, 1] write u = 1 - rho.  The normalised map
J1(rho) = (sin t + (pi - t) rho) / pi satisfies J1 = rho + u^{3/2} H(u) with H
analytic on [0, 1] (H(0) = 2 sqrt(2) / (3 pi)): sin t - t cos t is t^3 times
an even series and t^2 is u times an analytic series.  H is fitted by a
polynomial of degree 4 (and one of degree 3) minimising the maximum relative error of J1 (weight
u^{3/2} / J1), using Lawson's iteratively reweighted least squares on 4000
Chebyshev points, with H evaluated in 40-digit arithmetic.  Negative rho uses
J1(rho) = J1(|rho|) - |rho|, so the same polynomial covers [-1, 1].

The adjoint needs dJ1/drho = (pi - t) / pi with t = acos(rho).  For
rho = 1 - u, t = sqrt(u) G(u) with G analytic on [0, 1] (G(0) = sqrt 2);
G is fitted by a degree-5 polynomial minimising the maximum absolute error of
sqrt(u) G(u) / pi (Lawson again; 2.0e-7) for the adjoint (NK_ACOSD5_C0..C5),
and by one of degree 4 (1.5e-6) for the tangent kernel's forward pass
(NK_ACOSD4_C0..C4); negative rho uses acos(-r) = pi - acos(r).

Run: python gen_relu_poly.py  (prints the coefficients and the fit errors).
"""
import mpmath as mp
import numpy as np


def main(degree: int = 4, m: int = 4000, prefix: str = "NK_J1_C"):
    mp.mp.dps = 40

    def j1(rho):
        th = mp.acos(rho)
        return (mp.sin(th) + (mp.pi - th) * rho) / mp.pi

    def h(u):
        u = mp.mpf(u)
        if u == 0:
            return 2 * mp.sqrt(2) / (3 * mp.pi)
        return (j1(1 - u) - (1 - u)) / u ** mp.mpf(1.5)

    us = (1 - np.cos(np.pi * (np.arange(m) + 0.5) / m)) / 2
    us = np.concatenate([[0.0], us, [1.0]])
    hs = np.array([float(h(u)) for u in us])
    js = (1 - us) + us ** 1.5 * hs
    w = us ** 1.5 / js
    v = np.vander(us, degree + 1, increasing=True)
    lw = np.ones(len(us)) / len(us)
    for _ in range(500):
        sw = np.sqrt(lw) * w
        c, *_ = np.linalg.lstsq(v * sw[:, None], hs * sw, rcond=None)
        e = np.abs((v @ c - hs) * w)
        lw = lw * e
        lw /= lw.sum()
    print(f"max relative error of J1 (float64 evaluation): {e.max():.3e}")
    for k, ck in enumerate(c.astype(np.float32)):
        print(f"#define {prefix}{k} {float(ck)!r}f")


def main_acos(degree: int = 5, m: int = 3000, prefix: str = "NK_ACOSD5_C"):
    mp.mp.dps = 40

    def g(u):
        u = mp.mpf(u)
        if u == 0:
            return mp.sqrt(2)
        return mp.acos(1 - u) / mp.sqrt(u)

    us = (1 - np.cos(np.pi * (np.arange(m) + 0.5) / m)) / 2
    us = np.concatenate([[0.0], us, [1.0]])
    gs = np.array([float(g(u)) for u in us])
    w = np.sqrt(us) / np.pi
    v = np.vander(us, degree + 1, increasing=True)
    lw = np.ones(len(us)) / len(us)
    for _ in range(400):
        sw = np.sqrt(lw) * np.maximum(w, 1e-3)
        c, *_ = np.linalg.lstsq(v * sw[:, None], gs * sw, rcond=None)
        e = np.abs((v @ c - gs) * w)
        lw = lw * np.maximum(e, 1e-30)
        lw /= lw.sum()
    print(f"max absolute error of dJ1/drho (float64 evaluation): {e.max():.3e}")
    for k, ck in enumerate(c.astype(np.float32)):
        print(f"#define {prefix}{k} {float(ck)!r}f")


if __name__ == "__main__":
    main()
    main(3, prefix="NK_J1D3_C")
    main_acos()
    main_acos(4, prefix="NK_ACOSD4_C")
