"""Generates the float32 coefficients of the ReLU arc-cosine map used by the
HIP kernels (nk_common.h, NK_J1_C0..NK_J1_C5).

For cos t = rho in [0, 1] write u = 1 - rho.  The normalised map
J1(rho) = (sin t + (pi - t) rho) / pi satisfies J1 = rho + u^{3/2} H(u) with H
analytic on [0, 1] (H(0) = 2 sqrt(2) / (3 pi)): sin t - t cos t is t^3 times
an even series and t^2 is u times an analytic series.  H is fitted by a
polynomial of degree 5 minimising the maximum relative error of J1 (weight
u^{3/2} / J1), using Lawson's iteratively reweighted least squares on 4000
Chebyshev points, with H evaluated in 40-digit arithmetic.  Negative rho uses
J1(rho) = J1(|rho|) - |rho|, so the same polynomial covers [-1, 1].

Run: python gen_relu_poly.py  (prints the coefficients and the fit error).
"""
import mpmath as mp
import numpy as np


def main(degree: int = 5, m: int = 4000):
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
        print(f"#define NK_J1_C{k} {float(ck)!r}f")


if __name__ == "__main__":
    main()
