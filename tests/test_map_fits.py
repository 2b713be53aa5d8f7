"""The polynomial fits of the ReLU arc-cosine map that the HIP kernels
evaluate (coefficients in csrc/nk_common.h, written by csrc/gen_relu_poly.py),
checked on the CPU against the closed forms on a dense grid of u = 1 - rho in
[0, 1]:
  J1(rho) = (sin t + (pi - t) rho) / pi,  t = acos(rho)   (the normalised
  arc-cosine map of a ReLU layer; the kernels evaluate 1 - u (1 - sqrt(u) H(u))),
  acos(rho) / pi                                          (its derivative is
  1 - acos(rho) / pi; the kernels evaluate sqrt(u) G(u) / pi).
The bounds are the fits' stated errors with room for the float32 rounding of
the coefficients; a wrong or swapped coefficient fails them by orders of
magnitude."""
import os
import re

import numpy as np
import pytest

HDR = os.path.join(os.path.dirname(__file__), "..", "paper_2303_05420_amd", "csrc", "nk_common.h")


def _coeffs(prefix):
    text = open(HDR).read()
    found = dict((int(k), float(v)) for k, v in re.findall(r"#define\s+" + prefix + r"(\d+)\s+([-+0-9.eE]+)f", text))
    return [found[k] for k in range(len(found))]


def _poly(c, u):
    p = np.full_like(u, c[-1])
    for ck in reversed(c[:-1]):
        p = p * u + ck
    return p


U = np.concatenate([np.linspace(0.0, 1.0, 200001), np.geomspace(1e-12, 1e-3, 2000)])


@pytest.mark.parametrize("prefix,bound", [("NK_J1_C", 3e-7), ("NK_J1D3_C", 2e-6)])
def test_relu_map_fit(prefix, bound):
    c = _coeffs(prefix)
    rho = 1.0 - U
    t = np.arccos(rho)
    exact = (np.sin(t) + (np.pi - t) * rho) / np.pi
    fit = 1.0 - U * (1.0 - np.sqrt(U) * _poly(c, U))
    err = np.max(np.abs(fit - exact) / exact)
    assert err <= bound, err
    # the fit's value at u = 0: H(0) = 2 sqrt(2) / (3 pi)
    assert abs(c[0] - 2 * np.sqrt(2) / (3 * np.pi)) <= 1e-3 * c[0]


@pytest.mark.parametrize("prefix,bound", [("NK_ACOSD5_C", 3e-7), ("NK_ACOSD4_C", 2e-6)])
def test_acos_fit(prefix, bound):
    c = _coeffs(prefix)
    exact = np.arccos(1.0 - U) / np.pi
    fit = np.sqrt(U) * _poly(c, U) / np.pi
    err = np.max(np.abs(fit - exact))
    assert err <= bound, err
    # G(0) = sqrt(2)
    assert abs(c[0] - np.sqrt(2)) <= 1e-4


def test_planted_coefficient_error_is_caught():
    # a swap of two coefficients of the degree-3 map moves it far past its bound
    c = _coeffs("NK_J1D3_C")
    c[1], c[2] = c[2], c[1]
    rho = 1.0 - U
    t = np.arccos(rho)
    exact = (np.sin(t) + (np.pi - t) * rho) / np.pi
    fit = 1.0 - U * (1.0 - np.sqrt(U) * _poly(c, U))
    assert np.max(np.abs(fit - exact) / exact) > 1e-3
