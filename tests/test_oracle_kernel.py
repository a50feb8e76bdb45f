"""Pins of the oracle's cubic B-spline (section 3.1.1) against mathematics, not against
its own formula: normalisation of the 3-D kernel by quadrature with the paper's
printed constant, derivative consistency by finite differences, continuity of the
pieces, compact support."""
import json
import math
import os

import numpy as np
import pytest
from scipy import integrate

from oracle import native

GOLD = os.path.join(os.path.dirname(__file__), "golden", "kernel_constants.json")


@pytest.mark.parametrize("h", [1.0, 0.15, 2.4 / 128.0, 3.7])
def test_normalisation_3d(h):
    # integral of W over R^3 = 1 (the defining property of the constant s = 8/pi)
    # each piece of r^2 W(r) is a polynomial of degree 5: 8-point Gauss-Legendre per
    # piece is exact; scipy's adaptive quadrature must agree
    f = lambda r: 4.0 * math.pi * r * r * native.kernel(r, h)[0]
    xg, wg = np.polynomial.legendre.leggauss(8)
    val = 0.0
    for a, b in ((0.0, 0.5 * h), (0.5 * h, h)):
        val += 0.5 * (b - a) * sum(wi * f(0.5 * (b - a) * xi + 0.5 * (b + a)) for xi, wi in zip(xg, wg))
    assert abs(val - 1.0) < 1e-13
    q, _ = integrate.quad(f, 0.0, h, points=[0.5 * h], epsabs=0, epsrel=1e-12, limit=200)
    assert abs(q - 1.0) < 1e-11


def test_printed_constant_is_the_3d_one():
    g = json.load(open(GOLD))
    assert abs(g["s_value"]["3"] - 8.0 / math.pi) < 1e-15
    # W(0) = s/h^3 for the 3-D constant printed in the paper
    h = 0.7
    assert abs(native.kernel(0.0, h)[0] * h ** 3 - g["s_value"]["3"]) < 1e-14


@pytest.mark.parametrize("h", [1.0, 0.15])
def test_derivative_matches_finite_difference(h):
    rs = np.linspace(0.01, 0.99, 97) * h
    for r in rs:
        if abs(r / h - 0.5) < 1e-3:
            continue
        e = 1e-6 * h
        fd = (native.kernel(r + e, h)[0] - native.kernel(r - e, h)[0]) / (2 * e)
        dw = native.kernel(r, h)[1]
        scale = 6 * (8 / math.pi) / h ** 4
        assert abs(fd - dw) < 1e-7 * scale


def test_continuity_and_support():
    h = 1.3
    e = 1e-12
    wl, dl = native.kernel(0.5 * h - e * h, h)
    wr, dr = native.kernel(0.5 * h, h)
    s = 8 / math.pi
    assert abs(wl - wr) < 1e-9 * s / h ** 3
    assert abs(dl - dr) < 1e-9 * s / h ** 4
    # second derivative (finite differences of dW) agrees on both sides of q = 1/2
    d = 1e-5 * h
    d2l = (native.kernel(0.5 * h - d, h)[1] - native.kernel(0.5 * h - 2 * d, h)[1]) / d
    d2r = (native.kernel(0.5 * h + 2 * d, h)[1] - native.kernel(0.5 * h + d, h)[1]) / d
    assert abs(d2l - d2r) < 1e-3 * s / h ** 5 * 6
    # vanishes with its first derivative at the support radius and beyond
    assert native.kernel(h, h) == (0.0, 0.0)
    assert native.kernel(1.5 * h, h) == (0.0, 0.0)
    w1, d1 = native.kernel(h * (1 - 1e-4), h)
    assert 0 < w1 < 1e-10 * s / h ** 3 and -1e-6 * s / h ** 4 < d1 < 0


def test_shape():
    h = 1.0
    r = np.linspace(0, 0.999, 500)
    W = np.array([native.kernel(x, h)[0] for x in r])
    D = np.array([native.kernel(x, h)[1] for x in r])
    assert np.all(W > 0) and np.all(np.diff(W) < 0)
    assert D[0] == 0.0 and np.all(D[1:] < 0)
