"""Pins for the oracle's kernel pieces: closed forms, integrals, derivatives."""
import json
import math
import os

import numpy as np
import pytest
from scipy import integrate

import oracle

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")))


def test_wendland_c2_closed_forms():
    for rho, val in GOLD["wendland_c2"]["values"]:
        assert oracle.wendland_c2(np.array([rho]))[0] == pytest.approx(val, abs=1e-15)


def test_wendland_c6_closed_forms():
    for rho, val in GOLD["wendland_c6"]["values"]:
        assert oracle.wendland_c6(np.array([rho]))[0] == pytest.approx(val, abs=1e-15)


def test_wendland_strict_support():
    rho = np.array([1.0, np.nextafter(1.0, 2.0), 3.0])
    assert np.all(oracle.wendland_c2(rho) == 0.0)
    assert np.all(oracle.wendland_c2_dr(rho, 0.7) == 0.0)
    assert oracle.wendland_c2(np.array([np.nextafter(1.0, 0.0)]))[0] > 0.0


def test_wendland_integrals():
    """Radial integrals over the unit disk / ball pin the whole polynomial."""
    f2 = lambda p: oracle.wendland_c2(np.array([p]))[0] * p * 2 * math.pi
    f3 = lambda p: oracle.wendland_c2(np.array([p]))[0] * p * p * 4 * math.pi
    v2 = integrate.quad(f2, 0, 1, epsabs=1e-14)[0]
    v3 = integrate.quad(f3, 0, 1, epsabs=1e-14)[0]
    assert v2 == pytest.approx(GOLD["wendland_c2"]["disk_integral_2d"], rel=1e-12)
    assert v3 == pytest.approx(GOLD["wendland_c2"]["ball_integral_3d"], rel=1e-12)


def test_wendland_radius_derivative_closed_form_and_fd():
    for rho, r, val in GOLD["wendland_c2"]["dW_dr"]:
        assert oracle.wendland_c2_dr(np.array([rho]), r)[0] == pytest.approx(val, rel=1e-14)
    # chain rule check against d/drho closed forms: dW/dr = -(rho/r) dW/drho
    for rho, dval in GOLD["wendland_c2"]["dW_drho"]:
        r = 1.7
        assert oracle.wendland_c2_dr(np.array([rho]), r)[0] == pytest.approx(-rho / r * dval, rel=1e-14)
    # central finite differences of W(d / r) in r
    d = np.linspace(0.01, 0.99, 37)
    r = 1.0
    h = 1e-6
    fd = (oracle.wendland_c2(d / (r + h)) - oracle.wendland_c2(d / (r - h))) / (2 * h)
    np.testing.assert_allclose(oracle.wendland_c2_dr(d / r, r), fd, rtol=1e-7, atol=1e-10)


def test_wendland_c6_radius_derivative_and_integral():
    """The printed member (Eq. wendland): d/dr closed form at rho = 1/2, central
    differences in r, and its integral over the unit disk from Beta functions."""
    from fractions import Fraction
    from math import factorial
    import scipy.integrate
    # 22 (1/2)^2 (1/2)^7 (16/4 + 7/2 + 1) / r at r = 2
    assert oracle.wendland_c6_dr(np.array([0.5]), 2.0)[0] == pytest.approx(float(Fraction(22 * 17, 4 * 128 * 2 * 2)),
                                                                            rel=1e-14)
    d = np.linspace(0.01, 0.99, 37)
    h = 1e-6
    fd = (oracle.wendland_c6(d / (1.0 + h)) - oracle.wendland_c6(d / (1.0 - h))) / (2 * h)
    np.testing.assert_allclose(oracle.wendland_c6_dr(d, 1.0), fd, rtol=1e-7, atol=1e-9)  # FD rounding ~eps/h
    # int_0^1 W(rho) rho drho = sum_k c_k B(k + 2, 9) with W = (1-rho)^8 sum_k c_k rho^k
    beta = lambda a, b: Fraction(factorial(a - 1) * factorial(b - 1), factorial(a + b - 1))
    exact = sum(Fraction(c) * beta(k + 2, 9) for k, c in [(0, 1), (1, 8), (2, 25), (3, 32)])
    num, _ = scipy.integrate.quad(lambda t: oracle.wendland_c6(np.array([t]))[0] * t, 0, 1, epsabs=1e-15)
    assert num == pytest.approx(float(exact), rel=1e-12)
    assert oracle.wendland(d, "c6") is not None and np.array_equal(oracle.wendland(d, "c6"), oracle.wendland_c6(d))
    with pytest.raises(ValueError):
        oracle.wendland(d, "c4")


def test_bump_closed_forms():
    w = 0.5
    c = np.array([[0.3, 0.4]])
    for s, val in GOLD["bump"]["values_by_s"]:
        # a point at squared distance s * w^2 along the first axis
        x = np.array([[0.3 + math.sqrt(s) * w, 0.4]])
        g, b, gamma = oracle.bump_values(x, c, w, np.array([1.0]))
        assert b[0, 0] == pytest.approx(val, rel=1e-12, abs=1e-300)
        assert gamma[0] == (s < 1.0)


def test_bump_mask_is_weighted_sum():
    rng = np.random.default_rng(3)
    x = rng.random((50, 3))
    c = rng.random((5, 3))
    wts = rng.uniform(0.5, 1.5, 5)
    g, b, gamma = oracle.bump_values(x, c, 0.4, wts)
    for k in range(5):
        gk, bk, _ = oracle.bump_values(x, c[k:k + 1], 0.4, np.array([1.0]))
        np.testing.assert_array_equal(bk[:, 0], b[:, k])
    np.testing.assert_allclose(g, b @ wts, rtol=0, atol=0)
    assert np.array_equal(gamma, (b > 0).any(axis=1) | gamma)
    # a point outside every bump has g == 0 exactly and gamma false
    far = np.array([[10.0, 10.0, 10.0]])
    g2, _, gam2 = oracle.bump_values(far, c, 0.4, wts)
    assert g2[0] == 0.0 and not gam2[0]
