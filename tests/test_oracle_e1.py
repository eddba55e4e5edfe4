"""Pins for the oracle's exponential integral E1 (definition after Eq. 2, Sec. II).

E1 is computed three independent ways (power series, continued fraction,
quadrature of the defining integral) and checked against two libraries
(mpmath at 40 digits, scipy) and against properties fixed by the mathematics:
the integral of E1 over (0, inf) is 1, E1'(x) = -exp(-x)/x, and the small- and
large-argument asymptotes.  A dropped term, a wrong sign or a wrong Euler
constant in any one form breaks at least one of these.
"""
import math

import mpmath
import numpy as np
import pytest
import scipy.integrate
import scipy.special

XS = np.concatenate([np.geomspace(1e-12, 1e-2, 11), np.linspace(0.05, 4, 40),
                     np.geomspace(4.5, 700, 25)])


def test_matches_mpmath(ora):
    mpmath.mp.dps = 40
    for x in XS:
        ref = float(mpmath.e1(mpmath.mpf(float(x))))
        assert abs(ora.e1(float(x)) - ref) <= 2.5e-16 * ref, x


def test_matches_scipy(ora):
    for x in XS:
        ref = scipy.special.exp1(x)
        assert abs(ora.e1(float(x)) - ref) <= 4e-15 * ref, x


@pytest.mark.parametrize("x", [0.2, 0.5, 0.9, 1.0, 1.1, 1.7, 2.5, 3.5])
def test_series_cf_quadrature_agree(ora, x):
    s, c, q = ora.e1_series(x), ora.e1_cf(x), ora.e1_quad(x)
    assert abs(s - c) <= 1e-15 * c
    assert abs(q - c) <= 1e-15 * c


@pytest.mark.parametrize("x", [1e-9, 1e-3, 0.3, 3.0, 30.0, 300.0, 650.0])
def test_quadrature_everywhere(ora, x):
    assert abs(ora.e1_quad(x) - ora.e1(x)) <= 1e-15 * ora.e1(x)


def test_integral_is_one(ora):
    # int_0^inf E1(x) dx = 1; the log singularity at 0 is integrable.
    a, _ = scipy.integrate.quad(ora.e1, 0, 1, limit=200)
    b, _ = scipy.integrate.quad(ora.e1, 1, 60, limit=200)
    assert abs(a + b - 1.0) < 1e-9


@pytest.mark.parametrize("x", [0.01, 0.4, 0.99, 1.01, 2.0, 8.0, 40.0])
def test_derivative(ora, x):
    h = 1e-3 * x  # fourth-order central stencil
    d = (8 * (ora.e1(x + h) - ora.e1(x - h)) - (ora.e1(x + 2 * h) - ora.e1(x - 2 * h))) / (12 * h)
    exact = -math.exp(-x) / x
    assert abs(d - exact) <= 1e-7 * abs(exact)


def test_small_argument_asymptote(ora):
    # E1(x) = -gamma - ln x + x - x^2/4 + O(x^3)
    for x in (1e-6, 1e-4, 1e-3):
        approx = -np.euler_gamma - math.log(x) + x - x * x / 4
        assert abs(ora.e1(x) - approx) <= x ** 3 + 4e-16 * abs(approx)


def test_large_argument_asymptote(ora):
    # x e^x E1(x) = 1 - 1/x + 2/x^2 - 6/x^3 + O(x^-4)
    for x in (50.0, 200.0, 600.0):
        lhs = x * math.exp(x) * ora.e1(x) if x < 700 else None
        approx = 1 - 1 / x + 2 / x ** 2 - 6 / x ** 3
        assert abs(lhs - approx) <= 30 / x ** 4


def test_binary128_e1_matches_mpmath(ora):
    mpmath.mp.dps = 40
    for x in XS:
        ref = float(mpmath.e1(mpmath.mpf(float(x))))
        assert abs(ora.e1_q(float(x)) - ref) <= 1.2e-16 * ref, x


@pytest.mark.parametrize("a,dt,tau,sig,D", [
    (5.0, 1e-3, 1.0, 1.0, 1e-4),      # E1 arguments differ by 1 part in 5e6
    (1e5, 1e5, 1.0, 0.4, 0.5),        # far lag, far probe
    (0.25, 3e5, 1.0, 0.4, 0.5),       # far lag, near probe
    (2.0, 1.0, 1.0, 0.2, 1e-4),
])
def test_binary128_bracket_resolves_cancellation(ora, a, dt, tau, sig, D):
    # E1(a/b1) - E1(a/b0) at 60 digits; the binary128 bracket keeps ~1e-16
    mpmath.mp.dps = 60
    Ds = mpmath.mpf(sig) ** 2
    b1 = 2 * Ds + 4 * mpmath.mpf(D) * mpmath.mpf(dt)
    b0 = 2 * Ds + 4 * mpmath.mpf(D) * max(mpmath.mpf(dt) - mpmath.mpf(tau), 0)
    ref = float(mpmath.e1(mpmath.mpf(a) / b1) - mpmath.e1(mpmath.mpf(a) / b0))
    assert abs(ora.phi_bracket_q(a, dt, tau, sig, D) - ref) <= 2e-16 * ref
    # the long-double bracket agrees within its cancellation-limited accuracy
    ld = ora.phi(a, dt, tau, sig, D, 4 * math.pi * D)
    cond = float(mpmath.e1(mpmath.mpf(a) / b1)) / ref
    assert abs(ld - ref) <= 4e-18 * cond * ref + 4e-16 * ref
