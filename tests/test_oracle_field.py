"""Pins for the oracle's single-visit field (Eqs. 1-4) and cumulative sum (Eq. 6).

Independent checks, none of which re-types the closed form:
* brute-force time quadrature of a Gaussian probe (variance r_s^2 per axis)
  spread by the 2-D heat kernel -- the physical model of Sec. II, whose time
  integral Eqs. 1-2 are;
* the a -> 0 limit of Eqs. 1-2 against the log forms Eqs. 3-4;
* continuity of the on/off forms at t = t_i + tau, and zero field at t = t_i;
* the long-time heat-kernel limit;
* linearity in Q0.
"""
import math

import mpmath
import pytest

# Config "plain FP64 8x8" physical parameters (SI).
SIG, D, TAU, Q0 = 0.5e-9, 2.5e-13, 1e-6, 1.0


def heat_quadrature(a, dt, tau, sig, D, Q0):
    """Q0 * int over the dwell of a Gaussian (variance sig^2 + 2D s per axis)."""
    mpmath.mp.dps = 30
    Ds = mpmath.mpf(sig) ** 2
    a = mpmath.mpf(a)

    def g(u):  # u = time since deposition
        var = Ds + 2 * mpmath.mpf(D) * u
        return mpmath.exp(-a / (2 * var)) / (2 * mpmath.pi * var)

    lo = max(0.0, dt - tau)
    return float(Q0 * mpmath.quad(g, [lo, (lo + dt) / 2, dt]))


CASES = [
    # (a in units of pitch^2, dt in units of tau)
    (0.0, 0.3), (0.0, 1.0), (0.0, 2.5), (0.0625, 0.5), (1.0, 1.0), (1.0, 3.0),
    (2.0, 0.01), (5.0, 10.0), (25.0, 40.0), (0.5, 1.0 + 1e-9), (9.0, 200.0),
]


@pytest.mark.parametrize("a_p2,dt_tau", CASES)
def test_closed_form_equals_heat_kernel_quadrature(ora, a_p2, dt_tau):
    a, dt = a_p2 * 1e-18, dt_tau * TAU
    got = ora.phi(a, dt, TAU, SIG, D, Q0)
    ref = heat_quadrature(a, dt, TAU, SIG, D, Q0)
    assert abs(got - ref) <= 1e-13 * abs(ref), (got, ref)


@pytest.mark.parametrize("dt_tau", [0.2, 1.0, 3.0, 50.0])
def test_log_form_is_limit_of_e1_form(ora, dt_tau):
    dt = dt_tau * TAU
    at0 = ora.phi(0.0, dt, TAU, SIG, D, Q0)
    near = ora.phi(1e-32, dt, TAU, SIG, D, Q0)  # a / (2 Ds) ~ 2e-14
    assert abs(at0 - near) <= 1e-11 * at0


def test_on_off_continuity(ora):
    for a in (0.0, 0.3e-18, 4e-18):
        before = ora.phi(a, TAU * (1 - 1e-12), TAU, SIG, D, Q0)
        after = ora.phi(a, TAU * (1 + 1e-12), TAU, SIG, D, Q0)
        assert abs(before - after) <= 1e-9 * abs(before)


def test_zero_before_and_at_start(ora):
    for a in (0.0, 1e-18):
        assert ora.phi(a, 0.0, TAU, SIG, D, Q0) == 0.0
        assert ora.phi(a, -TAU, TAU, SIG, D, Q0) == 0.0


def test_long_time_heat_kernel_limit(ora):
    # dt >> tau, Ds/D: phi -> Q0 tau exp(-a/(4 D dt)) / (4 pi D dt)
    dt = 2e4 * TAU
    for a in (0.0, 1e-17, 1e-14):
        got = ora.phi(a, dt, TAU, SIG, D, Q0)
        lim = Q0 * TAU * math.exp(-a / (4 * D * dt)) / (4 * math.pi * D * dt)
        assert abs(got - lim) <= 2e-4 * lim


def test_linear_in_q0(ora):
    for a in (0.0, 2e-18):
        one = ora.phi(a, 2 * TAU, TAU, SIG, D, 1.0)
        assert abs(ora.phi(a, 2 * TAU, TAU, SIG, D, 7.5) - 7.5 * one) <= 1e-15 * 7.5 * one
