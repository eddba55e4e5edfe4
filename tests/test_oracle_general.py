"""Pins for the oracle's general visit list (per-visit start time and dwell).

Each visit is the single-probe source of Sec. II with its own dwell, and the
field is their sum (Eq. 6).  Independent checks:
* brute-force time quadrature of the heat kernel for a handful of visits with
  unequal dwells, gaps (flyback / dead time) and repeated positions;
* a uniform scan written as a general list reproduces the scan oracle, which
  derives visit times from indices by its own code;
* splitting a dwell into two back-to-back half dwells at the same position
  leaves the field unchanged (the dose integral is additive in time), during
  and after the beam;
* visit order does not matter; nothing is felt before a visit starts.
"""
import math

import mpmath
import numpy as np
import pytest

SIG, D = 0.5e-9, 2.5e-13


def heat_sum(vis, x, y, t):
    """Sum over visits of Q0 * int_{beam on} Gaussian(var sig^2 + 2 D u) du."""
    mpmath.mp.dps = 30
    Ds = mpmath.mpf(SIG) ** 2
    tot = mpmath.mpf(0)
    for vx, vy, t0, dw in vis:
        if not t0 < t:
            continue
        dt = t - t0
        a = mpmath.mpf(x - vx) ** 2 + mpmath.mpf(y - vy) ** 2

        def g(u):
            var = Ds + 2 * mpmath.mpf(D) * u
            return mpmath.exp(-a / (2 * var)) / (2 * mpmath.pi * var)

        lo = max(0.0, dt - dw)
        tot += mpmath.quad(g, [lo, (lo + dt) / 2, dt])
    return float(tot)


def general(ora, vis, Q0=1.0):
    v = np.asarray(vis, dtype=np.float64)
    return ora.Visits(v[:, 0], v[:, 1], v[:, 2], v[:, 3], SIG, D, Q0)


VIS = [  # x, y, t0, dwell: unequal dwells, a flyback gap, a revisit of (0, 0)
    (0.0, 0.0, 0.0, 1e-6),
    (1e-9, 0.0, 1.0e-6, 0.3e-6),
    (2e-9, 0.5e-9, 1.3e-6, 2.2e-6),
    (0.0, 1e-9, 6.0e-6, 0.7e-6),
    (0.0, 0.0, 6.7e-6, 1.5e-6),
]


@pytest.mark.parametrize("x,y,t", [
    (0.0, 0.0, 0.5e-6), (0.0, 0.0, 6.9e-6), (1.3e-9, 0.2e-9, 3.0e-6),
    (0.5e-9, 0.5e-9, 9.0e-6), (-2e-9, 3e-9, 40e-6), (2e-9, 0.5e-9, 1.3e-6 + 1e-9),
])
def test_general_list_equals_heat_kernel_quadrature(ora, x, y, t):
    got = general(ora, VIS).psi_points([x], [y], [t])[0]
    ref = heat_sum(VIS, x, y, t)
    assert abs(got - ref) <= 1e-12 * abs(ref), (got, ref)


@pytest.mark.parametrize("seed", [0, 1])
def test_uniform_scan_as_general_list(ora, seed):
    nx, ny, pitch, tau = 9, 7, 1e-9, 1e-6
    ids = np.random.default_rng(seed).permutation(nx * ny).astype(np.int32)
    s = ora.Scan(nx, ny, ids, pitch, tau, SIG, D)
    vis = [((i % nx) * pitch, (i // nx) * pitch, k * tau, tau) for k, i in enumerate(ids)]
    g = general(ora, vis)
    a, b = s.psi_arrival(), g.psi_arrival()
    assert np.max(np.abs(a - b) / np.abs(a).max()) <= 1e-13
    ts = [2.5 * tau, 40.4 * tau, nx * ny * tau, 3 * nx * ny * tau]
    m1 = s.psi_map(-1.5e-9, -0.5e-9, 0.7e-9, 0.6e-9, 17, 15, ts)
    m2 = g.psi_map(-1.5e-9, -0.5e-9, 0.7e-9, 0.6e-9, 17, 15, ts)
    assert np.max(np.abs(m1 - m2)) <= 1e-13 * np.abs(m1).max()


def test_split_dwell_is_additive(ora):
    halves = []
    for x, y, t0, dw in VIS:
        halves += [(x, y, t0, dw / 2), (x, y, t0 + dw / 2, dw / 2)]
    rng = np.random.default_rng(3)
    px = rng.uniform(-1e-9, 3e-9, 200)
    py = rng.uniform(-1e-9, 2e-9, 200)
    pt = rng.uniform(0.0, 12e-6, 200)  # inside and after dwells, halves included
    a = general(ora, VIS).psi_points(px, py, pt)
    b = general(ora, halves).psi_points(px, py, pt)
    assert np.max(np.abs(a - b) / np.maximum(np.abs(a), 1e-300)) <= 1e-12


def test_order_free_and_causal(ora):
    rng = np.random.default_rng(4)
    perm = rng.permutation(len(VIS))
    px, py, pt = [0.3e-9, 1e-9], [0.1e-9, 0.8e-9], [4e-6, 7e-6]
    a = general(ora, VIS).psi_points(px, py, pt)
    b = general(ora, [VIS[k] for k in perm]).psi_points(px, py, pt)
    assert np.allclose(a, b, rtol=1e-14, atol=0)
    # nothing before the first visit starts; a visit starting exactly at t adds nothing
    assert general(ora, VIS).psi_points([0.0], [0.0], [0.0])[0] == 0.0
    only_first = general(ora, VIS[:3]).psi_points([0.0], [1e-9], [6.0e-6])[0]
    assert general(ora, VIS).psi_points([0.0], [1e-9], [6.0e-6])[0] == only_first
    # linear in Q0
    q = general(ora, VIS, Q0=2.5).psi_points(px, py, pt)
    assert np.allclose(q, 2.5 * a, rtol=1e-15, atol=0)


def test_bad_arguments(ora):
    with pytest.raises(ValueError):
        ora.Visits([0.0], [0.0], [0.0], [0.0], SIG, D).psi_points([0.0], [0.0], [1.0])
    with pytest.raises(ValueError):
        ora.Visits([0.0], [0.0], [0.0, 1.0], [1e-6], SIG, D)
    with pytest.raises(ValueError):
        ora.Visits([0.0], [0.0], [0.0], [1e-6], -SIG, D).psi_points([0.0], [0.0], [1.0])
    assert math.isfinite(general(ora, VIS).psi_points([0.0], [0.0], [1.0])[0])
