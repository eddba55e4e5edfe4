"""Pins for the oracle's cumulative sum (Eq. 6) and its scan orders (Sec. I).

* scan orders: hand-written golden lists (tests/golden), permutation and seed
  properties, and the published first outputs of SplitMix64;
* a 2x2 scan evaluated by brute-force heat-kernel time quadrature, summed over
  the visits that started (no E1 anywhere);
* mass balance: the field integrates to Q0 times the dwell time elapsed;
* Fick's second law (Eq. 5): the residual equals the Gaussian source while a
  beam is on and vanishes otherwise;
* mirror symmetry and the similarity scaling of the closed form.
"""
import math
import os

import mpmath
import numpy as np
import pytest
import scipy.integrate

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        rows = [l for l in f if not l.startswith("#") and l.strip()]
    return np.array(" ".join(rows).split(), dtype=np.int32)


def test_interleaved_golden(ora):
    assert np.array_equal(ora.visits(ora.INTERLEAVED, 4, 4, stride=2),
                          _golden("interleaved_4x4_s2.txt"))
    assert np.array_equal(ora.visits(ora.INTERLEAVED, 5, 3, stride=2),
                          _golden("interleaved_5x3_s2.txt"))


def test_raster_and_multiframe(ora):
    assert np.array_equal(ora.visits(ora.RASTER, 3, 2), np.arange(6))
    mf = ora.visits(ora.MULTIFRAME, 3, 2, frames=4)
    assert np.array_equal(mf, np.tile(np.arange(6), 4))


def test_splitmix64_published_outputs(ora):
    # First outputs of SplitMix64 from state 0 (Steele, Lea & Flood 2014;
    # the values printed by the reference implementation).
    assert ora.splitmix64_stream(0, 3) == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4,
                                           0x06C45D188009454F]


def test_random_is_seeded_permutation(ora):
    a = ora.visits(ora.RANDOM, 17, 13, seed=3)
    assert np.array_equal(np.sort(a), np.arange(17 * 13))
    assert np.array_equal(a, ora.visits(ora.RANDOM, 17, 13, seed=3))
    assert not np.array_equal(a, ora.visits(ora.RANDOM, 17, 13, seed=4))
    # position of each id is close to uniform over many seeds (no gross bias)
    counts = np.zeros((5, 5))
    for s in range(2000):
        p = ora.visits(ora.RANDOM, 5, 1, seed=s)
        counts[np.arange(5), p] += 1
    assert np.all(np.abs(counts - 400) < 5 * math.sqrt(400))


def test_bad_order_arguments(ora):
    with pytest.raises(ValueError):
        ora.visits(ora.RASTER, 0, 4)
    with pytest.raises(ValueError):
        ora.visits(ora.MULTIFRAME, 2, 2, frames=0)


# A small physical scan in convenient units (pitch 1, dwell 1).
P, TAU, SIG, DIF, Q0 = 1.0, 1.0, 0.5, 0.25, 2.0


def small_scan(ora, ids, nx=2, ny=2, **kw):
    args = dict(pitch=P, tau_v=TAU, sigma=SIG, D=DIF, Q0=Q0)
    args.update(kw)
    return ora.Scan(nx, ny, ids, **args)


def brute_force_psi(ids, nx, x, y, t):
    """Sum over started visits of a Gaussian source's heat-kernel time integral."""
    mpmath.mp.dps = 25
    total = mpmath.mpf(0)
    for v, pid in enumerate(ids):
        tv = v * TAU
        if not tv < t:
            break
        px, py = (pid % nx) * P, (pid // nx) * P
        a = (x - px) ** 2 + (y - py) ** 2

        def g(s):
            var = SIG ** 2 + 2 * DIF * s
            return mpmath.exp(-a / (2 * var)) / (2 * mpmath.pi * var)

        dt = t - tv
        lo = max(0.0, dt - TAU)
        total += Q0 * mpmath.quad(g, [lo, dt])
    return float(total)


def test_scan_against_brute_force(ora):
    ids = np.array([0, 3, 1, 2], dtype=np.int32)
    s = small_scan(ora, ids)
    pts = [(0.0, 0.0, 0.5), (0.0, 0.0, 2.0), (0.25, 0.75, 3.5), (1.0, 1.0, 4.0),
           (-1.5, 2.0, 9.0), (0.5, 0.5, 1.0)]
    x, y, t = (np.array(c) for c in zip(*pts))
    got = s.psi_points(x, y, t)
    for k, (xx, yy, tt) in enumerate(pts):
        ref = brute_force_psi(ids, 2, xx, yy, tt)
        assert abs(got[k] - ref) <= 1e-12 * ref, (pts[k], got[k], ref)


def test_arrival_excludes_current_visit(ora):
    ids = ora.visits(ora.RASTER, 3, 3)
    s = small_scan(ora, ids, 3, 3)
    arr = s.psi_arrival()
    assert arr[0] == 0.0  # nothing has been deposited before the first visit
    # arrival value at visit j equals psi at (r_j, t_j) over visits < j
    j = 5
    x, y = (ids[j] % 3) * P, (ids[j] // 3) * P
    assert arr[j] == s.psi_points([x], [y], [j * TAU])[0]


@pytest.mark.parametrize("t", [0.5, 2.0, 4.0, 7.0])
def test_mass_balance(ora, t):
    # int psi dA = Q0 * sum_v clip(t - t_v, 0, tau)   (assumptions of Sec. II)
    ids = np.array([0, 3, 1, 2], dtype=np.int32)
    s = small_scan(ora, ids)
    # radial integral per visit of the single-visit field, pi * int phi da
    total = 0.0
    for v in range(len(ids)):
        dt = t - v * TAU
        if dt <= 0:
            continue
        f = lambda a: math.pi * ora.phi(a, dt, TAU, SIG, DIF, Q0)
        total += scipy.integrate.quad(f, 0, np.inf, limit=400, epsabs=0, epsrel=1e-12)[0]
    expect = Q0 * sum(min(max(t - v * TAU, 0.0), TAU) for v in range(len(ids)))
    assert abs(total - expect) <= 1e-9 * expect
    # the same through the map path on a wide, fine grid (trapezoid rule)
    h, half = 0.125, 14.0
    n = int(2 * half / h) + 1
    m = s.psi_map(-half + 0.5, -half + 0.5, h, h, n, n, [t])[0]
    assert abs(m.sum() * h * h - expect) <= 1e-6 * expect


def test_fick_second_law(ora):
    # d psi/dt - D lap psi = Q0 * Gaussian(r - r_active) while a beam is on (Eq. 5)
    ids = np.array([0, 3, 1, 2], dtype=np.int32)
    s = small_scan(ora, ids)
    h, ht = 2e-3, 2e-4
    for (x, y, t, active) in [(0.3, 0.2, 1.5, 3), (1.2, -0.4, 2.6, 1), (0.7, 0.9, 6.0, None)]:
        xs = np.array([x, x + h, x - h, x, x, x, x])
        ys = np.array([y, y, y, y + h, y - h, y, y])
        ts = np.array([t, t, t, t, t, t + ht, t - ht])
        v = s.psi_points(xs, ys, ts)
        lap = (v[1] + v[2] + v[3] + v[4] - 4 * v[0]) / h ** 2
        dpsi = (v[5] - v[6]) / (2 * ht)
        resid = dpsi - DIF * lap
        if active is None:
            src = 0.0
        else:
            ax, ay = (active % 2) * P, (active // 2) * P
            a = (x - ax) ** 2 + (y - ay) ** 2
            src = Q0 * math.exp(-a / (2 * SIG ** 2)) / (2 * math.pi * SIG ** 2)
        scale = max(abs(dpsi), abs(src), 1e-3)
        assert abs(resid - src) <= 2e-4 * scale, (x, y, t, resid, src)


def test_mirror_symmetry(ora):
    nx, ny = 4, 3
    ids = ora.visits(ora.RANDOM, nx, ny, seed=11)
    mirrored = (ids // nx) * nx + (nx - 1 - ids % nx)
    s1, s2 = small_scan(ora, ids, nx, ny), small_scan(ora, mirrored, nx, ny)
    w = 4 * nx - 3
    t = [3.0, 7.5, 12.0]
    m1 = s1.psi_map(0, 0, 0.25, 0.25, w, 4 * ny - 3, t)
    m2 = s2.psi_map(0, 0, 0.25, 0.25, w, 4 * ny - 3, t)
    assert np.allclose(m1, m2[:, :, ::-1], rtol=1e-15, atol=0)
    a1, a2 = s1.psi_arrival(), s2.psi_arrival()
    assert np.allclose(a1, a2, rtol=1e-15, atol=0)


def test_similarity_scaling(ora):
    # psi * 4 pi D / Q0 is unchanged when pitch, sigma and sqrt(D tau) scale together
    ids = ora.visits(ora.INTERLEAVED, 4, 4, stride=2)
    lam = 3.0
    s1 = small_scan(ora, ids, 4, 4)
    s2 = small_scan(ora, ids, 4, 4, pitch=lam * P, sigma=lam * SIG, D=lam ** 2 * DIF)
    a1 = s1.psi_arrival() * 4 * math.pi * DIF / Q0
    a2 = s2.psi_arrival() * 4 * math.pi * lam ** 2 * DIF / Q0
    assert np.allclose(a1, a2, rtol=1e-14, atol=0)


def test_superposition_over_visits(ora):
    # a scan is the sum of its visits (explicit visit lists of one visit each,
    # shifted in time by padding with far-away visits is not needed: phi alone)
    ids = ora.visits(ora.RANDOM, 3, 3, seed=5)
    s = small_scan(ora, ids, 3, 3)
    x, y, t = 0.75, 1.25, 6.3
    tot = sum(ora.phi((x - (i % 3)) ** 2 + (y - (i // 3)) ** 2, t - v * TAU, TAU, SIG, DIF, Q0)
              for v, i in enumerate(ids))
    assert abs(s.psi_points([x], [y], [t])[0] - tot) <= 1e-14 * tot
