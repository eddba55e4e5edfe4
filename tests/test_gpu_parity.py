"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Tolerances: 1e-10 relative for the FP64 path and 1e-6 for the mixed path,
per element, with values below a floor (1e-250 resp. 1e-30 times Q0/(4 pi D))
compared absolutely.  Inputs come from paper_2507_00294_amd.workloads."""
import math

import numpy as np
import pytest

from gpu_util import TOL, assert_close, oracle_scan, rel_err

pytestmark = pytest.mark.gpu

PRECS = ("fp64", "mixed")


@pytest.fixture(scope="module")
def dd():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2507_00294_amd as dd

    dd.load_library()
    return dd


@pytest.fixture(scope="module")
def wl():
    from paper_2507_00294_amd import workloads

    return workloads


# ---------------------------------------------------------------------------
# pair terms: device E1 difference against the oracle's single-visit field
A_VALUES = [0.0, 0.0625, 0.25, 1.0, 2.0, 5.0, 13.0, 100.0, 1.0e3, 1.0e4, 1.0e5, 522242.0]
LAGS = [1e-3, 0.3, 1.0, 1.5, 2.0, 7.0, 100.0, 1e4, 262143.0]


@pytest.mark.parametrize("kappa", [1e-4, 1e-2, 0.25, 0.5, 10.0, 100.0])
@pytest.mark.parametrize("sigma_hat", [0.2, 0.5, 1.0])
def test_pair_terms(dd, ora, kappa, sigma_hat):
    import torch

    a, lag = np.meshgrid(np.array(A_VALUES), np.array(LAGS), indexing="ij")
    a, lag = a.ravel(), lag.ravel()
    # oracle bracket of Eqs. 1-4 in binary128 (units pitch = tau = 1, D = kappa),
    # which resolves the nearly coincident E1 pairs the long-double form cannot
    ref = np.array([ora.phi_bracket_q(x, t, 1.0, sigma_hat, kappa) for x, t in zip(a, lag)])
    for prec, floor in (("fp64", 1e-290), ("mixed", 1e-36)):
        got = dd.pair_terms(kappa, sigma_hat, torch.tensor(a, device="cuda"),
                            torch.tensor(lag, device="cuda"), prec).cpu().numpy()
        tol = 1e-12 if prec == "fp64" else 1e-6
        err = np.abs(got - ref) / np.maximum(np.abs(ref), floor)
        k = int(err.argmax())
        assert err.max() <= tol, (prec, a[k], lag[k], got[k], ref[k], err[k])


# ---------------------------------------------------------------------------
# small raster: 64 maps of 32x32 at the end of every dwell, and arrival
@pytest.mark.parametrize("prec", PRECS)
def test_small_raster_maps(dd, ora, wl, prec):
    spec = wl.small_raster()
    scan = dd.Scan(**spec.kwargs())
    m = wl.small_raster_maps(spec)
    got = scan.damage_map(m.x0_m, m.y0_m, m.dx_m, m.dy_m, m.w, m.h, m.times_s, prec).cpu().numpy()
    ref = oracle_scan(ora, spec, scan).psi_map(m.x0_m, m.y0_m, m.dx_m, m.dy_m, m.w, m.h,
                                                        m.times_s)
    assert_close(got, ref, spec, prec, "small raster maps")


@pytest.mark.parametrize("prec", PRECS)
def test_small_raster_arrival(dd, ora, wl, prec):
    spec = wl.small_raster()
    scan = dd.Scan(**spec.kwargs())
    got = scan.arrival(prec).cpu().numpy()
    ref = oracle_scan(ora, spec, scan).psi_arrival()
    assert got[0] == 0.0
    assert_close(got, ref, spec, prec, "small raster arrival")


# ---------------------------------------------------------------------------
# 32x32 raster and interleaved scans, D log-uniform: arrival for all 16 scans,
# 128x128 final map for one scan of each order
@pytest.mark.parametrize("prec", PRECS)
def test_medium_arrival(dd, ora, wl, prec):
    for spec in wl.medium_scans():
        scan = dd.Scan(**spec.kwargs())
        got = scan.arrival(prec).cpu().numpy()
        ref = oracle_scan(ora, spec, scan).psi_arrival()
        assert_close(got, ref, spec, prec, f"medium arrival D={spec.D_m2s:.3e} {spec.order}")


@pytest.mark.parametrize("prec", PRECS)
def test_medium_final_map(dd, ora, wl, prec):
    specs = wl.medium_scans()
    for spec in (specs[0], specs[-1]):
        scan = dd.Scan(**spec.kwargs())
        m = wl.medium_final_map(spec)
        got = scan.damage_map(m.x0_m, m.y0_m, m.dx_m, m.dy_m, m.w, m.h, m.times_s,
                              prec).cpu().numpy()
        ref = oracle_scan(ora, spec, scan).psi_map(m.x0_m, m.y0_m, m.dx_m, m.dy_m, m.w,
                                                            m.h, m.times_s)
        assert_close(got, ref, spec, prec, "medium final map")


# ---------------------------------------------------------------------------
# 512x512 random scan at full size, sampled against the oracle, in the launch
# configuration the benchmark times
@pytest.fixture(scope="module")
def large_random_oracle(dd, ora, wl):
    """The oracle at 2048 stratified visits of the 512x512 random scan (one
    per 128-visit stratum, first and last included): about 2.7e8 pairs."""
    spec = wl.large_random()
    scan = dd.Scan(**spec.kwargs())
    idx = wl.stratified_visits(spec.n_visits, 2048, seed=31)
    assert idx.size == 2048
    return spec, scan, idx, oracle_scan(ora, spec, scan).psi_arrival(idx)


@pytest.mark.parametrize("prec", PRECS)
def test_large_random_sampled(large_random_oracle, prec):
    spec, scan, idx, ref = large_random_oracle
    got = scan.arrival(prec).cpu().numpy()
    assert_close(got[idx], ref, spec, prec, "large random arrival (2048 stratified visits)")
    assert np.all(got >= 0) and np.all(np.isfinite(got))


def test_large_random_mixed_vs_fp64(dd, wl):
    spec = wl.large_random()
    scan = dd.Scan(**spec.kwargs())
    g64 = scan.arrival("fp64").cpu().numpy()
    g32 = scan.arrival("mixed").cpu().numpy()
    err = rel_err(g32, g64, spec, "mixed")
    assert err.max() <= TOL["mixed"], float(err.max())


# The far rows of long lags take the lighter mixed forms: without the
# exponent's rounding correction where every pair has x1 log2(e) <= 8, and
# the folded single exponential where it is <= 4 and dx <= 2e-4.  128x128
# random scans: at D = 1e-13 no row qualifies (the full form alone), at
# 1e-12 and 1e-11 the rows from about lag 3000 resp. 300 on do.
@pytest.mark.parametrize("D", [1e-13, 1e-12, 1e-11])
def test_long_lag_forms(dd, ora, wl, D):
    spec = wl.ScanSpec(128, 128, "random", 1e-9, 0.5e-6, 0.4e-9, D, 1.0, seed=9)
    scan = dd.Scan(**spec.kwargs())
    idx = wl.stratified_visits(spec.n_visits, 512, seed=41)
    ref = oracle_scan(ora, spec, scan).psi_arrival(idx)
    got = scan.arrival("mixed").cpu().numpy()
    assert_close(got[idx], ref, spec, "mixed", f"long-lag forms, D {D}")
    g64 = scan.arrival("fp64").cpu().numpy()
    assert rel_err(got, g64, spec, "mixed").max() <= TOL["mixed"]
    # the far launch's algorithmic FLOPs per pair show which forms ran: the
    # full form takes at least 15 (degree <= 1), the lighter ones 9 + 2M
    # and 9
    import torch

    dd.profile_read("arrival_far", reset=True)
    dd.profiling(True)
    try:
        again = scan.arrival("mixed").cpu().numpy()
        torch.cuda.synchronize()
    finally:
        dd.profiling(False)
    st = dd.profile_read("arrival_far", reset=True)
    assert np.array_equal(again, got)
    fpp = st["flops"] / st["pairs"]
    if D < 1e-12:
        assert fpp >= 15.0, fpp
    else:
        assert fpp < 14.5, fpp


def test_bitwise_reproducible(dd, wl):
    spec = wl.large_random(128)
    scan = dd.Scan(**spec.kwargs())
    for prec in PRECS:
        a = scan.arrival(prec).cpu().numpy()
        b = scan.arrival(prec).cpu().numpy()
        assert np.array_equal(a, b)


# ---------------------------------------------------------------------------
# edge cases
def _both(dd, ora, spec, what):
    scan = dd.Scan(**spec.kwargs())
    ref = oracle_scan(ora, spec, scan).psi_arrival()
    for prec in PRECS:
        got = scan.arrival(prec).cpu().numpy()
        assert_close(got, ref, spec, prec, what)


def test_single_probe(dd, ora, wl):
    spec = wl.ScanSpec(1, 1)
    scan = dd.Scan(**spec.kwargs())
    assert scan.arrival("fp64").cpu().numpy().tolist() == [0.0]
    t = [0.0, 0.25e-6, 1e-6, 3e-6]
    for prec in PRECS:
        got = scan.damage_map(-1e-9, -1e-9, 0.5e-9, 0.5e-9, 5, 5, t, prec).cpu().numpy()
        ref = oracle_scan(ora, spec, scan).psi_map(-1e-9, -1e-9, 0.5e-9, 0.5e-9, 5, 5, t)
        assert_close(got, ref, spec, prec, "single probe map")
        assert np.all(got[0] == 0)


@pytest.mark.parametrize("side", [(1, 2), (3, 1), (17, 5), (23, 29)])
def test_ragged_tiles(dd, ora, wl, side):
    for order in ("raster", "random", "interleaved"):
        _both(dd, ora, wl.ScanSpec(side[0], side[1], order, seed=7, stride=3), f"ragged {order}")


def test_multiframe_revisits(dd, ora, wl):
    spec = wl.ScanSpec(9, 7, "multiframe", dwell_s=2e-6, frames=4, D_m2s=1e-12)
    _both(dd, ora, spec, "multiframe")


def test_explicit_with_repeats(dd, ora, wl):
    spec = wl.ScanSpec(3, 3, "explicit", visits=[4, 4, 0, 8, 4, 2, 2, 6])
    _both(dd, ora, spec, "explicit")


@pytest.mark.parametrize("D,sigma,dwell", [(1e-15, 0.2e-9, 1e-7), (1e-11, 1e-9, 1e-5),
                                           (1e-15, 1e-9, 1e-5), (1e-11, 0.2e-9, 1e-7)])
def test_extreme_physics(dd, ora, wl, D, sigma, dwell):
    for order in ("raster", "random"):
        spec = wl.ScanSpec(40, 40, order, dwell_s=dwell, sigma_m=sigma, D_m2s=D, seed=9)
        _both(dd, ora, spec, f"extreme {order} D={D} s={sigma} dwell={dwell}")


def test_fractional_and_late_times(dd, ora, wl):
    spec = wl.ScanSpec(6, 5, "random", D_m2s=3e-13, seed=5)
    scan = dd.Scan(**spec.kwargs())
    tau = spec.tau_v
    times = [0.0, 0.5 * tau, 1.0 * tau, 2.37 * tau, 17.999 * tau, 30 * tau, 31.5 * tau, 500 * tau]
    ref = oracle_scan(ora, spec, scan).psi_map(0.3e-9, -0.7e-9, 0.37e-9, 0.29e-9, 11, 9,
                                                        times)
    for prec in PRECS:
        got = scan.damage_map(0.3e-9, -0.7e-9, 0.37e-9, 0.29e-9, 11, 9, times, prec).cpu().numpy()
        # pixels off the probes' lattice: mixed maps of such grids run on the
        # FP64 kernels, so both precisions meet their own bound
        tol = TOL[prec]
        err = rel_err(got, ref, spec, prec)
        assert err.max() <= tol, (prec, float(err.max()))
