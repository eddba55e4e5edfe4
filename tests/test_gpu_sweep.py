"""Time-sampled simulation (``dd_damage_sweep``): maps every dt over a whole
scan, mid-dwell times included, against the oracle; equal bit for bit to
``dd_damage_map`` on the same list of times, across the library's time
chunks, and through the host-output path."""
import ctypes

import numpy as np
import pytest

from gpu_util import assert_close, oracle_scan

pytestmark = pytest.mark.gpu
PRECS = ["fp64", "mixed"]


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


@pytest.mark.parametrize("prec", PRECS)
def test_sweep_whole_scan_vs_oracle(dd, ora, wl, prec):
    # 8x8 raster, 32x32 pixels at 0.25 nm, a map every quarter dwell from
    # t = 0 to two dwells past the end of the scan (264 maps)
    spec = wl.small_raster()
    scan = dd.Scan(**spec.kwargs())
    dt = spec.tau_v / 4
    n_t = 4 * spec.n_visits + 8
    got = scan.damage_sweep(0.0, 0.0, 0.25e-9, 0.25e-9, 32, 32, 0.0, dt, n_t, prec).cpu().numpy()
    times = [k * dt for k in range(n_t)]
    ref = oracle_scan(ora, spec, scan).psi_map(0.0, 0.0, 0.25e-9, 0.25e-9, 32, 32, times)
    assert np.all(got[0] == 0.0)  # nothing has started at t = 0
    assert_close(got, ref, spec, prec, "sweep")


@pytest.mark.parametrize("prec", PRECS)
def test_sweep_off_lattice_vs_oracle(dd, ora, wl, prec):
    # three raster frames, a grid offset from the probes, and a step
    # incommensurate with the dwell (a different in-dwell phase every map)
    spec = wl.ScanSpec(6, 5, "multiframe", 1e-9, 3e-6, 0.4e-9, 4e-13, 2.0, frames=3)
    scan = dd.Scan(**spec.kwargs())
    dt = 0.37 * spec.tau_v
    n_t = 260
    args = (0.3e-9, -0.2e-9, 0.45e-9, 0.45e-9, 13, 11)
    got = scan.damage_sweep(*args, 0.05 * spec.tau_v, dt, n_t, prec).cpu().numpy()
    times = [0.05 * spec.tau_v + k * dt for k in range(n_t)]
    ref = oracle_scan(ora, spec, scan).psi_map(*args, times)
    assert_close(got, ref, spec, prec, "off-lattice sweep")
    same = scan.damage_map(*args, times, prec).cpu().numpy()
    assert np.array_equal(got, same)


def test_sweep_chunks_and_host_output(dd, wl):
    # 128x128 pixels: the library takes 2048 times per map call, so 2050
    # times run as two calls; each equals dd_damage_map on its own times
    import torch

    spec = wl.small_raster()
    scan = dd.Scan(**spec.kwargs())
    args = (0.0, 0.0, 0.0625e-9, 0.0625e-9, 128, 128)
    dt = spec.tau_v / 32
    n_t = 2050
    got = scan.damage_sweep(*args, 0.0, dt, n_t, "mixed")
    times = [k * dt for k in range(n_t)]
    first = scan.damage_map(*args, times[:2048], "mixed")
    second = scan.damage_map(*args, times[2048:], "mixed")
    assert torch.equal(got[:2048], first)
    assert torch.equal(got[2048:], second)
    # host output through the C ABI
    lib = dd.load_library()
    host = np.empty((n_t, 128, 128))
    g = dd.Grid(*args)
    torch.cuda.synchronize()
    st = lib.dd_damage_sweep(scan.handle, ctypes.byref(g), 0.0, dt, n_t, 1,
                             host.ctypes.data_as(ctypes.c_void_p), 0, None)
    assert st == dd.DD_OK
    assert np.array_equal(host, got.cpu().numpy())


@pytest.mark.parametrize("prec", PRECS)
def test_bench_sweep_sampled_vs_oracle(dd, ora, wl, prec):
    # the benchmark's sweep in the call it times: 64x64 raster, 128x128 maps
    # at half the pitch every half dwell over the whole scan (8192 maps);
    # 64 sampled (map, pixel) values against the oracle
    import torch

    spec = wl.ScanSpec(64, 64, "raster", 1e-9, 1e-6, 0.5e-9, 2.5e-13, 1.0)
    scan = dd.Scan(**spec.kwargs())
    n_t, w, dt = 2 * spec.n_visits, 128, spec.tau_v / 2
    out = scan.damage_sweep(0.0, 0.0, 0.5e-9, 0.5e-9, w, w, 0.0, dt, n_t, prec)
    rng = np.random.default_rng(41)
    m = rng.integers(0, n_t, 64)
    m[:2] = (n_t - 1, 1)
    u, v = rng.integers(0, w, 64), rng.integers(0, w, 64)
    got = out[torch.as_tensor(m, device="cuda"), torch.as_tensor(v, device="cuda"),
              torch.as_tensor(u, device="cuda")].cpu().numpy()
    del out
    ref = oracle_scan(ora, spec, scan).psi_points(u * 0.5e-9, v * 0.5e-9, m * dt)
    assert_close(got, ref, spec, prec, "bench sweep (sampled)")
