"""Handle behaviour on the GPU: the non-finite output check (dd_scan_check,
host-output calls, batched and general-list calls), the order of one
handle's calls across streams, and distinct handles used from concurrent
host threads.  Failures are forced from the host: a scan whose prefactor
Q0/(4 pi D) is so large that psi overflows to infinity (every kernel runs
normally; only the result is not finite)."""
import ctypes
import threading

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dd():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2507_00294_amd as dd

    dd.load_library()
    return dd


def _overflow_spec(wl):
    # kappa = D tau / p^2 = 1e11: the first pair term is ln(1 + 4 kappa / (2 sigma^2))
    # ~ 27, and Q0/(4 pi D) ~ 8e307, so psi at visit 1 exceeds the double range
    return wl.ScanSpec(6, 5, "raster", D_m2s=0.1, Q0_us=1e308)


def test_nonfinite_output_reported(dd):
    import torch

    from paper_2507_00294_amd import workloads as wl

    lib = dd.load_library()
    bad = dd.Scan(**_overflow_spec(wl).kwargs())
    good = dd.Scan(**wl.small_raster().kwargs())
    V = bad.num_visits
    # device outputs: the call succeeds, dd_scan_check names the first index
    for prec in ("fp64", "mixed"):
        out = bad.arrival(prec)
        assert bad.check() == 1
        o = out.cpu().numpy()
        assert o[0] == 0.0 and np.isinf(o[1])
        good.arrival(prec)
        assert good.check() == -1
    # host outputs: the call itself returns DD_EDEVICE
    host = (ctypes.c_double * V)()
    st = lib.dd_damage_at_probe_arrival(bad.handle, 0, ctypes.cast(host, ctypes.c_void_p), 0,
                                        None)
    assert st == dd.DD_EDEVICE and b"index 1" in lib.dd_last_error()
    st = lib.dd_damage_at_probe_arrival_range(bad.handle, 3, 6, 1,
                                              ctypes.cast(host, ctypes.c_void_p), 0, None)
    assert st == dd.DD_EDEVICE and b"index 0" in lib.dd_last_error()
    g = dd.Grid(0.0, 0.0, 1e-9, 1e-9, 6, 5)
    t = (ctypes.c_double * 2)(0.0, V * 1e-6)
    maps = (ctypes.c_double * (2 * 6 * 5))()  # two maps of the 6 x 5 grid
    st = lib.dd_damage_map(bad.handle, ctypes.byref(g), t, 2, 0, ctypes.cast(maps, ctypes.c_void_p),
                           0, None)
    assert st == dd.DD_EDEVICE and b"index 30" in lib.dd_last_error()  # map 0 is all zero
    st = lib.dd_damage_sweep(bad.handle, ctypes.byref(g), 0.0, V * 1e-6, 2, 0,
                             ctypes.cast(maps, ctypes.c_void_p), 0, None)
    assert st == dd.DD_EDEVICE and b"index 30" in lib.dd_last_error()
    # a later good call clears the report
    good_host = (ctypes.c_double * good.num_visits)()
    assert lib.dd_damage_at_probe_arrival(good.handle, 1, ctypes.cast(good_host, ctypes.c_void_p),
                                          0, None) == dd.DD_OK
    # batched: the host-output call names the scan; each scan's check its own index
    outs = [(ctypes.c_double * (s.num_visits + s.nx * s.ny))() for s in (good, bad)]
    hs = (ctypes.c_void_p * 2)(good.handle.value, bad.handle.value)
    os_ = (ctypes.c_void_p * 2)(*(ctypes.cast(o, ctypes.c_void_p).value for o in outs))
    st = lib.dd_batch_solve(hs, 2, 3, 1, os_, 0, None)
    assert st == dd.DD_EDEVICE and b"scan 1" in lib.dd_last_error()
    dev = dd.batch_solve([good, bad], dd.Q_FINAL_AT_PROBES, "fp64")
    assert good.check() == -1 and bad.check() == 0
    assert np.all(np.isfinite(dev[0].cpu().numpy()))
    torch.cuda.synchronize()


def test_nonfinite_visit_list_reported(dd):
    from paper_2507_00294_amd import workloads as wl

    vl = wl.visit_list("flyback", 5, 4, seed=3, D_m2s=0.1, Q0_us=1e308)
    ok = wl.visit_list("flyback", 5, 4, seed=3)
    bad = dd.Visits(vl.x_m, vl.y_m, vl.t0_s, vl.dwell_s, **vl.kwargs())
    good = dd.Visits(ok.x_m, ok.y_m, ok.t0_s, ok.dwell_s, **ok.kwargs())
    with pytest.raises(dd.DDError) as e:
        bad.arrival()
    assert e.value.status == dd.DD_EDEVICE and "list 0" in str(e.value)
    good.arrival()
    with pytest.raises(dd.DDError) as e:
        dd.visits_batch_arrival([good, bad], "mixed")
    assert "list 1" in str(e.value)


def test_one_handle_on_two_streams(dd):
    """Calls on one handle from two streams without host synchronization give
    the results of single-stream calls, bit for bit: each call waits for the
    handle's previous call when that ran on another stream."""
    import torch

    from paper_2507_00294_amd import workloads as wl

    spec = wl.large_random(96)
    scan = dd.Scan(**spec.kwargs())
    grid = (0.0, 0.0, 0.5e-9, 0.5e-9, 100, 90)
    times = [1000 * spec.tau_v, spec.n_visits * spec.tau_v]
    ref_a = scan.arrival("mixed").cpu()
    ref_r = scan.arrival_range(4000, 5000, "fp64").cpu()
    ref_m = scan.damage_map(*grid, times, "mixed").cpu()
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    n = 8
    oa = [torch.empty_like(ref_a, device="cuda") for _ in range(n)]
    orr = [torch.empty_like(ref_r, device="cuda") for _ in range(n)]
    om = [torch.empty_like(ref_m, device="cuda") for _ in range(n)]
    torch.cuda.synchronize()
    for k in range(n):
        s0, s1 = streams[k % 2], streams[(k + 1) % 2]
        scan.arrival("mixed", out=oa[k], stream=s0)
        scan.damage_map(*grid, times, "mixed", out=om[k], stream=s1)
        scan.arrival_range(4000, 5000, "fp64", out=orr[k], stream=s0)
    torch.cuda.synchronize()
    for k in range(n):
        assert torch.equal(oa[k].cpu(), ref_a), k
        assert torch.equal(om[k].cpu(), ref_m), k
        assert torch.equal(orr[k].cpu(), ref_r), k


def test_distinct_handles_in_threads(dd):
    """Two host threads, each creating, querying and destroying scans of its
    own on a stream of its own, get the results of serial calls."""
    import torch

    from paper_2507_00294_amd import workloads as wl

    specs = [wl.ScanSpec(40, 36, "random", seed=21, D_m2s=4e-13),
             wl.ScanSpec(33, 41, "interleaved", stride=3, D_m2s=2e-12)]
    grid = (0.0, 0.0, 1e-9, 1e-9, 40, 41)

    def run(spec):
        s = dd.Scan(**spec.kwargs())
        a = s.arrival("mixed").cpu()
        m = s.damage_map(*grid, [spec.n_visits * spec.tau_v], "fp64").cpu()
        b = dd.batch_solve([s], dd.Q_ARRIVAL, "mixed")[0].cpu()
        s.close()
        return a, m, b

    ref = [run(sp) for sp in specs]
    got = [[None] * 6 for _ in specs]
    errors = []

    def worker(i):
        try:
            torch.cuda.set_device(0)
            st = torch.cuda.Stream()
            with torch.cuda.stream(st):
                for rep in range(6):
                    got[i][rep] = run(specs[i])
                st.synchronize()
        except Exception as e:  # reported on the main thread
            errors.append(e)

    th = [threading.Thread(target=worker, args=(i,)) for i in range(len(specs))]
    for t in th:
        t.start()
    for t in th:
        t.join(timeout=120)
    assert not errors, errors
    for i in range(len(specs)):
        for rep in range(6):
            for x, y in zip(got[i][rep], ref[i]):
                assert torch.equal(x, y), (i, rep)
