"""The no-allocation streaming query (dd_damage_at_probe_arrival_range_noalloc)
through the C ABI against the allocating one (dd_damage_at_probe_arrival_range)
on the same scan: equal bit for bit, on two calls in a row, the second over a
smaller range, in both precisions.  The scratch array is shared by every call
on the GPU and keeps the previous call's contents, so the second call checks
that nothing stale is read."""
import ctypes

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


def _noalloc(dd, scan, j0, j1, prec, out, stream=None):
    lib = dd.load_library()
    st = dd._stream(stream)
    return lib.dd_damage_at_probe_arrival_range_noalloc(scan.handle, j0, j1, dd.PRECISIONS[prec],
                                                        ctypes.c_void_p(out.data_ptr()), st)


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_noalloc_equals_allocating_query(dd, prec):
    import torch

    from paper_2507_00294_amd import workloads as wl

    spec = wl.large_random()
    scan = dd.Scan(**spec.kwargs())
    V = scan.num_visits
    # not resident yet: rejected before any work
    out = torch.empty(1024, dtype=torch.float64, device="cuda")
    assert _noalloc(dd, scan, V - 1024, V, prec, out) == dd.DD_EINVAL
    scan.arrival_range(0, 1, prec)  # builds the scan's tables
    for (j0, j1) in ((V - 1024, V), (V - 300, V - 44)):  # the second range is smaller
        ref = scan.arrival_range(j0, j1, prec)
        got = torch.full((j1 - j0,), float("nan"), dtype=torch.float64, device="cuda")
        assert _noalloc(dd, scan, j0, j1, prec, got) == dd.DD_OK, dd.load_library().dd_last_error()
        torch.cuda.synchronize()
        assert torch.equal(got, ref), (j0, j1, float((got - ref).abs().max()))
        assert scan.check() == -1
    # a range whose scratch exceeds the static array is rejected, nothing runs
    big = torch.empty(V, dtype=torch.float64, device="cuda")
    assert _noalloc(dd, scan, 0, V, prec, big) == dd.DD_EINVAL
    assert b"scratch" in dd.load_library().dd_last_error()


def test_noalloc_small_scan_and_edges(dd):
    """A small scan (ranges at the start, across tile edges and at the end),
    alternating with a second scan so that each call finds the other's
    contents in the scratch."""
    import torch

    from paper_2507_00294_amd import workloads as wl

    a = dd.Scan(**wl.ScanSpec(23, 29, "random", seed=7, D_m2s=1e-12).kwargs())
    b = dd.Scan(**wl.ScanSpec(40, 40, "interleaved", stride=3).kwargs())
    for s in (a, b):
        s.arrival("mixed")
    ranges = [(0, 1), (0, 300), (250, 270), (255, 513), (600, 667)]
    for (j0, j1) in ranges:
        for s in (a, b):
            for prec in ("mixed", "fp64"):
                ref = s.arrival_range(j0, j1, prec)
                got = torch.empty(j1 - j0, dtype=torch.float64, device="cuda")
                assert _noalloc(dd, s, j0, j1, prec, got) == dd.DD_OK
                torch.cuda.synchronize()
                assert torch.equal(got, ref), (j0, j1, prec)
    lib = dd.load_library()
    assert _noalloc(dd, a, 5, 4, "mixed", torch.empty(1, device="cuda",
                                                      dtype=torch.float64)) == dd.DD_EINVAL
    assert lib.dd_damage_at_probe_arrival_range_noalloc(a.handle, 3, 3, 1, None,
                                                        None) == dd.DD_OK
