"""Streaming form of the arrival query (``dd_damage_at_probe_arrival_range``):
psi at a range of visits equals the full arrival query on those visits (to
the rounding of a different summation order) and the oracle, for ranges at
the start, in the middle, across tile boundaries and at the end of scans,
single visits included; an empty range does nothing."""
import numpy as np
import pytest

from gpu_util import assert_close, oracle_scan

pytestmark = pytest.mark.gpu


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


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_ranges_equal_full_arrival_and_oracle(dd, ora, wl, prec):
    specs = [wl.ScanSpec(33, 31, "random", 1e-9, 1e-6, 0.5e-9, 3e-13, 1.0, seed=9),
             wl.ScanSpec(24, 20, "multiframe", 1e-9, 4e-6, 0.3e-9, 2e-12, 1.0, frames=4)]
    for spec in specs:
        scan = dd.Scan(**spec.kwargs())
        V = scan.num_visits
        full = scan.arrival(prec).cpu().numpy()
        ref = oracle_scan(ora, spec, scan.visits()).psi_arrival()
        for j0, j1 in ((0, 1), (0, 300), (5, 6), (255, 257), (300, V - 100), (V - 256, V),
                       (V - 1, V), (0, V)):
            got = scan.arrival_range(j0, j1, prec).cpu().numpy()
            assert got.shape == (j1 - j0,)
            # FP64: the same terms summed in another order.  Mixed: the lag
            # chunks differ, and the items on a tile's causal edge sum their
            # FP32 terms with one more rounding (a masked product is not
            # fused into the running sum), ~1e-8 of a term.
            np.testing.assert_allclose(got, full[j0:j1], rtol=1e-13 if prec == "fp64" else 2e-7,
                                       atol=0)
            assert_close(got, ref[j0:j1], spec, prec, f"range {j0}:{j1}")
        empty = scan.arrival_range(7, 7, prec)
        assert empty.numel() == 0
