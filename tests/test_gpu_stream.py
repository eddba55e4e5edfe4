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
        ref = oracle_scan(ora, spec, scan).psi_arrival()
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


@pytest.mark.parametrize("R,RN", [(2, 4), (4, 4), (2, 2)])
def test_ranges_with_other_tile_shapes(dd, ora, wl, R, RN, tmp_path):
    # tuned tile shapes (R, RN in {2, 4}) where the near tile (64 RN
    # visits) is wider than or as wide as the far tile (64 R): the range's
    # partial columns start at the earlier of the two tile origins
    import json

    default = {"arch": "gfx950", "arrival_mixed": {"R": 4, "RN": 2, "K": 2048},
               "arrival_fp64": {"R": 2, "RN": 2, "K": 1024}, "map_mixed": {"R": 4, "K": 4096},
               "map_fp64": {"R": 1}}
    spec = wl.ScanSpec(23, 29, "random", 1e-9, 1e-6, 0.5e-9, 5e-13, 1.0, seed=13)
    scan = dd.Scan(**spec.kwargs())
    V = scan.num_visits
    ref = oracle_scan(ora, spec, scan).psi_arrival()
    try:
        for prec, key in (("fp64", "arrival_fp64"), ("mixed", "arrival_mixed")):
            cfg = json.loads(json.dumps(default))
            cfg[key]["R"], cfg[key]["RN"] = R, RN
            path = tmp_path / f"tune_{prec}.json"
            path.write_text(json.dumps(cfg))
            dd.tune_load(str(path))
            full = scan.arrival(prec).cpu().numpy()
            for j0, j1 in ((70, 200), (129, 130), (250, 520), (V - 300, V)):
                got = scan.arrival_range(j0, j1, prec).cpu().numpy()
                np.testing.assert_allclose(got, full[j0:j1],
                                           rtol=1e-13 if prec == "fp64" else 2e-7, atol=0)
                assert_close(got, ref[j0:j1], spec, prec, f"R={R} RN={RN} range {j0}:{j1}")
    finally:
        path = tmp_path / "tune_default.json"
        path.write_text(json.dumps(default))
        dd.tune_load(str(path))


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_bench_range_sampled_vs_oracle(dd, ora, wl, prec):
    # the benchmark's streaming call: the last 1024 visits of the 512x512
    # random scan, against the full arrival query and, at 24 sampled visits,
    # the oracle
    spec = wl.large_random()
    scan = dd.Scan(**spec.kwargs())
    V = scan.num_visits
    got = scan.arrival_range(V - 1024, V, prec).cpu().numpy()
    full = scan.arrival(prec).cpu().numpy()
    np.testing.assert_allclose(got, full[V - 1024:], rtol=1e-13 if prec == "fp64" else 2e-7,
                               atol=0)
    idx = np.sort(np.random.default_rng(42).choice(1024, 24, replace=False)) + (V - 1024)
    ref = oracle_scan(ora, spec, scan).psi_arrival(idx)
    assert_close(got[idx - (V - 1024)], ref, spec, prec, "bench range (sampled)")
