"""Batched persistent solve: equal, bit for bit, to the per-scan calls, and
within tolerance of the oracle on sampled scans of the batched configuration
(256 scans of side 16..256, four orders, D, dwell and sigma sampled)."""
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
def test_batch_equals_per_scan(dd, wl, prec):
    specs = wl.batch_scans(12, seed=41, side_lo=9, side_hi=70)
    scans = [dd.Scan(**s.kwargs()) for s in specs]
    outs = dd.batch_solve(scans, dd.Q_ARRIVAL | dd.Q_FINAL_AT_PROBES, prec)
    for s, o in zip(scans, outs):
        o = o.cpu().numpy()
        arr = s.arrival(prec).cpu().numpy()
        fin = s.final_at_probes(prec).cpu().numpy().ravel()
        assert np.array_equal(o[:s.num_visits], arr)
        assert np.array_equal(o[s.num_visits:], fin)
    # single queries
    only = dd.batch_solve(scans[:3], dd.Q_FINAL_AT_PROBES, prec)
    for s, o in zip(scans[:3], only):
        assert np.array_equal(o.cpu().numpy(), s.final_at_probes(prec).cpu().numpy().ravel())


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_batch_small_vs_oracle(dd, ora, wl, prec):
    specs = wl.batch_scans(8, seed=43, side_lo=5, side_hi=24)
    scans = [dd.Scan(**s.kwargs()) for s in specs]
    outs = dd.batch_solve(scans, dd.Q_ARRIVAL | dd.Q_FINAL_AT_PROBES, prec)
    for spec, s, o in zip(specs, scans, outs):
        o = o.cpu().numpy()
        ora_s = oracle_scan(ora, spec, s)
        assert_close(o[:s.num_visits], ora_s.psi_arrival(), spec, prec, f"batch arrival {spec.order}")
        fin = ora_s.psi_map(0.0, 0.0, spec.pitch_m, spec.pitch_m, spec.nx, spec.ny,
                            [spec.n_visits * spec.tau_v])[0].ravel()
        assert_close(o[s.num_visits:], fin, spec, prec, f"batch final {spec.order}")


def test_batched_configuration_sampled(dd, ora, wl):
    """All 256 scans in one call (mixed), 16 of them checked on samples."""
    specs = wl.batch_scans()
    scans = [dd.Scan(**s.kwargs()) for s in specs]
    outs = dd.batch_solve(scans, dd.Q_ARRIVAL | dd.Q_FINAL_AT_PROBES, "mixed")
    rng = np.random.default_rng(17)
    for k in rng.choice(len(specs), size=16, replace=False):
        spec, s, o = specs[k], scans[k], outs[k].cpu().numpy()
        ora_s = oracle_scan(ora, spec, s)
        idx = wl.sampled_visits(spec.n_visits, 6, seed=int(k))
        assert_close(o[idx], ora_s.psi_arrival(idx), spec, "mixed", f"scan {k} arrival")
        pix = rng.choice(spec.nx * spec.ny, size=6, replace=False)
        x = (pix % spec.nx) * spec.pitch_m
        y = (pix // spec.nx) * spec.pitch_m
        t = np.full(pix.size, spec.n_visits * spec.tau_v)
        assert_close(o[spec.n_visits + pix], ora_s.psi_points(x, y, t), spec, "mixed",
                     f"scan {k} final")


DEFAULT_TUNE = {"arch": "gfx950", "arrival_mixed": {"R": 4, "RN": 2, "K": 2048},
                "arrival_fp64": {"R": 2, "RN": 2, "K": 1024}, "map_mixed": {"R": 4, "K": 4096},
                "map_fp64": {"R": 1}}


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_map_tile_width_leaves_results_unchanged(dd, wl, prec, tmp_path):
    """A pixel's sum is the same whatever the number of pixels per lane of
    the map tile (1, 2 or 4): maps of several sizes, by the per-scan call and
    by the batched call, are equal bit for bit across tile widths."""
    import json

    specs = wl.batch_scans(5, seed=45, side_lo=30, side_hi=90)
    scans = [dd.Scan(**s.kwargs()) for s in specs]
    key = "map_mixed" if prec == "mixed" else "map_fp64"
    ref = None
    try:
        for R in (4, 2, 1):
            cfg = json.loads(json.dumps(DEFAULT_TUNE))
            cfg[key]["R"] = R
            path = tmp_path / f"tune_{R}.json"
            path.write_text(json.dumps(cfg))
            dd.tune_load(str(path))
            single = [s.final_at_probes(prec).cpu().numpy().ravel() for s in scans]
            batch = [o.cpu().numpy() for o in dd.batch_solve(scans, dd.Q_FINAL_AT_PROBES, prec)]
            if ref is None:
                ref = single
            for a, b, c in zip(ref, single, batch):
                assert np.array_equal(a, b), R
                assert np.array_equal(a, c), R
    finally:
        path = tmp_path / "tune_default.json"
        path.write_text(json.dumps(DEFAULT_TUNE))
        dd.tune_load(str(path))


def test_batch_output_buffers(dd, wl):
    """The three ways of handing over outputs give the same values: one view
    per scan of a call-allocated buffer, one tensor per scan, and a single
    caller buffer holding every scan's result back to back."""
    import torch

    specs = wl.batch_scans(5, seed=47, side_lo=8, side_hi=30)
    scans = [dd.Scan(**s.kwargs()) for s in specs]
    q = dd.Q_ARRIVAL | dd.Q_FINAL_AT_PROBES
    views = dd.batch_solve(scans, q, "mixed")
    sizes = [s.num_visits + s.nx * s.ny for s in scans]
    assert [v.numel() for v in views] == sizes
    own = [torch.empty(n, dtype=torch.float64, device="cuda") for n in sizes]
    assert dd.batch_solve(scans, q, "mixed", outs=own) is own
    flat = torch.empty(sum(sizes), dtype=torch.float64, device="cuda")
    assert dd.batch_solve(scans, q, "mixed", out=flat) is flat
    off = 0
    for v, o, n in zip(views, own, sizes):
        assert torch.equal(v, o)
        assert torch.equal(v, flat[off:off + n])
        off += n
    with pytest.raises(ValueError):
        dd.batch_solve(scans, q, "mixed", out=flat[:-1])
