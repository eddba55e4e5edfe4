"""Autotuner: runs on the GPU, writes a cache that loads back, and the tuned
shapes still meet the parity bar and keep the batched path equal to the
per-scan path.  Named to run after the other GPU tests (it changes the
process-wide tile shapes)."""
import json

import numpy as np
import pytest

from gpu_util import assert_close, oracle_scan

pytestmark = pytest.mark.gpu


def test_autotune_roundtrip(ora, tmp_path):
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2507_00294_amd as dd
    from paper_2507_00294_amd import workloads as wl

    path = tmp_path / "tune.json"
    dd.autotune(str(path))
    cache = json.loads(path.read_text())
    assert cache["arch"] == "gfx950"
    for key in ("arrival_mixed", "arrival_fp64", "map_mixed", "map_fp64"):
        assert cache[key]["ms"] > 0
    dd.tune_load(str(path))
    spec = wl.medium_scans(1)[0]
    scan = dd.Scan(**spec.kwargs())
    ref = oracle_scan(ora, spec, scan).psi_arrival()
    for prec in ("fp64", "mixed"):
        assert_close(scan.arrival(prec).cpu().numpy(), ref, spec, prec, "tuned arrival")
    specs = wl.batch_scans(6, seed=77, side_lo=8, side_hi=40)
    scans = [dd.Scan(**s.kwargs()) for s in specs]
    outs = dd.batch_solve(scans, dd.Q_ARRIVAL | dd.Q_FINAL_AT_PROBES, "mixed")
    for s, o in zip(scans, outs):
        o = o.cpu().numpy()
        assert np.array_equal(o[:s.num_visits], s.arrival("mixed").cpu().numpy())
        assert np.array_equal(o[s.num_visits:], s.final_at_probes("mixed").cpu().numpy().ravel())
