"""Checkpoint format of surrogate training (host only): the arrays written
come back unchanged, the write replaces the file atomically, and a
checkpoint refuses to resume a run with other settings."""
import json
import os

import numpy as np
import pytest


def test_checkpoint_roundtrip(tmp_path):
    from paper_2507_00294_amd import surrogate as sg

    rng = np.random.default_rng(4)
    arrays = dict(params=rng.normal(size=1000).astype(np.float32),
                  adam_m=rng.normal(size=1000).astype(np.float32),
                  adam_v=rng.random(1000).astype(np.float32),
                  adam_step=np.array(1234, np.int64),
                  rng=rng.integers(0, 256, 16, dtype=np.uint8),
                  perm=rng.permutation(64).astype(np.int32), pos=np.array(40, np.int64),
                  step=np.array(1234, np.int64), lr_scale=np.array(0.25),
                  rollbacks=np.array(2, np.int64),
                  settings=np.array(json.dumps(dict(steps=5000, lr=1e-3))))
    path = str(tmp_path / "ckpt.npz")
    sg.write_checkpoint(path, arrays)
    assert not os.path.exists(path + ".tmp")
    back = sg.read_checkpoint(path)
    for k, v in arrays.items():
        assert back[k].dtype == v.dtype and np.array_equal(back[k], v), k
    assert json.loads(str(back["settings"])) == dict(steps=5000, lr=1e-3)
    # a second write replaces the first whole
    arrays["step"] = np.array(2000, np.int64)
    sg.write_checkpoint(path, arrays)
    assert int(sg.read_checkpoint(path)["step"]) == 2000


def test_checkpoint_checks(tmp_path):
    from paper_2507_00294_amd import surrogate as sg

    sg.check_settings(dict(steps=10, lr=1e-3), dict(steps=10, lr=1e-3))
    with pytest.raises(ValueError):
        sg.check_settings(dict(steps=10, lr=1e-3), dict(steps=10, lr=2e-3))
    path = str(tmp_path / "other.npz")
    np.savez(path, params=np.zeros(3))
    with pytest.raises(ValueError):
        sg.read_checkpoint(path)
