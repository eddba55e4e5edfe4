"""Surrogate training resumed from a checkpoint continues bit for bit, and a
run whose loss turns non-finite rolls back to its last checkpoint.  The
failure is forced from the host (one parameter set to NaN between steps);
every kernel runs normally."""
import math

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


@pytest.fixture(scope="module")
def data(dd):
    from paper_2507_00294_amd import surrogate as sg
    from paper_2507_00294_amd import workloads as wl

    return sg.generate(wl.surrogate_scans(48, seed=31))


def _net(dd, data):
    from paper_2507_00294_amd import surrogate as sg

    net = dd.UNet(seed=2)
    sg.init_head(net, data[1], data[2])
    return net


KW = dict(batch=8, lr=1e-3, warmup=10, log_every=1000, checkpoint_every=20)


def test_resume_matches_uninterrupted_run(dd, data, tmp_path):
    from paper_2507_00294_amd import surrogate as sg

    x, own, t = data
    full = _net(dd, data)
    sg.train(full, x, own, t, 50, checkpoint=str(tmp_path / "a.npz"), **KW)
    part = _net(dd, data)
    ck = str(tmp_path / "b.npz")
    sg.train(part, x, own, t, 50, checkpoint=ck, stop_at=27, **KW)
    assert int(sg.read_checkpoint(ck)["step"]) == 27
    part.close()
    resumed = dd.UNet(seed=9)  # other initial weights: everything comes from the file
    sg.train(resumed, x, own, t, 50, checkpoint=ck, resume=True, **KW)
    assert np.array_equal(resumed.params(), full.params())
    ma, va, sa = full.adam_state()
    mb, vb, sb = resumed.adam_state()
    assert sa == sb == 50 and np.array_equal(ma, mb) and np.array_equal(va, vb)
    # a checkpoint of another run is refused
    with pytest.raises(ValueError):
        sg.train(resumed, x, own, t, 60, checkpoint=ck, resume=True, **KW)


def test_nonfinite_loss_rolls_back(dd, data, tmp_path):
    from paper_2507_00294_amd import surrogate as sg

    x, own, t = data
    net = _net(dd, data)
    hit = []

    def corrupt(step, n):
        if step == 33 and not hit:  # once: a weight of the first layer becomes NaN
            p = n.params()
            p[5] = np.nan
            n.set_params(p)
            hit.append(step)

    ck = str(tmp_path / "c.npz")
    hist = sg.train(net, x, own, t, 50, checkpoint=ck, callback=corrupt, **KW)
    c = sg.read_checkpoint(ck)
    assert hit == [33]
    assert int(c["rollbacks"]) == 1 and float(c["lr_scale"]) == 0.5 and int(c["step"]) == 50
    assert [k for k, v in hist if not math.isfinite(v)] == [39]  # the discarded step
    assert math.isfinite(hist[-1][1])
    assert np.all(np.isfinite(net.params()))
    # without a checkpoint there is nothing to roll back to
    net2 = _net(dd, data)
    hit.clear()
    with pytest.raises(FloatingPointError):
        sg.train(net2, x, own, t, 50, callback=corrupt, **dict(KW, log_every=1))
