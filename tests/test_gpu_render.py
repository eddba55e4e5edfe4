"""Visualisation (dd_render_maps) against a numpy rendering of oracle values.

The rule (include/dd.h) turns a value into a colour by float decisions
(which bin of t, which level for iso-lines).  A pixel must equal the numpy
rendering exactly unless one of its decisions lies so close to a boundary
that the rounding of a logarithm or of the psi value itself (<= 1e-10
relative against the oracle) can move it: there both colours are right."""
import numpy as np
import pytest

from gpu_util import oracle_scan
from render_ref import render

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dd():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2507_00294_amd as dd

    dd.load_library()
    return dd


def _compare(got, ref, margin, slack):
    got = np.asarray(got)
    diff = np.any(got != ref, axis=-1)
    near = margin < slack
    bad = diff & ~near
    assert not bad.any(), f"{int(bad.sum())} pixels differ away from a boundary"
    return int(diff.sum()), int(near.sum())


@pytest.mark.parametrize("opts", [dict(), dict(levels=6), dict(decades=3.0, levels=3),
                                  dict(log_scale=False), dict(log_scale=False, levels=8)])
def test_render_oracle_maps(dd, ora, opts):
    """The small raster's maps (8x8 probes, 32x32 pixels, 16 times): the GPU
    renders the GPU's psi, numpy renders the oracle's."""
    import torch

    from paper_2507_00294_amd import workloads as wl

    spec = wl.small_raster()
    scan = dd.Scan(**spec.kwargs())
    m = wl.small_raster_maps(spec)
    times = m.times_s[::4]
    psi = scan.damage_map(m.x0_m, m.y0_m, m.dx_m, m.dy_m, m.w, m.h, times, "fp64")
    ref_psi = oracle_scan(ora, spec, scan).psi_map(m.x0_m, m.y0_m, m.dx_m, m.dy_m, m.w, m.h, times)
    got = dd.render_maps(psi, **opts).cpu().numpy()
    ref, margin = render(ref_psi, **opts)
    # psi agrees to 1e-10 relative: t moves by at most ~1e-10 / ln(10^6)
    ndiff, nnear = _compare(got, ref, margin, 1e-9)
    assert ndiff <= nnear
    assert got.shape == (len(times), 32, 32, 3)
    torch.cuda.synchronize()


def test_render_same_values_exact(dd):
    """Identical input values on both sides: equal except where a decision
    is within 1e-12 of a boundary (the last bit of a logarithm)."""
    import torch

    rng = np.random.default_rng(5)
    for (n, h, w) in ((3, 17, 29), (1, 1, 1), (2, 64, 63), (5, 7, 1)):
        v = 10.0 ** rng.uniform(-3, 9, size=(n, h, w))
        v[rng.random((n, h, w)) < 0.05] = 0.0
        for opts in (dict(), dict(levels=9), dict(lo=1e-2, hi=1e7), dict(lo=1e-2, hi=1e7, levels=4),
                     dict(log_scale=False, lo=-1e8, hi=2e8, levels=5), dict(decades=2.5)):
            got = dd.render_maps(torch.tensor(v, device="cuda"), **opts).cpu().numpy()
            ref, margin = render(v, **opts)
            _compare(got, ref, margin, 1e-12)


def test_render_block_per_map_equals_general_kernel(dd):
    """Maps of at most 16384 pixels, a multiple of 4 (any width, 1 and 2
    included), into an aligned image go
    to the one-block-per-map kernel; an output one byte off alignment takes
    the general kernel.  Both must give the same image bit for bit."""
    import torch

    rng = np.random.default_rng(11)
    for (n, h, w) in ((3, 128, 128), (8, 64, 64), (2, 60, 20), (5, 1, 4), (3, 8, 2), (2, 12, 1),
                      (4, 3, 12)):
        v = 10.0 ** rng.uniform(-4, 8, size=(n, h, w))
        v[rng.random((n, h, w)) < 0.03] = 0.0
        v[0, 0, :1] = np.nan
        v[-1] = -1.0  # a map with no positive value
        psi = torch.tensor(v, device="cuda")
        size = n * h * w * 3
        for opts in (dict(), dict(levels=7), dict(decades=2.0, levels=3), dict(lo=1e-2, hi=1e6),
                     dict(lo=1e-2, hi=1e6, levels=5), dict(log_scale=False, levels=4),
                     dict(log_scale=False, lo=-1e7, hi=5e7)):
            fast = dd.render_maps(psi, **opts)
            buf = torch.empty(size + 1, dtype=torch.uint8, device="cuda")
            slow = dd.render_maps(psi, out=buf[1:].view(n, h, w, 3), **opts)
            assert slow.data_ptr() % 4 == 1
            assert torch.equal(fast, slow), (n, h, w, opts)
            # psi 8 bytes off 16-byte alignment also takes the general kernel
            pbuf = torch.empty(psi.numel() + 1, dtype=torch.float64, device="cuda")
            psi8 = pbuf[1:].view(n, h, w)
            psi8.copy_(psi)
            assert psi8.data_ptr() % 16 == 8
            assert torch.equal(dd.render_maps(psi8, **opts), fast), (n, h, w, opts)


def test_render_special_values(dd):
    import torch

    v = np.array([[[0.0, -1.0, np.nan, np.inf, -np.inf, 1e-300, 5e-324, 1.0, 1e6, 1e300]]])
    for opts in (dict(), dict(lo=1e-3, hi=1e3), dict(log_scale=False), dict(levels=4)):
        got = dd.render_maps(torch.tensor(v, device="cuda"), **opts).cpu().numpy()
        ref, margin = render(v, **opts)
        _compare(got, ref, margin, 1e-12)
    # a map with no positive value is black under an automatic range
    z = torch.zeros((2, 3, 4), dtype=torch.float64, device="cuda")
    z[1] = -5.0
    assert int(dd.render_maps(z).sum()) == 0
    assert int(dd.render_maps(z, log_scale=False, levels=3).sum()) == 0


def test_render_sweep_frames(dd):
    """Frames of a time-sampled simulation: every frame rendered in one call
    equals the frame rendered alone, and the last frame's brightest pixel
    sits where its largest value is."""
    import torch

    from paper_2507_00294_amd import workloads as wl

    spec = wl.ScanSpec(16, 16, "raster", D_m2s=1e-12)
    scan = dd.Scan(**spec.kwargs())
    frames = scan.damage_sweep(0.0, 0.0, 0.5e-9, 0.5e-9, 31, 31, 0.0, 8 * spec.tau_v, 33, "mixed")
    rgb = dd.render_maps(frames, levels=6)
    for k in (0, 7, 32):
        one = dd.render_maps(frames[k].contiguous(), levels=6)
        assert torch.equal(one[0], rgb[k])
    last = frames[-1].cpu().numpy()
    img = dd.render_maps(frames[-1].contiguous()).cpu().numpy()[0]
    y, x = np.unravel_index(np.argmax(last), last.shape)
    assert tuple(img[y, x]) == (255, 255, 232)  # the top colour at the maximum
