"""General visit lists (``dd_visits_*``): per-visit dwell, flyback and dead
time, sparse random subsets, revisits with unequal dwells and off-lattice
positions, against the oracle's general list element by element (the FP64
and the mixed bound); a uniform scan written as a list against the scan
kernels; input order, host output, several tiles, visit chunks and launch
groups with ragged tails, and the benchmark's list sampled at full size."""
import ctypes

import numpy as np
import pytest

from gpu_util import assert_close

pytestmark = pytest.mark.gpu
KINDS = ["flyback", "sparse", "frames", "drift"]
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


def both(dd, ora, vl):
    g = dd.Visits(vl.x_m, vl.y_m, vl.t0_s, vl.dwell_s, **vl.kwargs())
    o = ora.Visits(vl.x_m, vl.y_m, vl.t0_s, vl.dwell_s, vl.sigma_m, vl.D_m2s, vl.Q0_us)
    return g, o


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("D", [2.5e-13, 3e-11])
def test_arrival_vs_oracle(dd, ora, wl, kind, D, prec):
    # 9x7 lattice; D spans a diffusion length well below and well above the pitch
    vl = wl.visit_list(kind, 9, 7, seed=11, D_m2s=D)
    g, o = both(dd, ora, vl)
    got = g.arrival(prec).cpu().numpy()
    ref = o.psi_arrival()
    assert_close(got, ref, vl, prec, f"{kind} arrival")


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("kind", KINDS)
def test_maps_vs_oracle(dd, ora, wl, kind, prec):
    # off-lattice grid; times before the first start, mid-dwell, in a dead
    # time, at a dwell boundary and after the end
    vl = wl.visit_list(kind, 8, 6, seed=12, D_m2s=1e-12, sigma_m=0.4e-9)
    g, o = both(dd, ora, vl)
    i = vl.n_visits // 2
    times = [float(vl.t0_s[0]) * 0.5, float(vl.t0_s[1] + 0.3 * vl.dwell_s[1]),
             float(vl.t0_s[i]), float(vl.t0_s[i] + vl.dwell_s[i]), vl.t_end, 3 * vl.t_end]
    args = (-1.1e-9, -0.7e-9, 0.37e-9, 0.41e-9, 29, 21)
    got = g.damage_map(*args, times, prec).cpu().numpy()
    ref = o.psi_map(*args, times)
    assert_close(got, ref, vl, prec, f"{kind} maps")
    if vl.t0_s.min() > times[0]:
        assert np.all(got[0] == 0.0)


@pytest.mark.parametrize("prec", PRECS)
def test_many_tiles_and_chunks_vs_oracle(dd, ora, wl, prec):
    # 1480 visits: 6 tiles (the last ragged) against 3 visit chunks of 512
    # (the last ragged); maps of 3 x 2400 pixels (10 tiles per time)
    vl = wl.visit_list("flyback", 40, 37, seed=13, D_m2s=1e-12)
    g, o = both(dd, ora, vl)
    assert_close(g.arrival(prec).cpu().numpy(), o.psi_arrival(), vl, prec, "arrival")
    times = [0.37 * vl.t_end, 0.81 * vl.t_end, vl.t_end]
    args = (-2e-9, -1e-9, 0.9e-9, 0.8e-9, 60, 40)
    assert_close(g.damage_map(*args, times, prec).cpu().numpy(), o.psi_map(*args, times), vl,
                 prec, "maps")


def test_uniform_scan_as_list_matches_scan_kernels(dd, wl):
    # a random-order scan written as a general list: the same field as the
    # scan's own FP64 kernels (arrival and a final map)
    spec = wl.ScanSpec(24, 20, "random", 1e-9, 1e-6, 0.5e-9, 4e-13, 1.0, seed=5)
    scan = dd.Scan(**spec.kwargs())
    ids = scan.visits()
    k = np.arange(ids.size)
    g = dd.Visits((ids % spec.nx) * spec.pitch_m, (ids // spec.nx) * spec.pitch_m, k * spec.tau_v,
                  np.full(ids.size, spec.tau_v), sigma_m=spec.sigma_m, D_m2s=spec.D_m2s,
                  Q0_us=spec.Q0_us)
    a = scan.arrival("fp64").cpu().numpy()
    b = g.arrival().cpu().numpy()
    assert_close(b, a, spec, "fp64", "arrival")
    t = [ids.size * spec.tau_v]
    args = (0.0, 0.0, 0.5e-9, 0.5e-9, 48, 40)
    assert_close(g.damage_map(*args, t).cpu().numpy(), scan.damage_map(*args, t, "fp64").cpu().numpy(),
                 spec, "fp64", "map")


def test_input_order_and_host_output(dd, wl):
    vl = wl.visit_list("sparse", 30, 30, seed=14, D_m2s=2e-12)
    g = dd.Visits(vl.x_m, vl.y_m, vl.t0_s, vl.dwell_s, **vl.kwargs())
    a = g.arrival().cpu().numpy()
    p = np.random.default_rng(15).permutation(vl.n_visits)
    h = dd.Visits(vl.x_m[p], vl.y_m[p], vl.t0_s[p], vl.dwell_s[p], **vl.kwargs())
    b = h.arrival().cpu().numpy()
    assert np.array_equal(b, a[p])  # same start order inside, the same sums
    lib = dd.load_library()
    out = np.empty(vl.n_visits)
    assert lib.dd_visits_arrival(g._h, 0, ctypes.c_void_p(out.ctypes.data), 0, None) == 0
    assert np.array_equal(out, a)
    gr = dd.Grid(0.0, 0.0, 1e-9, 1e-9, 30, 30)
    t = np.array([0.5 * vl.t_end, vl.t_end])
    mo = np.empty((2, 30, 30))
    assert lib.dd_visits_map(g._h, ctypes.byref(gr), t.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                             2, 0, ctypes.c_void_p(mo.ctypes.data), 0, None) == 0
    assert np.array_equal(mo, g.damage_map(0.0, 0.0, 1e-9, 1e-9, 30, 30, t).cpu().numpy())


def test_single_visit_and_coincident_revisit(dd, ora):
    # one visit, then the same position visited again: the a = 0 (log) form
    g = dd.Visits([1e-9, 1e-9], [2e-9, 2e-9], [0.0, 3e-6], [1e-6, 2e-6], sigma_m=0.5e-9,
                  D_m2s=1e-12)
    o = ora.Visits([1e-9, 1e-9], [2e-9, 2e-9], [0.0, 3e-6], [1e-6, 2e-6], 0.5e-9, 1e-12)
    got = g.arrival().cpu().numpy()
    assert got[0] == 0.0
    ref = o.psi_arrival()
    assert abs(got[1] - ref[1]) <= 1e-10 * ref[1]
    one = dd.Visits([0.0], [0.0], [1e-6], [1e-6], sigma_m=0.5e-9, D_m2s=1e-12)
    assert one.arrival().cpu().numpy()[0] == 0.0


@pytest.mark.parametrize("prec", PRECS)
def test_bench_workload_sampled_vs_oracle(dd, ora, wl, prec):
    # the benchmark's list (256x256 raster, dwell jitter, flyback; 65536
    # visits) in the same calls the benchmark times: arrival at 48 sampled
    # visits and the final map at 48 sampled probes against the oracle
    vl = wl.visit_list("flyback", 256, 256, seed=21)
    g, o = both(dd, ora, vl)
    arr = g.arrival(prec).cpu().numpy()
    idx = wl.sampled_visits(vl.n_visits, 48, seed=22)
    ref = o.psi_points(vl.x_m[idx], vl.y_m[idx], vl.t0_s[idx])
    assert_close(arr[idx], ref, vl, prec, "arrival (sampled)")
    fin = g.damage_map(0.0, 0.0, 1e-9, 1e-9, 256, 256, [vl.t_end], prec).cpu().numpy()[0]
    pix = wl.sampled_visits(256 * 256, 48, seed=23)
    u, v = pix % 256, pix // 256
    ref = o.psi_points(u * 1e-9, v * 1e-9, np.full(pix.size, vl.t_end))
    assert_close(fin[v, u], ref, vl, prec, "final map (sampled)")


def test_map_launch_groups(dd, ora, wl):
    # 70 maps of 128x128 = 4480 point tiles: more than one launch group of
    # 4096 tiles; every map equals the same map asked for alone, bit for
    # bit, and sampled pixels match the oracle
    vl = wl.visit_list("drift", 20, 15, seed=24, D_m2s=5e-13)
    g, o = both(dd, ora, vl)
    times = np.linspace(0.02, 1.3, 70) * vl.t_end
    args = (-3e-9, -3e-9, 0.2e-9, 0.2e-9, 128, 128)
    many = g.damage_map(*args, times).cpu().numpy()
    for m in (0, 35, 63, 64, 69):
        one = g.damage_map(*args, [times[m]]).cpu().numpy()[0]
        assert np.array_equal(many[m], one), m
    rng = np.random.default_rng(25)
    m = rng.integers(0, 70, 64)
    u, v = rng.integers(0, 128, 64), rng.integers(0, 128, 64)
    ref = o.psi_points(-3e-9 + u * 0.2e-9, -3e-9 + v * 0.2e-9, times[m])
    assert_close(many[m, v, u], ref, vl, "fp64", "maps (sampled)")


@pytest.mark.parametrize("prec", PRECS)
def test_superposition_of_single_visits(dd, wl, prec):
    # the field of a list is the sum of the fields of its visits taken one
    # at a time: a check of the tiling, chunking and slot sums that does not
    # go through the oracle
    vl = wl.visit_list("sparse", 16, 16, seed=26, D_m2s=8e-13)
    args = (-1e-9, -1e-9, 0.6e-9, 0.6e-9, 31, 29)
    times = [0.5 * vl.t_end, vl.t_end]
    whole = dd.Visits(vl.x_m, vl.y_m, vl.t0_s, vl.dwell_s, **vl.kwargs()).damage_map(
        *args, times, prec).cpu().numpy()
    parts = np.zeros_like(whole)
    for i in range(vl.n_visits):
        one = dd.Visits(vl.x_m[i:i + 1], vl.y_m[i:i + 1], vl.t0_s[i:i + 1], vl.dwell_s[i:i + 1],
                        **vl.kwargs())
        parts += one.damage_map(*args, times, prec).cpu().numpy()
    np.testing.assert_allclose(whole, parts, rtol=1e-12 if prec == "fp64" else 1e-6,
                               atol=1e-250 * vl.Q0_us / (4 * np.pi * vl.D_m2s))


@pytest.mark.parametrize("prec", PRECS)
def test_batch_arrival_equals_single_lists(dd, wl, prec):
    # lists of every shape, size and physics in one launch: each list's
    # values equal its own call bit for bit (device and host outputs)
    vls = [wl.visit_list(kind, nx, ny, seed=30 + k, D_m2s=D)
           for k, (kind, nx, ny, D) in enumerate([
               ("flyback", 9, 7, 2.5e-13), ("sparse", 40, 30, 3e-11), ("frames", 12, 11, 1e-12),
               ("drift", 33, 17, 5e-13), ("flyback", 1, 1, 1e-12), ("sparse", 70, 70, 2e-13)])]
    lists = [dd.Visits(v.x_m, v.y_m, v.t0_s, v.dwell_s, **v.kwargs()) for v in vls]
    single = [g.arrival(prec).cpu().numpy() for g in lists]
    batch = [t.cpu().numpy() for t in dd.visits_batch_arrival(lists, prec)]
    for a, b in zip(single, batch):
        assert np.array_equal(a, b)
    lib = dd.load_library()
    outs = [np.empty(g.num_visits) for g in lists]
    hs = (ctypes.c_void_p * len(lists))(*[g._h.value for g in lists])
    os_ = (ctypes.c_void_p * len(lists))(*[o.ctypes.data for o in outs])
    assert lib.dd_visits_batch_arrival(hs, len(lists), dd.PRECISIONS[prec], os_, 0, None) == 0
    for a, o in zip(single, outs):
        assert np.array_equal(a, o)


@pytest.mark.parametrize("prec", PRECS)
def test_batch_map_equals_single_lists(dd, wl, prec):
    # maps of several lists on their own grids and times in one launch,
    # more than one launch group in all: each equals its own call bit for bit
    vls = [wl.visit_list(kind, nx, ny, seed=50 + k, D_m2s=D)
           for k, (kind, nx, ny, D) in enumerate([
               ("flyback", 9, 7, 2.5e-13), ("sparse", 30, 20, 3e-11), ("drift", 12, 11, 1e-12)])]
    lists = [dd.Visits(v.x_m, v.y_m, v.t0_s, v.dwell_s, **v.kwargs()) for v in vls]
    grids = [(-1e-9, -1e-9, 0.4e-9, 0.5e-9, 37, 23), (0.0, 0.0, 1e-9, 1e-9, 128, 128),
             (0.3e-9, -0.2e-9, 0.7e-9, 0.3e-9, 17, 45)]
    times = [np.linspace(0.1, 1.2, 5) * v.t_end for v in vls]
    times[1] = np.linspace(0.05, 1.0, 70) * vls[1].t_end  # 70 x 64 tiles
    batch = dd.visits_batch_map(lists, grids, times, prec)
    for g, gr, t, b in zip(lists, grids, times, batch):
        assert np.array_equal(g.damage_map(*gr, t, prec).cpu().numpy(), b.cpu().numpy())


@pytest.mark.parametrize("prec", PRECS)
def test_overlaps_equal_starts_negative_times(dd, ora, prec):
    # visits that overlap in time, share a start time, start before t = 0,
    # and a far-away visit: against the oracle; Q0 = 0 gives zeros
    rng = np.random.default_rng(60)
    n = 300
    x = rng.uniform(-5e-9, 5e-9, n)
    y = rng.uniform(-5e-9, 5e-9, n)
    t0 = np.sort(rng.uniform(-20e-6, 40e-6, n))
    t0[10:14] = t0[10]                     # four visits starting together
    dw = rng.uniform(0.2e-6, 8e-6, n)      # long dwells: neighbours overlap
    x[-1], y[-1] = 1e-6, -1e-6             # far from everything
    kw = dict(sigma_m=0.4e-9, D_m2s=6e-13)
    g = dd.Visits(x, y, t0, dw, **kw)
    o = ora.Visits(x, y, t0, dw, 0.4e-9, 6e-13, 1.0)
    spec = type("S", (), {"Q0_us": 1.0, "D_m2s": 6e-13})
    assert_close(g.arrival(prec).cpu().numpy(), o.psi_arrival(), spec, prec, "arrival")
    times = [-10e-6, 0.0, 13.3e-6, 45e-6, 200e-6]
    args = (-6e-9, -6e-9, 0.5e-9, 0.5e-9, 25, 25)
    assert_close(g.damage_map(*args, times, prec).cpu().numpy(), o.psi_map(*args, times), spec,
                 prec, "maps")
    z = dd.Visits(x, y, t0, dw, sigma_m=0.4e-9, D_m2s=6e-13, Q0_us=0.0)
    assert np.all(z.arrival(prec).cpu().numpy() == 0.0)


def _b_hat(t, t0, dwell, sigma, D):
    """b0, db, b1 of Eqs. 1-2 over sigma^2 for visits (t0, dwell) seen at time t."""
    th4 = 4.0 * D / sigma ** 2
    lag = t - t0
    on = np.minimum(lag, dwell)
    b0 = 2.0 + th4 * (lag - on)
    db = th4 * on
    return b0, db, b0 + db


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-13), ("mixed", 1e-6)])
def test_arrival_bulk_polynomial_vs_oracle(dd, ora, prec, tol):
    # a list whose every pair lies in the arrival's bulk domain (u = db/b1 <=
    # 2^-8 and v = x1 u <= 2^-5, the FP64 one; the mixed one is wider), so
    # every term takes the two-variable polynomial.  FP64 is held to that
    # form's own truncation and rounding level, where a wrong high-order
    # coefficient would show.
    rng = np.random.default_rng(41)
    n, sigma, D, tau = 48, 0.5e-9, 2.5e-13, 1e-6
    t0 = np.cumsum(tau * rng.uniform(500.0, 900.0, n))
    dwell = tau * rng.uniform(0.5, 1.5, n)
    x = rng.uniform(0.0, 190.0, n) * sigma
    y = rng.uniform(0.0, 190.0, n) * sigma
    for p in range(1, n):
        b0, db, b1 = _b_hat(t0[p], t0[:p], dwell[:p], sigma, D)
        a = ((x[p] - x[:p]) ** 2 + (y[p] - y[:p]) ** 2) / sigma ** 2
        u = db / b1
        assert np.all(u <= 2.0 ** -8) and np.all(a / b1 * u <= 2.0 ** -5)
    g = dd.Visits(x, y, t0, dwell, sigma_m=sigma, D_m2s=D)
    o = ora.Visits(x, y, t0, dwell, sigma, D)
    got = g.arrival(prec).cpu().numpy()
    ref = o.psi_arrival()
    assert got[0] == 0.0 and ref[0] == 0.0
    err = np.abs(got[1:] - ref[1:]) / ref[1:]
    assert err.max() <= tol, f"{prec}: max rel err {err.max():.3e} at {int(err.argmax()) + 1}"


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("mixed", 1e-6)])
def test_map_series_rows_vs_oracle(dd, ora, prec, tol):
    # a map whose rows are all lean (dx <= 1 at every pixel for every visit)
    # and reach the highest degrees (dx up to ~1): FP64 held to 1e-12, where
    # a wrong coefficient of the per-visit series would show; lags from 5 to
    # 60 dwells, so q = db/b0 runs from 0.02 to 0.22
    rng = np.random.default_rng(42)
    sigma, D, tau = 0.5e-9, 2.5e-13, 1e-6
    lags = np.array([5.0, 7.0, 9.0, 12.0, 17.0, 25.0, 40.0, 60.0]) * tau
    t = 100.0 * tau
    t0 = t - lags[::-1]
    dwell = np.full(t0.size, tau)
    x = rng.uniform(-2.0, 2.0, t0.size) * sigma
    y = rng.uniform(-2.0, 2.0, t0.size) * sigma
    w = h = 16
    x0, d = -5.0 * sigma, 10.0 * sigma / (w - 1)
    gx, gy = np.meshgrid(x0 + d * np.arange(w), x0 + d * np.arange(h))
    b0, db, b1 = _b_hat(t, t0, dwell, sigma, D)
    a = ((gx.ravel()[:, None] - x) ** 2 + (gy.ravel()[:, None] - y) ** 2) / sigma ** 2
    dx = a * db / (b0 * b1)
    assert dx.max() <= 1.0 and dx.max() > 0.5 and np.all(db / b0 <= 0.25)
    g = dd.Visits(x, y, t0, dwell, sigma_m=sigma, D_m2s=D)
    o = ora.Visits(x, y, t0, dwell, sigma, D)
    got = g.damage_map(x0, x0, d, d, w, h, [t], prec).cpu().numpy()[0]
    ref = o.psi_map(x0, x0, d, d, w, h, [t])[0]
    err = np.abs(got - ref) / ref
    assert err.max() <= tol, f"{prec}: max rel err {err.max():.3e}"
