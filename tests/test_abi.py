"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every symbol include/dd.h declares, validates its arguments, generates the
scan orders exactly as the oracle does, and fails loudly without a device."""
import ctypes
import os
import re
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def dd():
    import paper_2507_00294_amd as dd

    if not os.path.exists(dd.LIB_PATH):
        from paper_2507_00294_amd import build

        build.build()
    dd.load_library()
    return dd


def test_exports_every_header_symbol(dd):
    with open(os.path.join(ROOT, "include", "dd.h")) as f:
        header = f.read()
    declared = set(re.findall(r"\b(dd_[a-z_0-9]+)\s*\(", header))
    assert declared == set(dd.EXPORTS)
    lib = dd.load_library()
    for name in declared:
        assert hasattr(lib, name), name
    nm = subprocess.run(["nm", "-D", "--defined-only", dd.LIB_PATH], capture_output=True,
                        text=True, check=True).stdout
    for name in declared:
        assert re.search(rf"\bT {name}\b", nm), name


def test_visit_orders_match_oracle(dd, ora):
    cases = [
        ("raster", dict(nx=7, ny=5), dict(order=ora.RASTER)),
        ("interleaved", dict(nx=4, ny=4, stride=2), dict(order=ora.INTERLEAVED, stride=2)),
        ("interleaved", dict(nx=9, ny=7, stride=3), dict(order=ora.INTERLEAVED, stride=3)),
        ("random", dict(nx=33, ny=17, seed=3), dict(order=ora.RANDOM, seed=3)),
        ("random", dict(nx=512, ny=512, seed=3), dict(order=ora.RANDOM, seed=3)),
        ("random", dict(nx=5, ny=5, seed=2 ** 63 + 12345), dict(order=ora.RANDOM,
                                                               seed=2 ** 63 + 12345)),
        ("multiframe", dict(nx=6, ny=3, frames=4), dict(order=ora.MULTIFRAME, frames=4)),
    ]
    for order, kw, okw in cases:
        s = dd.Scan(kw["nx"], kw["ny"], order, **{k: v for k, v in kw.items()
                                                  if k not in ("nx", "ny")})
        o = ora.visits(okw.pop("order"), kw["nx"], kw["ny"], **okw)
        assert np.array_equal(s.visits(), o), (order, kw)
        assert s.num_visits == o.size


def _specs_match_oracle(dd, ora, specs, what):
    from gpu_util import oracle_visits

    for k, spec in enumerate(specs):
        s = dd.Scan(**spec.kwargs())
        o = oracle_visits(ora, spec)
        assert s.num_visits == o.size == spec.n_visits, (what, k)
        assert np.array_equal(s.visits(), o), (what, k, spec.order, spec.nx, spec.seed)


def test_visit_orders_of_every_workload_match_oracle(dd, ora):
    """Every scan the parity tests, the benchmark and the surrogate data use:
    the 32x32 raster and interleaved (stride 2) scans, the 512x512 random
    scan, all 256 scans of the batched configuration (seed 4) and the
    surrogate's training, test and validation sets (seeds 5, 6, 7)."""
    from paper_2507_00294_amd import workloads as wl

    _specs_match_oracle(dd, ora, wl.medium_scans(), "medium")
    _specs_match_oracle(dd, ora, [wl.small_raster(), wl.large_random()], "small/large")
    batch = wl.batch_scans()
    assert {s.order for s in batch} == {"raster", "interleaved", "random", "multiframe"}
    _specs_match_oracle(dd, ora, batch, "batched seed 4")
    for seed, n in ((5, 30000), (6, 2000), (7, 2000)):
        _specs_match_oracle(dd, ora, wl.surrogate_scans(n, seed), f"surrogate seed {seed}")


def test_largest_grid_side_accepted(dd):
    # 2048 probes per side is the largest grid (exact FP32 lattice distances)
    for nx, ny in ((2048, 1), (1, 2048), (2048, 2048)):
        assert dd.Scan(nx, ny).num_visits == nx * ny


def test_explicit_order_copied(dd):
    v = [3, 1, 1, 0, 2]
    s = dd.Scan(2, 2, "explicit", visits=v)
    assert s.visits().tolist() == v
    assert s.num_visits == 5


@pytest.mark.parametrize("kw", [
    dict(nx=0, ny=4), dict(nx=4, ny=-1), dict(nx=4, ny=4, pitch_m=0.0),
    dict(nx=4, ny=4, pitch_m=float("nan")), dict(nx=4, ny=4, dwell_s=-1e-6),
    dict(nx=4, ny=4, sigma_m=0.0), dict(nx=4, ny=4, D_m2s=0.0),
    dict(nx=4, ny=4, D_m2s=float("inf")), dict(nx=4, ny=4, Q0_us=-1.0),
    dict(nx=4, ny=4, order="interleaved", stride=0),
    dict(nx=4, ny=4, order="multiframe", frames=0),
    dict(nx=2, ny=2, order="explicit", visits=[0, 4]),
    dict(nx=2, ny=2, order="explicit", visits=[0, -1]),
    dict(nx=3000, ny=2), dict(nx=2049, ny=1), dict(nx=1, ny=2049),
])
def test_invalid_descriptions(dd, kw):
    nx, ny = kw.pop("nx"), kw.pop("ny")
    order = kw.pop("order", "raster")
    with pytest.raises(dd.DDError) as e:
        dd.Scan(nx, ny, order, **kw)
    assert e.value.status == dd.DD_EINVAL


def test_null_and_bad_arguments(dd):
    lib = dd.load_library()
    h = ctypes.c_void_p()
    assert lib.dd_scan_create(None, ctypes.byref(h)) == dd.DD_EINVAL
    assert lib.dd_scan_num_visits(None) == -1
    lib.dd_scan_destroy(None)  # NULL is allowed
    s = dd.Scan(2, 2)
    assert lib.dd_damage_at_probe_arrival(s.handle, 7, ctypes.c_void_p(16), 1, None) == dd.DD_EINVAL
    assert lib.dd_batch_solve(None, 0, 1, 0, None, 1, None) == dd.DD_EINVAL
    g = dd.Grid(0, 0, 1e-9, 1e-9, 0, 4)
    t = (ctypes.c_double * 1)(0.0)
    assert lib.dd_damage_map(s.handle, ctypes.byref(g), t, 1, 0, ctypes.c_void_p(16), 1,
                             None) == dd.DD_EINVAL
    g = dd.Grid(0, 0, 1e-9, 1e-9, 4, 4)
    t = (ctypes.c_double * 1)(-1.0)
    assert lib.dd_damage_map(s.handle, ctypes.byref(g), t, 1, 0, ctypes.c_void_p(16), 1,
                             None) == dd.DD_EINVAL
    assert lib.dd_pair_terms(-1.0, 0.5, 1, None, None, 0, None, None) == dd.DD_EINVAL
    assert b"kappa" in lib.dd_last_error()
    # the time sweep rejects bad times before touching a device
    o = ctypes.c_void_p(16)
    for t0, dt, n_t in ((-1.0, 1e-6, 4), (0.0, 0.0, 4), (0.0, -1e-6, 4), (0.0, 1e-6, 0),
                        (float("nan"), 1e-6, 4), (0.0, float("inf"), 4), (0.0, 1e308, 4)):
        assert lib.dd_damage_sweep(s.handle, ctypes.byref(g), t0, dt, n_t, 0, o, 1,
                                   None) == dd.DD_EINVAL, (t0, dt, n_t)
    # the streaming arrival query checks its visit range (V = 4 here)
    for j0, j1 in ((-1, 2), (3, 2), (0, 5)):
        assert lib.dd_damage_at_probe_arrival_range(s.handle, j0, j1, 1, o, 1,
                                                    None) == dd.DD_EINVAL, (j0, j1)
    assert lib.dd_damage_at_probe_arrival_range(s.handle, 2, 2, 1, None, 1, None) == dd.DD_OK
    bad = dd.Grid(0, 0, 1e-9, 1e-9, 4, 0)
    assert lib.dd_damage_sweep(s.handle, ctypes.byref(bad), 0.0, 1e-6, 4, 0, o, 1,
                               None) == dd.DD_EINVAL
    assert lib.dd_damage_sweep(s.handle, ctypes.byref(g), 0.0, 1e-6, 4, 9, o, 1,
                               None) == dd.DD_EINVAL


def test_queries_fail_loudly_without_device(dd):
    import torch

    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    lib = dd.load_library()
    s = dd.Scan(2, 2)
    out = (ctypes.c_double * 4)()
    st = lib.dd_damage_at_probe_arrival(s.handle, 0, ctypes.cast(out, ctypes.c_void_p), 0, None)
    assert st == dd.DD_EDEVICE
    assert lib.dd_last_error()
    g = dd.Grid(0, 0, 1e-9, 1e-9, 2, 2)
    st = lib.dd_damage_sweep(s.handle, ctypes.byref(g), 0.0, 1e-6, 1, 0,
                             ctypes.cast(out, ctypes.c_void_p), 0, None)
    assert st == dd.DD_EDEVICE


def test_out_of_memory_path():
    # a per-allocation limit makes scan creation of a large grid fail cleanly
    code = ("import paper_2507_00294_amd as dd\n"
            "try:\n    dd.Scan(1024, 1024)\nexcept dd.DDError as e:\n    print(e.status)\n")
    env = dict(os.environ, DD_ALLOC_LIMIT_BYTES="1000000", PYTHONPATH=ROOT)
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env,
                         cwd=ROOT, timeout=120)
    assert out.stdout.strip() == "-2", out.stderr


def test_tune_cache_load(dd, tmp_path):
    good = tmp_path / "tune.json"
    good.write_text('{\n  "arch": "gfx950",\n  "version": 1,\n'
                    '  "arrival_mixed": {"R": 4, "RN": 2, "K": 2048, "ms": 1.0},\n'
                    '  "arrival_fp64": {"R": 2, "RN": 2, "K": 1024, "ms": 1.0},\n'
                    '  "map_mixed": {"R": 2, "K": 4096, "ms": 1.0},\n'
                    '  "map_fp64": {"R": 1, "K": 4096, "ms": 1.0}\n}\n')
    dd.tune_load(str(good))
    bad = tmp_path / "bad.json"
    bad.write_text(good.read_text().replace('"R": 4', '"R": 3'))
    with pytest.raises(dd.DDError) as e:
        dd.tune_load(str(bad))
    assert e.value.status == dd.DD_EINVAL
    with pytest.raises(dd.DDError):
        dd.tune_load(str(tmp_path / "missing.json"))
    other = tmp_path / "other.json"
    other.write_text(good.read_text().replace("gfx950", "gfx942"))
    with pytest.raises(dd.DDError):
        dd.tune_load(str(other))
    dd.tune_load(str(good))  # leave the defaults in place


def test_visit_list_validation(dd):
    lib = dd.load_library()
    D = ctypes.c_double
    x = (D * 3)(0.0, 1e-9, 2e-9)
    t0 = (D * 3)(0.0, 1e-6, 2e-6)
    dw = (D * 3)(1e-6, 1e-6, 1e-6)
    bad_dw = (D * 3)(1e-6, 0.0, 1e-6)
    nan_t = (D * 3)(0.0, float("nan"), 2e-6)
    h = ctypes.c_void_p()
    vp = lambda a: ctypes.cast(a, ctypes.c_void_p)  # noqa: E731
    for args in [(0, x, x, t0, dw, 0.5e-9, 1e-13, 1.0),      # no visits
                 (3, x, x, t0, bad_dw, 0.5e-9, 1e-13, 1.0),  # dwell 0
                 (3, x, x, nan_t, dw, 0.5e-9, 1e-13, 1.0),   # start not finite
                 (3, x, x, t0, dw, 0.0, 1e-13, 1.0),         # sigma 0
                 (3, x, x, t0, dw, 0.5e-9, -1.0, 1.0),       # D < 0
                 (3, x, x, t0, dw, 0.5e-9, 1e-13, -1.0)]:    # Q0 < 0
        n, *arrs, sig, Dm, q = args
        assert lib.dd_visits_create(n, *map(vp, arrs), sig, Dm, q, ctypes.byref(h)) == dd.DD_EINVAL
        assert not h.value
    assert lib.dd_visits_create(3, vp(x), None, vp(t0), vp(dw), 0.5e-9, 1e-13, 1.0,
                                ctypes.byref(h)) == dd.DD_EINVAL
    v = dd.Visits([0.0, 1e-9, 2e-9], [0.0] * 3, [2e-6, 0.0, 1e-6], [1e-6] * 3)
    assert v.num_visits == 3
    assert lib.dd_visits_count(None) == -1
    out = (D * 3)()
    g = dd.Grid(0, 0, 1e-9, 1e-9, 2, 2)
    t = (D * 1)(1e-6)
    assert lib.dd_visits_arrival(None, 0, vp(out), 0, None) == dd.DD_EINVAL
    assert lib.dd_visits_arrival(v._h, 7, vp(out), 0, None) == dd.DD_EINVAL  # precision
    assert lib.dd_visits_map(v._h, ctypes.byref(g), t, 0, 0, vp(out), 0, None) == dd.DD_EINVAL
    assert lib.dd_visits_map(v._h, ctypes.byref(g), t, 1, 5, vp(out), 0, None) == dd.DD_EINVAL
    g_bad = dd.Grid(0, 0, 1e-9, 1e-9, 0, 2)
    assert lib.dd_visits_map(v._h, ctypes.byref(g_bad), t, 1, 0, vp(out), 0, None) == dd.DD_EINVAL
    t_bad = (D * 1)(float("inf"))
    assert lib.dd_visits_map(v._h, ctypes.byref(g), t_bad, 1, 0, vp(out), 0, None) == dd.DD_EINVAL
    lib.dd_visits_destroy(None)


def test_visit_list_fails_loudly_without_device(dd):
    import torch

    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    lib = dd.load_library()
    v = dd.Visits([0.0, 1e-9], [0.0, 0.0], [0.0, 1e-6], [1e-6, 1e-6])
    out = (ctypes.c_double * 2)()
    assert lib.dd_visits_arrival(v._h, 0, ctypes.cast(out, ctypes.c_void_p), 0,
                                 None) == dd.DD_EDEVICE
    assert lib.dd_last_error()


def test_visit_batch_validation(dd):
    lib = dd.load_library()
    v = dd.Visits([0.0, 1e-9], [0.0, 0.0], [0.0, 1e-6], [1e-6, 1e-6])
    out = (ctypes.c_double * 2)()
    hs = (ctypes.c_void_p * 1)(v._h.value)
    os_ = (ctypes.c_void_p * 1)(ctypes.cast(out, ctypes.c_void_p).value)
    assert lib.dd_visits_batch_arrival(None, 1, 0, os_, 0, None) == dd.DD_EINVAL
    assert lib.dd_visits_batch_arrival(hs, 0, 0, os_, 0, None) == dd.DD_EINVAL
    assert lib.dd_visits_batch_arrival(hs, 1, 9, os_, 0, None) == dd.DD_EINVAL
    nul = (ctypes.c_void_p * 1)(None)
    assert lib.dd_visits_batch_arrival(nul, 1, 0, os_, 0, None) == dd.DD_EINVAL
    assert lib.dd_visits_batch_arrival(hs, 1, 0, nul, 0, None) == dd.DD_EINVAL
    import torch

    if not torch.cuda.is_available():
        assert lib.dd_visits_batch_arrival(hs, 1, 0, os_, 0, None) == dd.DD_EDEVICE


def test_visit_batch_map_validation(dd):
    lib = dd.load_library()
    D, I32 = ctypes.c_double, ctypes.c_int32
    v = dd.Visits([0.0, 1e-9], [0.0, 0.0], [0.0, 1e-6], [1e-6, 1e-6])
    w = dd.Visits([0.0], [0.0], [0.0], [1e-6])
    out = (D * 8)()
    t = (D * 2)(1e-6, 2e-6)
    P = ctypes.POINTER(D)
    one = lambda *xs: (ctypes.c_void_p * len(xs))(*xs)  # noqa: E731
    grids = (dd.Grid * 2)(dd.Grid(0, 0, 1e-9, 1e-9, 2, 2), dd.Grid(0, 0, 1e-9, 1e-9, 2, 2))
    tp = (P * 2)(ctypes.cast(t, P), ctypes.cast(t, P))
    nt = (I32 * 2)(2, 2)
    o = ctypes.cast(out, ctypes.c_void_p).value
    ok = lambda hs, g=grids, n=nt: lib.dd_visits_batch_map(hs, 2, g, tp, n, 0, one(o, o), 0,  # noqa
                                                          None)
    assert ok(one(v._h.value, v._h.value)) == dd.DD_EINVAL  # the same list twice
    bad = (dd.Grid * 2)(dd.Grid(0, 0, 1e-9, 1e-9, 2, 2), dd.Grid(0, 0, 1e-9, 1e-9, 0, 2))
    assert ok(one(v._h.value, w._h.value), g=bad) == dd.DD_EINVAL
    assert ok(one(v._h.value, w._h.value), n=(I32 * 2)(2, 0)) == dd.DD_EINVAL
    assert lib.dd_visits_batch_map(None, 2, grids, tp, nt, 0, one(o, o), 0, None) == dd.DD_EINVAL
    assert lib.dd_visits_batch_map(one(v._h.value, w._h.value), 2, grids, tp, nt, 4, one(o, o), 0,
                                   None) == dd.DD_EINVAL


def test_handles_created_and_destroyed_in_threads(dd):
    """Distinct handles are independent: threads create, read and destroy
    scans and visit lists of their own concurrently (each handle keeps its
    plans and device state itself; no table is shared between handles)."""
    import threading

    errors = []

    def worker(seed):
        try:
            for k in range(40):
                s = dd.Scan(8 + k % 5, 7, "random", seed=seed + k)
                ids = s.visits()
                assert np.array_equal(np.sort(ids), np.arange(ids.size))
                if k % 3 == 0:
                    lib = dd.load_library()
                    bad = ctypes.c_int64(0)
                    assert lib.dd_scan_check(s.handle, ctypes.byref(bad)) == dd.DD_OK
                    assert bad.value == -1
                s.close()
                v = dd.Visits(np.arange(4.0) * 1e-9, np.zeros(4), np.arange(4.0) * 1e-6,
                              np.full(4, 1e-6))
                assert v.num_visits == 4
                v.close()
        except Exception as e:  # reported on the main thread
            errors.append(e)

    th = [threading.Thread(target=worker, args=(100 * i,)) for i in range(8)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    assert not errors, errors


def test_render_arguments_checked_before_device(dd):
    lib = dd.load_library()
    o = ctypes.c_void_p(16)
    ok = dd.RenderOpts(0.0, 0.0, 6.0, 1, 0)
    assert lib.dd_render_maps(o, 1, 4, 4, None, o, None) == dd.DD_EINVAL
    for n, w, h in ((-1, 4, 4), (1, 0, 4), (1, 4, 0)):
        assert lib.dd_render_maps(o, n, w, h, ctypes.byref(ok), o, None) == dd.DD_EINVAL
    assert lib.dd_render_maps(None, 1, 4, 4, ctypes.byref(ok), o, None) == dd.DD_EINVAL
    for bad in (dd.RenderOpts(0.0, 0.0, 0.0, 1, 0), dd.RenderOpts(0.0, 0.0, 301.0, 1, 0),
                dd.RenderOpts(0.0, 0.0, float("nan"), 1, 0), dd.RenderOpts(0.0, 1.0, 6.0, 1, 0),
                dd.RenderOpts(2.0, 1.0, 6.0, 0, 0), dd.RenderOpts(1.0, float("inf"), 6.0, 0, 0),
                dd.RenderOpts(0.0, 0.0, 6.0, 2, 0), dd.RenderOpts(0.0, 0.0, 6.0, 1, -1),
                dd.RenderOpts(0.0, 0.0, 6.0, 1, 257)):
        assert lib.dd_render_maps(o, 1, 4, 4, ctypes.byref(bad), o, None) == dd.DD_EINVAL


def test_save_png_roundtrip(dd, tmp_path):
    import struct
    import zlib

    rng = np.random.default_rng(3)
    img = rng.integers(0, 256, size=(7, 5, 3), dtype=np.uint8)
    path = str(tmp_path / "x.png")
    dd.save_png(path, img)
    data = open(path, "rb").read()
    assert data[:8] == b"\x89PNG\r\n\x1a\n"
    pos, chunks = 8, {}
    while pos < len(data):
        (n,) = struct.unpack(">I", data[pos:pos + 4])
        tag, body = data[pos + 4:pos + 8], data[pos + 8:pos + 8 + n]
        (crc,) = struct.unpack(">I", data[pos + 8 + n:pos + 12 + n])
        assert crc == zlib.crc32(tag + body) & 0xFFFFFFFF
        chunks[tag] = body
        pos += 12 + n
    w, h, depth, ctype = struct.unpack(">IIBB", chunks[b"IHDR"][:10])
    assert (w, h, depth, ctype) == (5, 7, 8, 2)
    raw = zlib.decompress(chunks[b"IDAT"])
    rows = [raw[y * (1 + 15):(y + 1) * (1 + 15)] for y in range(7)]
    assert all(r[0] == 0 for r in rows)
    back = np.frombuffer(b"".join(r[1:] for r in rows), dtype=np.uint8).reshape(7, 5, 3)
    assert np.array_equal(back, img)
