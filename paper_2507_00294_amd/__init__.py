"""MI355X (gfx950) library for the cumulative damage-diffusion distribution of a
STEM scan -- thin Python binding over the C ABI of ``include/dd.h``.

Paper: "Fast Simulation of Damage Diffusion Distribution in Scanning
Transmission Electron Microscopy", Sec. II: psi(r, t) is the sum, over every
probe visit that started before t, of the closed-form single-visit field
(Eqs. 1-4); Eq. 6 is that sum.  All arithmetic runs in the HIP kernels of
``libdd.so``; this module only marshals arguments.  PyTorch supplies device
memory and the current HIP stream.  There is no CPU fallback: if ``libdd.so``
is missing or no gfx950 device is present, calls raise.
"""
from __future__ import annotations

import ctypes
import os
from typing import Iterable, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# DD_LIBRARY names another build of the library (the host-sanitizer run)
LIB_PATH = os.environ.get("DD_LIBRARY") or os.path.join(_HERE, "libdd.so")

DD_OK, DD_EINVAL, DD_ENOMEM, DD_EDEVICE, DD_EUNSUPPORTED = 0, -1, -2, -3, -4
ORDERS = {"raster": 0, "interleaved": 1, "random": 2, "multiframe": 3, "explicit": 4}
PRECISIONS = {"fp64": 0, "mixed": 1}
Q_ARRIVAL, Q_FINAL_AT_PROBES = 1, 2

# Every symbol the header declares (checked by the tests).
EXPORTS = (
    "dd_scan_create", "dd_scan_destroy", "dd_scan_num_visits", "dd_scan_visits",
    "dd_damage_map", "dd_damage_sweep", "dd_damage_at_probe_arrival",
    "dd_damage_at_probe_arrival_range", "dd_damage_at_probe_arrival_range_noalloc",
    "dd_batch_solve", "dd_scan_check",
    "dd_pair_terms",
    "dd_autotune", "dd_tune_load", "dd_profiling", "dd_profile_read", "dd_unet_create",
    "dd_unet_destroy", "dd_unet_num_params", "dd_unet_params", "dd_unet_grads", "dd_unet_forward",
    "dd_unet_backward", "dd_unet_loss", "dd_unet_adam", "dd_unet_adam_state",
    "dd_surrogate_batch",
    "dd_surrogate_inputs", "dd_surrogate_targets", "dd_unet_predict", "dd_visits_create",
    "dd_visits_destroy", "dd_visits_count", "dd_visits_arrival", "dd_visits_map",
    "dd_visits_batch_arrival", "dd_visits_batch_map", "dd_render_maps", "dd_last_error",
)


class DDError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"libdd status {status}: {msg}")
        self.status = status


class ScanDesc(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("order", ctypes.c_int32),
        ("stride", ctypes.c_int32), ("frames", ctypes.c_int32), ("reserved", ctypes.c_int32),
        ("seed", ctypes.c_uint64), ("visits", ctypes.POINTER(ctypes.c_int32)),
        ("n_visits", ctypes.c_int64), ("pitch_m", ctypes.c_double), ("dwell_s", ctypes.c_double),
        ("sigma_m", ctypes.c_double), ("D_m2s", ctypes.c_double), ("Q0_us", ctypes.c_double),
    ]


class KernelStats(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double), ("launches", ctypes.c_int64), ("pairs", ctypes.c_double),
                ("flops", ctypes.c_double)]


class RenderOpts(ctypes.Structure):
    _fields_ = [("lo", ctypes.c_double), ("hi", ctypes.c_double), ("decades", ctypes.c_double),
                ("log_scale", ctypes.c_int32), ("levels", ctypes.c_int32)]


class Grid(ctypes.Structure):
    _fields_ = [("x0_m", ctypes.c_double), ("y0_m", ctypes.c_double), ("dx_m", ctypes.c_double),
                ("dy_m", ctypes.c_double), ("w", ctypes.c_int32), ("h", ctypes.c_int32)]


_lib = None


def load_library():
    """Load libdd.so (built by ``__graft_entry__.build()``); raises if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    P = ctypes.POINTER
    lib.dd_scan_create.argtypes = [P(ScanDesc), P(vp)]
    lib.dd_scan_destroy.argtypes = [vp]
    lib.dd_scan_destroy.restype = None
    lib.dd_scan_num_visits.argtypes = [vp]
    lib.dd_scan_num_visits.restype = i64
    lib.dd_scan_visits.argtypes = [vp, P(i32)]
    lib.dd_damage_map.argtypes = [vp, P(Grid), P(dbl), i32, ctypes.c_int, vp, i32, vp]
    lib.dd_damage_sweep.argtypes = [vp, P(Grid), dbl, dbl, i32, ctypes.c_int, vp, i32, vp]
    lib.dd_damage_at_probe_arrival_range.argtypes = [vp, i64, i64, ctypes.c_int, vp, i32, vp]
    lib.dd_damage_at_probe_arrival_range_noalloc.argtypes = [vp, i64, i64, ctypes.c_int, vp, vp]
    lib.dd_damage_at_probe_arrival.argtypes = [vp, ctypes.c_int, vp, i32, vp]
    lib.dd_batch_solve.argtypes = [P(vp), i32, ctypes.c_uint32, ctypes.c_int, P(vp), i32, vp]
    lib.dd_scan_check.argtypes = [vp, P(i64)]
    lib.dd_pair_terms.argtypes = [dbl, dbl, i64, vp, vp, ctypes.c_int, vp, vp]
    lib.dd_autotune.argtypes = [ctypes.c_char_p]
    lib.dd_tune_load.argtypes = [ctypes.c_char_p]
    lib.dd_profiling.argtypes = [i32]
    lib.dd_profile_read.argtypes = [ctypes.c_char_p, P(KernelStats), i32]
    lib.dd_unet_create.argtypes = [ctypes.c_uint64, P(vp)]
    lib.dd_unet_destroy.argtypes = [vp]
    lib.dd_unet_destroy.restype = None
    lib.dd_unet_num_params.argtypes = [vp]
    lib.dd_unet_num_params.restype = i64
    lib.dd_unet_params.argtypes = [vp, vp, vp]
    lib.dd_unet_grads.argtypes = [vp, vp]
    lib.dd_unet_forward.argtypes = [vp, i32, vp, vp, i32, vp]
    lib.dd_unet_backward.argtypes = [vp, vp, vp, vp]
    lib.dd_unet_loss.argtypes = [vp, i32, vp, vp, vp, ctypes.c_float, vp, P(dbl), vp]
    f32 = ctypes.c_float
    lib.dd_unet_adam.argtypes = [vp, f32, f32, f32, f32, f32, P(f32), vp]
    lib.dd_unet_adam_state.argtypes = [vp, vp, vp, P(i64), vp, vp, P(i64)]
    lib.dd_surrogate_batch.argtypes = [vp, vp, vp, i64, vp, vp, i32, vp, vp, vp, vp]
    lib.dd_surrogate_inputs.argtypes = [P(vp), i32, vp, vp, vp]
    lib.dd_surrogate_targets.argtypes = [P(vp), i32, vp, vp, vp]
    lib.dd_unet_predict.argtypes = [vp, P(vp), i32, dbl, ctypes.c_int, vp, P(i32), vp]
    lib.dd_visits_create.argtypes = [i64, vp, vp, vp, vp, dbl, dbl, dbl, P(vp)]
    lib.dd_visits_destroy.argtypes = [vp]
    lib.dd_visits_destroy.restype = None
    lib.dd_visits_count.argtypes = [vp]
    lib.dd_visits_count.restype = i64
    lib.dd_visits_arrival.argtypes = [vp, ctypes.c_int, vp, i32, vp]
    lib.dd_visits_map.argtypes = [vp, P(Grid), P(dbl), i32, ctypes.c_int, vp, i32, vp]
    lib.dd_visits_batch_arrival.argtypes = [P(vp), i32, ctypes.c_int, P(vp), i32, vp]
    lib.dd_visits_batch_map.argtypes = [P(vp), i32, P(Grid), P(P(dbl)), P(i32), ctypes.c_int,
                                        P(vp), i32, vp]
    lib.dd_render_maps.argtypes = [vp, i64, i32, i32, P(RenderOpts), vp, vp]
    lib.dd_last_error.restype = ctypes.c_char_p
    for name in ("dd_scan_create", "dd_scan_visits", "dd_damage_map", "dd_damage_sweep",
                 "dd_damage_at_probe_arrival", "dd_damage_at_probe_arrival_range",
                 "dd_damage_at_probe_arrival_range_noalloc", "dd_batch_solve", "dd_scan_check", "dd_pair_terms", "dd_autotune",
                 "dd_tune_load", "dd_profiling", "dd_profile_read", "dd_unet_create",
                 "dd_unet_params", "dd_unet_grads", "dd_unet_forward", "dd_unet_backward",
                 "dd_unet_loss", "dd_unet_adam", "dd_unet_adam_state", "dd_surrogate_batch",
                 "dd_surrogate_inputs",
                 "dd_surrogate_targets", "dd_unet_predict", "dd_visits_create",
                 "dd_visits_arrival", "dd_visits_map", "dd_visits_batch_arrival",
                 "dd_visits_batch_map", "dd_render_maps"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(status: int):
    if status != DD_OK:
        raise DDError(status, load_library().dd_last_error().decode(errors="replace"))


def _torch():
    import torch

    if not torch.cuda.is_available():
        raise DDError(DD_EDEVICE, "no GPU visible to torch")
    return torch


def _stream(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _prec(p: str) -> int:
    try:
        return PRECISIONS[p]
    except KeyError:
        raise ValueError(f"precision must be one of {list(PRECISIONS)}") from None


class Scan:
    """A scan handle (``dd_scan``): probe grid, visit order and physics.

    Parameters follow ``dd_scan_desc``: SI units (m, s, m^2/s, u/s)."""

    def __init__(self, nx: int, ny: int, order: str = "raster", *, pitch_m: float = 1e-9,
                 dwell_s: float = 1e-6, sigma_m: float = 0.5e-9, D_m2s: float = 2.5e-13,
                 Q0_us: float = 1.0, stride: int = 2, frames: int = 1, seed: int = 0,
                 visits: Sequence[int] | None = None):
        lib = load_library()
        self._visits_keep = None
        d = ScanDesc()
        d.nx, d.ny, d.order = nx, ny, ORDERS[order]
        d.stride, d.frames, d.reserved, d.seed = stride, frames, 0, seed
        if visits is not None:
            arr = np.ascontiguousarray(visits, dtype=np.int32)
            self._visits_keep = arr
            d.visits = arr.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
            d.n_visits = arr.size
        d.pitch_m, d.dwell_s, d.sigma_m, d.D_m2s, d.Q0_us = pitch_m, dwell_s, sigma_m, D_m2s, Q0_us
        h = ctypes.c_void_p()
        _check(lib.dd_scan_create(ctypes.byref(d), ctypes.byref(h)))
        self._h = h
        self._hv = h.value  # plain int for the handle arrays of batched calls
        self.nx, self.ny, self.order = nx, ny, order
        self.pitch_m, self.dwell_s, self.sigma_m, self.D_m2s, self.Q0_us = (
            pitch_m, dwell_s, sigma_m, D_m2s, Q0_us)
        self.frames = frames if order == "multiframe" else 1
        self.tau_v = dwell_s / self.frames

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load_library().dd_scan_destroy(self._h)
            self._h = ctypes.c_void_p()
            self._hv = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    @property
    def num_visits(self) -> int:
        return int(load_library().dd_scan_num_visits(self._h))

    def visits(self) -> np.ndarray:
        out = np.empty(self.num_visits, dtype=np.int32)
        _check(load_library().dd_scan_visits(
            self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))
        return out

    def check(self) -> int:
        """Waits for the handle's last query (``dd_scan_check``) and returns the
        first index of its output that is not finite, or -1."""
        bad = ctypes.c_int64(-1)
        st = load_library().dd_scan_check(self._h, ctypes.byref(bad))
        if st == DD_EDEVICE and bad.value >= 0:
            return int(bad.value)
        _check(st)
        return -1

    def arrival(self, precision: str = "fp64", out=None, stream=None):
        """psi at each visit at its start (``dd_damage_at_probe_arrival``) as a
        float64 CUDA tensor [V], enqueued on the current stream."""
        torch = _torch()
        if out is None:
            out = torch.empty(self.num_visits, dtype=torch.float64, device="cuda")
        assert out.dtype == torch.float64 and out.is_cuda and out.is_contiguous()
        assert out.numel() == self.num_visits
        _check(load_library().dd_damage_at_probe_arrival(
            self._h, _prec(precision), ctypes.c_void_p(out.data_ptr()), 1, _stream(stream)))
        return out

    def arrival_range(self, j0: int, j1: int, precision: str = "fp64", out=None, stream=None):
        """psi at visits j0 <= j < j1 at their start
        (``dd_damage_at_probe_arrival_range``) as a float64 CUDA tensor [j1 - j0]."""
        torch = _torch()
        if out is None:
            out = torch.empty(max(j1 - j0, 0), dtype=torch.float64, device="cuda")
        assert out.dtype == torch.float64 and out.is_cuda and out.is_contiguous()
        assert out.numel() == max(j1 - j0, 0)
        _check(load_library().dd_damage_at_probe_arrival_range(
            self._h, j0, j1, _prec(precision), ctypes.c_void_p(out.data_ptr()), 1,
            _stream(stream)))
        return out

    def arrival_range_noalloc(self, j0: int, j1: int, out, precision: str = "fp64",
                              stream=None):
        """The same values as ``arrival_range`` into the caller's float64 CUDA
        tensor ``out`` [j1 - j0], with no allocation
        (``dd_damage_at_probe_arrival_range_noalloc``); the scan's tables
        must be resident (any earlier query of the scan builds them)."""
        torch = _torch()
        assert out.dtype == torch.float64 and out.is_cuda and out.is_contiguous()
        assert out.numel() == max(j1 - j0, 0)
        _check(load_library().dd_damage_at_probe_arrival_range_noalloc(
            self._h, j0, j1, _prec(precision), ctypes.c_void_p(out.data_ptr()),
            _stream(stream)))
        return out

    def damage_map(self, x0_m: float, y0_m: float, dx_m: float, dy_m: float, w: int, h: int,
                   times_s: Iterable[float], precision: str = "fp64", out=None, stream=None):
        """psi on a w-by-h pixel grid at each time (``dd_damage_map``) as a
        float64 CUDA tensor [n_t, h, w]."""
        torch = _torch()
        t = np.ascontiguousarray(np.atleast_1d(np.asarray(times_s, dtype=np.float64)))
        if out is None:
            out = torch.empty((t.size, h, w), dtype=torch.float64, device="cuda")
        assert out.dtype == torch.float64 and out.is_cuda and out.is_contiguous()
        assert out.numel() == t.size * w * h
        g = Grid(x0_m, y0_m, dx_m, dy_m, w, h)
        _check(load_library().dd_damage_map(
            self._h, ctypes.byref(g), t.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), t.size,
            _prec(precision), ctypes.c_void_p(out.data_ptr()), 1, _stream(stream)))
        return out

    def damage_sweep(self, x0_m: float, y0_m: float, dx_m: float, dy_m: float, w: int, h: int,
                     t0_s: float, dt_s: float, n_t: int, precision: str = "fp64", out=None,
                     stream=None):
        """Maps at t0 + k dt, k < n_t (``dd_damage_sweep``) as a float64 CUDA
        tensor [n_t, h, w]."""
        torch = _torch()
        if out is None:
            out = torch.empty((n_t, h, w), dtype=torch.float64, device="cuda")
        assert out.dtype == torch.float64 and out.is_cuda and out.is_contiguous()
        assert out.numel() == n_t * w * h
        g = Grid(x0_m, y0_m, dx_m, dy_m, w, h)
        _check(load_library().dd_damage_sweep(self._h, ctypes.byref(g), t0_s, dt_s, n_t,
                                              _prec(precision), ctypes.c_void_p(out.data_ptr()),
                                              1, _stream(stream)))
        return out

    def final_at_probes(self, precision: str = "fp64", stream=None):
        """psi at every probe position at the end of the scan, [ny, nx]."""
        t_end = self.num_visits * self.tau_v
        return self.damage_map(0.0, 0.0, self.pitch_m, self.pitch_m, self.nx, self.ny, [t_end],
                               precision, stream=stream)[0]


class Visits:
    """A general visit list (``dd_visits``): visit i at (x_m[i], y_m[i]) with
    the beam on from t0_s[i] for dwell_s[i] seconds (any order, overlaps
    allowed), evaluated in FP64 or "mixed" (the near-pair integral in FP32).
    SI units as in ``Scan``."""

    def __init__(self, x_m, y_m, t0_s, dwell_s, *, sigma_m: float = 0.5e-9,
                 D_m2s: float = 2.5e-13, Q0_us: float = 1.0):
        lib = load_library()
        cols = [np.ascontiguousarray(c, dtype=np.float64).ravel() for c in (x_m, y_m, t0_s, dwell_s)]
        n = cols[0].size
        if any(c.size != n for c in cols):
            raise ValueError("x_m, y_m, t0_s and dwell_s need one entry per visit")
        h = ctypes.c_void_p()
        _check(lib.dd_visits_create(n, *(ctypes.c_void_p(c.ctypes.data) for c in cols), sigma_m,
                                    D_m2s, Q0_us, ctypes.byref(h)))
        self._h = h
        self.sigma_m, self.D_m2s, self.Q0_us = sigma_m, D_m2s, Q0_us

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load_library().dd_visits_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def num_visits(self) -> int:
        return int(load_library().dd_visits_count(self._h))

    def arrival(self, precision: str = "fp64", out=None, stream=None):
        """psi at each visit's position when its beam turns on
        (``dd_visits_arrival``), float64 CUDA tensor [n] in visit order."""
        torch = _torch()
        if out is None:
            out = torch.empty(self.num_visits, dtype=torch.float64, device="cuda")
        assert out.dtype == torch.float64 and out.is_cuda and out.is_contiguous()
        assert out.numel() == self.num_visits
        _check(load_library().dd_visits_arrival(self._h, _prec(precision),
                                                ctypes.c_void_p(out.data_ptr()), 1,
                                                _stream(stream)))
        return out

    def damage_map(self, x0_m: float, y0_m: float, dx_m: float, dy_m: float, w: int, h: int,
                   times_s: Iterable[float], precision: str = "fp64", out=None, stream=None):
        """psi on a w-by-h pixel grid at each time (``dd_visits_map``),
        float64 CUDA tensor [n_t, h, w]."""
        torch = _torch()
        t = np.ascontiguousarray(np.atleast_1d(np.asarray(times_s, dtype=np.float64)))
        if out is None:
            out = torch.empty((t.size, h, w), dtype=torch.float64, device="cuda")
        assert out.dtype == torch.float64 and out.is_cuda and out.is_contiguous()
        assert out.numel() == t.size * w * h
        g = Grid(x0_m, y0_m, dx_m, dy_m, w, h)
        _check(load_library().dd_visits_map(
            self._h, ctypes.byref(g), t.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), t.size,
            _prec(precision), ctypes.c_void_p(out.data_ptr()), 1, _stream(stream)))
        return out


def visits_batch_arrival(lists: Sequence[Visits], precision: str = "fp64", out=None,
                         stream=None):
    """Arrival queries of many visit lists in one launch
    (``dd_visits_batch_arrival``): a list of float64 CUDA tensors, views of
    one flat buffer (``out``, if given, of sum(num_visits) elements)."""
    torch = _torch()
    counts = [v.num_visits for v in lists]
    if out is None:
        out = torch.empty(sum(counts), dtype=torch.float64, device="cuda")
    assert out.dtype == torch.float64 and out.is_cuda and out.is_contiguous()
    assert out.numel() == sum(counts)
    views = list(torch.split(out, counts))
    n = len(lists)
    hs = (ctypes.c_void_p * n)(*[v._h.value for v in lists])
    os_ = (ctypes.c_void_p * n)(*[t.data_ptr() for t in views])
    _check(load_library().dd_visits_batch_arrival(hs, n, _prec(precision), os_, 1,
                                                  _stream(stream)))
    return views


def visits_batch_map(lists: Sequence[Visits], grids, times, precision: str = "fp64",
                     stream=None):
    """Maps of many visit lists in one launch (``dd_visits_batch_map``):
    list k on grids[k] = (x0_m, y0_m, dx_m, dy_m, w, h) at times[k]; a list of
    float64 CUDA tensors [n_t, h, w]."""
    torch = _torch()
    n = len(lists)
    ts = [np.ascontiguousarray(np.atleast_1d(np.asarray(t, dtype=np.float64))) for t in times]
    gs = (Grid * n)(*[Grid(*g) for g in grids])
    outs = [torch.empty((t.size, g[5], g[4]), dtype=torch.float64, device="cuda")
            for t, g in zip(ts, grids)]
    D = ctypes.POINTER(ctypes.c_double)
    tp = (D * n)(*[t.ctypes.data_as(D) for t in ts])
    nt = (ctypes.c_int32 * n)(*[t.size for t in ts])
    hs = (ctypes.c_void_p * n)(*[v._h.value for v in lists])
    os_ = (ctypes.c_void_p * n)(*[o.data_ptr() for o in outs])
    _check(load_library().dd_visits_batch_map(hs, n, gs, tp, nt, _prec(precision), os_, 1,
                                              _stream(stream)))
    return outs


def batch_solve(scans: Sequence[Scan], queries: int = Q_ARRIVAL | Q_FINAL_AT_PROBES,
                precision: str = "mixed", outs=None, stream=None, out=None):
    """Many scans in one call (``dd_batch_solve``).  Per scan the result is
    [V] arrival (if requested) then [ny*nx] final map, float64 on the GPU.

    By default one buffer holds every scan's result back to back and the call
    returns one view of it per scan.  ``outs`` gives one tensor per scan
    instead; ``out`` gives the single buffer (contiguous float64 of the total
    size, any shape), and the call then returns ``out`` itself."""
    torch = _torch()
    n = len(scans)
    hs = _handles(scans)
    if outs is not None:
        ptrs = np.array([o.data_ptr() for o in outs], dtype=np.uint64)
    else:
        arr = (queries & Q_ARRIVAL) != 0
        fin = (queries & Q_FINAL_AT_PROBES) != 0
        sizes = np.array([(s.num_visits if arr else 0) + (s.nx * s.ny if fin else 0) for s in scans],
                         dtype=np.int64)
        total = int(sizes.sum())
        if out is None:
            flat = torch.empty(total, dtype=torch.float64, device="cuda")
        else:
            if out.dtype != torch.float64 or not out.is_cuda or not out.is_contiguous() or \
                    out.numel() != total:
                raise ValueError(f"out must be a contiguous float64 CUDA tensor of {total} elements")
            flat = out
        offs = np.zeros(n, dtype=np.int64)
        if n > 1:
            np.cumsum(sizes[:-1], out=offs[1:])
        ptrs = (np.uint64(flat.data_ptr()) + offs.astype(np.uint64) * np.uint64(8))
    os_ = (ctypes.c_void_p * n).from_buffer(np.ascontiguousarray(ptrs, dtype=np.uint64)) if n \
        else (ctypes.c_void_p * 0)()
    _check(load_library().dd_batch_solve(hs, n, queries, _prec(precision), os_, 1,
                                         _stream(stream)))
    if outs is not None:
        return outs
    if out is not None:
        return out
    return list(torch.split(flat.view(-1), sizes.tolist()))


def pair_terms(kappa: float, sigma_hat: float, a, lag, precision: str = "fp64", stream=None):
    """Dimensionless pair terms (``dd_pair_terms``) for CUDA float64 tensors a, lag."""
    torch = _torch()
    a = a.contiguous()
    lag = lag.contiguous()
    out = torch.empty_like(a)
    _check(load_library().dd_pair_terms(kappa, sigma_hat, a.numel(), ctypes.c_void_p(a.data_ptr()),
                                        ctypes.c_void_p(lag.data_ptr()), _prec(precision),
                                        ctypes.c_void_p(out.data_ptr()), _stream(stream)))
    return out


def autotune(cache_path: str | None = None):
    _check(load_library().dd_autotune(cache_path.encode() if cache_path else None))


def tune_load(cache_path: str):
    _check(load_library().dd_tune_load(cache_path.encode()))


def profiling(enable: bool = True):
    """Turn HIP-event timing of the main kernels on or off (``dd_profiling``)."""
    _check(load_library().dd_profiling(1 if enable else 0))


def profile_read(kernel: str, reset: bool = True) -> dict:
    """Totals for one kernel since the last reset (``dd_profile_read``)."""
    st = KernelStats()
    _check(load_library().dd_profile_read(kernel.encode(), ctypes.byref(st), 1 if reset else 0))
    return {"ms": st.ms, "launches": int(st.launches), "pairs": st.pairs, "flops": st.flops}


# ---------------------------------------------------------------------------
# Learned surrogate (dd_unet_*): U-Net on 64x64 scans, BF16 MFMA kernels.
SIDE = 64
CHANNELS = 5  # DD_SURROGATE_CHANNELS


def render_maps(psi, lo: float = 0.0, hi: float = 0.0, decades: float = 6.0,
                log_scale: bool = True, levels: int = 0, out=None, stream=None):
    """8-bit RGB images [n, h, w, 3] (uint8 CUDA tensor) of psi maps [n, h, w]
    or [h, w] (float64 CUDA tensor), rendered on the device
    (``dd_render_maps``): log or linear scale over [lo, hi] (lo = hi = 0:
    per map, its maximum and `decades` below), fixed colour map, optional
    iso-lines between `levels` steps."""
    torch = _torch()
    assert psi.dtype == torch.float64 and psi.is_cuda and psi.is_contiguous()
    shp = tuple(psi.shape)
    if len(shp) == 2:
        shp = (1,) + shp
    n, h, w = shp
    if out is None:
        out = torch.empty((n, h, w, 3), dtype=torch.uint8, device="cuda")
    assert out.dtype == torch.uint8 and out.is_cuda and out.is_contiguous()
    assert out.numel() == n * h * w * 3
    opt = RenderOpts(lo, hi, decades, 1 if log_scale else 0, levels)
    _check(load_library().dd_render_maps(ctypes.c_void_p(psi.data_ptr()), n, w, h,
                                         ctypes.byref(opt), ctypes.c_void_p(out.data_ptr()),
                                         _stream(stream)))
    return out


def save_png(path: str, rgb) -> None:
    """Writes one RGB image (uint8 array [h, w, 3], host or device) to `path` as
    a PNG file (8-bit truecolour, no interlace)."""
    import struct
    import zlib

    a = np.ascontiguousarray(rgb.cpu().numpy() if hasattr(rgb, "cpu") else rgb, dtype=np.uint8)
    if a.ndim != 3 or a.shape[2] != 3:
        raise ValueError("rgb must be [h, w, 3]")
    h, w = a.shape[:2]
    raw = b"".join(b"\x00" + a[y].tobytes() for y in range(h))  # filter 0 per row

    def chunk(tag, data):
        return (struct.pack(">I", len(data)) + tag + data +
                struct.pack(">I", zlib.crc32(tag + data) & 0xFFFFFFFF))

    with open(path, "wb") as f:
        f.write(b"\x89PNG\r\n\x1a\n")
        f.write(chunk(b"IHDR", struct.pack(">IIBBBBB", w, h, 8, 2, 0, 0, 0)))
        f.write(chunk(b"IDAT", zlib.compress(raw, 6)))
        f.write(chunk(b"IEND", b""))


def _handles(scans):
    """The scans' handles as a C array (void *[n]); the pointer keeps the array
    alive.  Built with numpy from plain ints: a ctypes array built element by
    element costs ~0.1 us per scan, which showed in calls over 2000 scans."""
    a = np.fromiter((s._hv for s in scans), dtype=np.uintp, count=len(scans))
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_void_p))


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def surrogate_inputs(scans, stream=None):
    """Network inputs x [n, 64, 64, CHANNELS] and own-visit terms [n, 64, 64]
    (float32 CUDA) of 64x64 scans."""
    torch = _torch()
    n = len(scans)
    x = torch.empty((n, SIDE, SIDE, CHANNELS), dtype=torch.float32, device="cuda")
    own = torch.empty((n, SIDE, SIDE), dtype=torch.float32, device="cuda")
    _check(load_library().dd_surrogate_inputs(_handles(scans), n, _ptr(x), _ptr(own),
                                              _stream(stream)))
    return x, own


def surrogate_targets(scans, psi, stream=None):
    """Training targets psi 4 pi D / Q0 [n, 64, 64] (float32) from exact final maps."""
    torch = _torch()
    psi = psi.contiguous()
    assert psi.dtype == torch.float64 and psi.numel() == len(scans) * SIDE * SIDE
    t = torch.empty((len(scans), SIDE, SIDE), dtype=torch.float32, device="cuda")
    _check(load_library().dd_surrogate_targets(_handles(scans), len(scans), _ptr(psi), _ptr(t),
                                               _stream(stream)))
    return t


def surrogate_batch(x_all, own_all, t_all, idx, transform, stream=None):
    """Mini-batch (x, own, t) of maps idx under the square's symmetries
    `transform` (int32 CUDA tensors, values 0..7)."""
    torch = _torch()
    nb = int(idx.numel())
    assert idx.dtype == torch.int32 and transform.dtype == torch.int32 and transform.numel() == nb
    xb = torch.empty((nb, SIDE, SIDE, CHANNELS), dtype=torch.float32, device="cuda")
    ob = torch.empty((nb, SIDE, SIDE), dtype=torch.float32, device="cuda")
    tb = torch.empty_like(ob)
    assert x_all.shape[0] == own_all.shape[0] == t_all.shape[0]
    _check(load_library().dd_surrogate_batch(_ptr(x_all), _ptr(own_all), _ptr(t_all),
                                             x_all.shape[0], _ptr(idx.contiguous()),
                                             _ptr(transform.contiguous()),
                                             nb, _ptr(xb), _ptr(ob), _ptr(tb), _stream(stream)))
    return xb, ob, tb


class UNet:
    """The surrogate network (``dd_unet``); see include/dd.h for the layout."""

    def __init__(self, seed: int = 0):
        h = ctypes.c_void_p()
        _check(load_library().dd_unet_create(seed, ctypes.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load_library().dd_unet_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def num_params(self) -> int:
        return int(load_library().dd_unet_num_params(self._h))

    def params(self) -> np.ndarray:
        out = np.empty(self.num_params, dtype=np.float32)
        _check(load_library().dd_unet_params(self._h, ctypes.c_void_p(out.ctypes.data), None))
        return out

    def set_params(self, p) -> None:
        p = np.ascontiguousarray(p, dtype=np.float32)
        assert p.size == self.num_params
        _check(load_library().dd_unet_params(self._h, None, ctypes.c_void_p(p.ctypes.data)))

    def grads(self) -> np.ndarray:
        out = np.empty(self.num_params, dtype=np.float32)
        _check(load_library().dd_unet_grads(self._h, ctypes.c_void_p(out.ctypes.data)))
        return out

    def forward(self, x, train: bool = False, stream=None):
        torch = _torch()
        x = x.contiguous()
        assert x.dtype == torch.float32 and x.shape[1:] == (SIDE, SIDE, CHANNELS)
        y = torch.empty((x.shape[0], SIDE, SIDE), dtype=torch.float32, device="cuda")
        _check(load_library().dd_unet_forward(self._h, x.shape[0], _ptr(x), _ptr(y),
                                              1 if train else 0, _stream(stream)))
        self._x = x  # the backward pass reads the input again
        return y

    def backward(self, dy, stream=None):
        dy = dy.contiguous()
        _check(load_library().dd_unet_backward(self._h, _ptr(self._x), _ptr(dy), _stream(stream)))

    def loss(self, y, own, t, anchor: float = 1.0, want_loss: bool = True, stream=None):
        """Mean squared relative L2 error of own + exp(y) against t per map
        and the gradient dy of that loss plus the anchor term (include/dd.h);
        returns (loss or None, dy)."""
        torch = _torch()
        y, own, t = y.contiguous(), own.contiguous(), t.contiguous()
        dy = torch.empty_like(y)
        loss = ctypes.c_double(0.0)
        _check(load_library().dd_unet_loss(self._h, y.shape[0], _ptr(y), _ptr(own), _ptr(t),
                                           anchor, _ptr(dy),
                                           ctypes.byref(loss) if want_loss else None,
                                           _stream(stream)))
        return (loss.value if want_loss else None), dy

    def adam(self, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8,
             clip: float = 0.0, want_norm: bool = False, stream=None):
        """One Adam step with global-norm clipping; returns the gradient norm
        when want_norm (synchronizes)."""
        norm = ctypes.c_float(0.0)
        _check(load_library().dd_unet_adam(self._h, lr, beta1, beta2, eps, clip,
                                           ctypes.byref(norm) if want_norm else None,
                                           _stream(stream)))
        return norm.value if want_norm else None

    def adam_state(self):
        """(m, v, step): Adam's moments (float32 [num_params]) and step count."""
        m = np.empty(self.num_params, dtype=np.float32)
        v = np.empty(self.num_params, dtype=np.float32)
        step = ctypes.c_int64(0)
        _check(load_library().dd_unet_adam_state(self._h, ctypes.c_void_p(m.ctypes.data),
                                                 ctypes.c_void_p(v.ctypes.data),
                                                 ctypes.byref(step), None, None, None))
        return m, v, int(step.value)

    def set_adam_state(self, m, v, step: int) -> None:
        m = np.ascontiguousarray(m, dtype=np.float32)
        v = np.ascontiguousarray(v, dtype=np.float32)
        assert m.size == v.size == self.num_params
        st = ctypes.c_int64(int(step))
        _check(load_library().dd_unet_adam_state(self._h, None, None, None,
                                                 ctypes.c_void_p(m.ctypes.data),
                                                 ctypes.c_void_p(v.ctypes.data), ctypes.byref(st)))

    def predict(self, scans, spot_tol: float = 0.02, precision: str = "mixed", stream=None):
        """Final maps [n, 64, 64] (float64 CUDA, u/m^2) and the fallback flags."""
        torch = _torch()
        n = len(scans)
        psi = torch.empty((n, SIDE, SIDE), dtype=torch.float64, device="cuda")
        fb = (ctypes.c_int32 * n)()
        _check(load_library().dd_unet_predict(self._h, _handles(scans), n, spot_tol,
                                              _prec(precision), ctypes.c_void_p(psi.data_ptr()),
                                              fb, _stream(stream)))
        return psi, np.frombuffer(fb, dtype=np.int32).copy()
