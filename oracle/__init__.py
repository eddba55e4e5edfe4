"""CPU oracle for the cumulative damage-diffusion distribution (ctypes wrapper).

TEST INFRASTRUCTURE ONLY.  This package is the slow, plain reference that the
GPU library is checked against; only the tests, the smoke check and the CPU
baseline leg of the benchmark import it.  It shares no code with the GPU
library (``paper_2507_00294_amd``) and never imports it.

The arithmetic lives in ``ddo.c`` (long double, plain loops); this module only
marshals numpy arrays.  Paper: Sec. II, Eqs. 1-4 (single probe) and Eq. 6
(cumulative sum over visited probes).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ddo.c")
# DDO_LIBRARY names another build of ddo.c (the sanitizer run); it is used as is
_LIB_PATH = os.environ.get("DDO_LIBRARY") or os.path.join(_HERE, "libddo.so")
_lock = threading.Lock()
_lib = None

RASTER, INTERLEAVED, RANDOM, MULTIFRAME = 0, 1, 2, 3


def build(force: bool = False) -> str:
    """Compile ddo.c with gcc into oracle/libddo.so (plain -O2, no fast-math)."""
    if os.environ.get("DDO_LIBRARY"):
        return _LIB_PATH
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < max(
        os.path.getmtime(_SRC), os.path.getmtime(os.path.join(_HERE, "ddo.h"))
    ):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-std=c99", "-D_POSIX_C_SOURCE=200809L", "-fPIC", "-shared",
             "-Wall", "-o", tmp, _SRC, "-lquadmath", "-lm", "-lpthread"]
        )
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Scan(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("ids", ctypes.POINTER(ctypes.c_int32)), ("n_visits", ctypes.c_int64),
        ("pitch", ctypes.c_double), ("tau_v", ctypes.c_double), ("sigma", ctypes.c_double),
        ("D", ctypes.c_double), ("Q0", ctypes.c_double),
    ]


class _Visits(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64),
        ("x", ctypes.POINTER(ctypes.c_double)), ("y", ctypes.POINTER(ctypes.c_double)),
        ("t0", ctypes.POINTER(ctypes.c_double)), ("dwell", ctypes.POINTER(ctypes.c_double)),
        ("sigma", ctypes.c_double), ("D", ctypes.c_double), ("Q0", ctypes.c_double),
    ]


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build()
            lib = ctypes.CDLL(_LIB_PATH)
            LD, D, I32, I64, U64 = (ctypes.c_longdouble, ctypes.c_double, ctypes.c_int32,
                                    ctypes.c_int64, ctypes.c_uint64)
            P = ctypes.POINTER
            for name in ("ddo_e1_series", "ddo_e1_cf", "ddo_e1_quad"):
                getattr(lib, name).restype = LD
                getattr(lib, name).argtypes = [LD]
            lib.ddo_e1.restype = D
            lib.ddo_e1.argtypes = [D]
            lib.ddo_phi.restype = D
            lib.ddo_phi.argtypes = [D] * 6
            lib.ddo_phi_bracket_q.restype = D
            lib.ddo_phi_bracket_q.argtypes = [D] * 5
            lib.ddo_e1_q.restype = D
            lib.ddo_e1_q.argtypes = [D]
            lib.ddo_splitmix64.restype = U64
            lib.ddo_splitmix64.argtypes = [P(U64)]
            lib.ddo_visits.restype = I64
            lib.ddo_visits.argtypes = [ctypes.c_int, I32, I32, I32, I32, U64, P(I32), I64]
            lib.ddo_psi_points.restype = ctypes.c_int
            lib.ddo_psi_points.argtypes = [P(_Scan), I64, P(D), P(D), P(D), P(D), ctypes.c_int]
            lib.ddo_psi_arrival.restype = ctypes.c_int
            lib.ddo_psi_arrival.argtypes = [P(_Scan), I64, P(I64), P(D), ctypes.c_int]
            lib.ddo_psi_map.restype = ctypes.c_int
            lib.ddo_psi_map.argtypes = [P(_Scan), D, D, D, D, I32, I32, P(D), I32, P(D),
                                        ctypes.c_int]
            lib.ddo_psi_points_general.restype = ctypes.c_int
            lib.ddo_psi_points_general.argtypes = [P(_Visits), I64, P(D), P(D), P(D), P(D),
                                                   ctypes.c_int]
            lib.ddo_default_threads.restype = ctypes.c_int
            _lib = lib
    return _lib


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def e1_series(x: float) -> float:
    return float(_load().ddo_e1_series(x))


def e1_cf(x: float) -> float:
    return float(_load().ddo_e1_cf(x))


def e1_quad(x: float) -> float:
    return float(_load().ddo_e1_quad(x))


def e1(x: float) -> float:
    return float(_load().ddo_e1(x))


def phi(a, dt, tau, sigma, D, Q0=1.0) -> float:
    """Single-visit field (Eqs. 1-4) at squared distance a and lag dt."""
    return float(_load().ddo_phi(a, dt, tau, sigma, D, Q0))


def e1_q(x: float) -> float:
    """E1 in binary128, rounded to double."""
    return float(_load().ddo_e1_q(x))


def phi_bracket_q(a, dt, tau, sigma, D) -> float:
    """Dimensionless bracket of Eqs. 1-4 in binary128 (no Q0/(4 pi D))."""
    return float(_load().ddo_phi_bracket_q(a, dt, tau, sigma, D))


def splitmix64_stream(seed: int, n: int):
    st = ctypes.c_uint64(seed)
    lib = _load()
    return [int(lib.ddo_splitmix64(ctypes.byref(st))) for _ in range(n)]


def default_threads() -> int:
    return int(_load().ddo_default_threads())


def visits(order: int, nx: int, ny: int, stride: int = 2, frames: int = 1, seed: int = 0):
    """Probe ids (row*nx + col) in visit order, as int32 numpy array."""
    n = nx * ny * (frames if order == MULTIFRAME else 1)
    out = np.empty(max(n, 1), dtype=np.int32)
    got = _load().ddo_visits(order, nx, ny, stride, frames, seed,
                             out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), out.size)
    if got < 0:
        raise ValueError("bad scan-order arguments")
    return out[:got].copy()


class Scan:
    """A scan: visit list over an nx-by-ny probe grid, with per-visit dwell tau_v."""

    def __init__(self, nx, ny, ids, pitch, tau_v, sigma, D, Q0=1.0):
        self.ids = np.ascontiguousarray(ids, dtype=np.int32)
        self.nx, self.ny = int(nx), int(ny)
        self.pitch, self.tau_v, self.sigma, self.D, self.Q0 = (
            float(pitch), float(tau_v), float(sigma), float(D), float(Q0))
        self._s = _Scan(self.nx, self.ny,
                        self.ids.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                        self.ids.size, self.pitch, self.tau_v, self.sigma, self.D, self.Q0)

    @property
    def n_visits(self):
        return int(self.ids.size)

    def psi_points(self, x, y, t, nthreads=0):
        x, y, t = (np.ascontiguousarray(v, dtype=np.float64) for v in (x, y, t))
        out = np.empty(x.size, dtype=np.float64)
        if _load().ddo_psi_points(ctypes.byref(self._s), x.size, _dptr(x), _dptr(y), _dptr(t),
                                  _dptr(out), nthreads) != 0:
            raise ValueError("bad arguments")
        return out

    def psi_arrival(self, visit_idx=None, nthreads=0):
        if visit_idx is None:
            visit_idx = np.arange(self.n_visits, dtype=np.int64)
        idx = np.ascontiguousarray(visit_idx, dtype=np.int64)
        out = np.empty(idx.size, dtype=np.float64)
        if _load().ddo_psi_arrival(ctypes.byref(self._s), idx.size,
                                   idx.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                   _dptr(out), nthreads) != 0:
            raise ValueError("bad arguments")
        return out

    def psi_map(self, x0, y0, dx, dy, w, h, t, nthreads=0):
        t = np.ascontiguousarray(np.atleast_1d(t), dtype=np.float64)
        out = np.empty((t.size, h, w), dtype=np.float64)
        if _load().ddo_psi_map(ctypes.byref(self._s), x0, y0, dx, dy, w, h, _dptr(t), t.size,
                               _dptr(out), nthreads) != 0:
            raise ValueError("bad arguments")
        return out


class Visits:
    """A general visit list: visit v sits at (x[v], y[v]) (metres) with the beam
    on from t0[v] for dwell[v] seconds.  Each visit carries its own dwell and
    start time, so flyback and dead time, subsampled or repeated positions and
    any visit order are all expressed directly.  psi sums Eqs. 1-4 over the
    visits that started before the query time (Eq. 6)."""

    def __init__(self, x, y, t0, dwell, sigma, D, Q0=1.0):
        self.x, self.y, self.t0, self.dwell = (np.ascontiguousarray(v, dtype=np.float64)
                                               for v in (x, y, t0, dwell))
        n = self.x.size
        if not (self.y.size == n and self.t0.size == n and self.dwell.size == n):
            raise ValueError("x, y, t0 and dwell must have one entry per visit")
        self.sigma, self.D, self.Q0 = float(sigma), float(D), float(Q0)
        self._v = _Visits(n, _dptr(self.x), _dptr(self.y), _dptr(self.t0), _dptr(self.dwell),
                          self.sigma, self.D, self.Q0)

    @property
    def n_visits(self):
        return int(self.x.size)

    def psi_points(self, x, y, t, nthreads=0):
        x, y, t = (np.ascontiguousarray(v, dtype=np.float64) for v in (x, y, t))
        out = np.empty(x.size, dtype=np.float64)
        if _load().ddo_psi_points_general(ctypes.byref(self._v), x.size, _dptr(x), _dptr(y),
                                          _dptr(t), _dptr(out), nthreads) != 0:
            raise ValueError("bad arguments")
        return out

    def psi_arrival(self, nthreads=0):
        """psi at each visit's own position at the instant its beam turns on."""
        return self.psi_points(self.x, self.y, self.t0, nthreads)

    def psi_map(self, x0, y0, dx, dy, w, h, t, nthreads=0):
        t = np.atleast_1d(np.asarray(t, dtype=np.float64))
        xs = x0 + dx * np.arange(w, dtype=np.float64)
        ys = y0 + dy * np.arange(h, dtype=np.float64)
        X = np.broadcast_to(xs[None, None, :], (t.size, h, w))
        Y = np.broadcast_to(ys[None, :, None], (t.size, h, w))
        T = np.broadcast_to(t[:, None, None], (t.size, h, w))
        return self.psi_points(X.ravel(), Y.ravel(), T.ravel(), nthreads).reshape(t.size, h, w)
