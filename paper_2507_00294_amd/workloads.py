"""Seeded synthetic workloads shared by the tests, the benchmark and the smoke
check.  This module holds scan descriptions and seeded sampling only -- none of
the method's arithmetic -- so both the GPU path and the CPU oracle can be fed
the same inputs from it.

The paper (Sec. I, Sec. II) evaluates STEM scans of a probe grid in raster,
interleaved, random and multi-frame orders with a Gaussian probe, constant D
and deposition rate Q0; it ships no dataset, so every workload here is a
synthetic scan of that shape.  Units are SI.
"""
from __future__ import annotations

from dataclasses import dataclass, field, asdict
from typing import List

import numpy as np

NM = 1e-9
US = 1e-6


@dataclass
class ScanSpec:
    nx: int
    ny: int
    order: str = "raster"          # raster | interleaved | random | multiframe | explicit
    pitch_m: float = 1 * NM
    dwell_s: float = 1 * US        # per probe position (split over frames)
    sigma_m: float = 0.5 * NM
    D_m2s: float = 2.5e-13
    Q0_us: float = 1.0
    stride: int = 2
    frames: int = 1
    seed: int = 0
    visits: List[int] = field(default_factory=list)

    @property
    def tau_v(self) -> float:
        return self.dwell_s / (self.frames if self.order == "multiframe" else 1)

    @property
    def n_visits(self) -> int:
        if self.order == "explicit":
            return len(self.visits)
        return self.nx * self.ny * (self.frames if self.order == "multiframe" else 1)

    @property
    def kappa(self) -> float:
        return self.D_m2s * self.tau_v / self.pitch_m ** 2

    def kwargs(self) -> dict:
        d = asdict(self)
        if self.order != "explicit":
            d.pop("visits")
        return d


@dataclass
class MapSpec:
    x0_m: float
    y0_m: float
    dx_m: float
    dy_m: float
    w: int
    h: int
    times_s: List[float]


# ---- plain FP64, 8x8 raster; maps at the end of each of the 64 dwells ------
def small_raster() -> ScanSpec:
    return ScanSpec(8, 8, "raster", 1 * NM, 1 * US, 0.5 * NM, 2.5e-13, 1.0)


def small_raster_maps(spec: ScanSpec) -> MapSpec:
    # 32x32 pixels at 0.25 nm from the first probe; t_m = m tau, m = 1..64
    return MapSpec(0.0, 0.0, 0.25 * NM, 0.25 * NM, 32, 32,
                   [m * spec.tau_v for m in range(1, spec.n_visits + 1)])


# ---- plain FP64, 32x32 raster and interleaved, D log-uniform ----------------
def medium_scans(n_per_order: int = 8, seed: int = 2) -> List[ScanSpec]:
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for order in ("raster", "interleaved"):
        for _ in range(n_per_order):
            D = float(10.0 ** rng.uniform(-15, -11))
            out.append(ScanSpec(32, 32, order, 1 * NM, 1 * US, 0.5 * NM, D, 1.0, stride=2))
    return out


def medium_final_map(spec: ScanSpec) -> MapSpec:
    # 128x128 pixels at 0.25 nm covering the 32x32 probe grid; t = end of scan
    return MapSpec(0.0, 0.0, 0.25 * NM, 0.25 * NM, 128, 128, [spec.n_visits * spec.tau_v])


# ---- mixed vs FP64: 512x512 random scan ---------------------------------------
def large_random(side: int = 512) -> ScanSpec:
    return ScanSpec(side, side, "random", 1 * NM, 0.5 * US, 0.4 * NM, 1e-12, 1.0, seed=3)


# ---- batched: scans of uneven size, order and physics -------------------------
def batch_scans(n: int = 256, seed: int = 4, side_lo: int = 16, side_hi: int = 256,
                fixed_side: int | None = None) -> List[ScanSpec]:
    rng = np.random.Generator(np.random.PCG64(seed))
    orders = ("raster", "interleaved", "random", "multiframe")
    out = []
    for k in range(n):
        side = int(fixed_side) if fixed_side else int(rng.integers(side_lo, side_hi + 1))
        order = orders[int(rng.integers(0, 4))]
        dwell = float(10.0 ** rng.uniform(-7, -5))
        D = float(10.0 ** rng.uniform(-15, -11))
        sigma = float(rng.uniform(0.2, 1.0)) * NM
        out.append(ScanSpec(side, side, order, 1 * NM, dwell, sigma, D, 1.0, stride=2,
                            frames=4 if order == "multiframe" else 1,
                            seed=int(rng.integers(0, 2 ** 63))))
    return out


def surrogate_scans(n: int, seed: int) -> List[ScanSpec]:
    """Batched-style sampling at a fixed 64x64 grid (training seed 5, test seed 6)."""
    return batch_scans(n, seed=seed, fixed_side=64)


def causal_arrival_pairs(n_visits: int) -> int:
    """Number of (visit, earlier visit) pairs of an arrival query."""
    return n_visits * (n_visits - 1) // 2


def sampled_visits(n_visits: int, k: int, seed: int) -> np.ndarray:
    """k distinct visit indices, seeded, always including the first and last."""
    rng = np.random.Generator(np.random.PCG64(seed))
    k = min(k, n_visits)
    idx = set(rng.choice(n_visits, size=k, replace=False).tolist())
    idx.update({0, n_visits - 1})
    return np.array(sorted(idx), dtype=np.int64)


def stratified_visits(n_visits: int, k: int, seed: int) -> np.ndarray:
    """k visit indices, one drawn uniformly (seeded) from each of k equal
    strata of [0, n_visits); the first stratum gives visit 0 and the last
    gives the last visit, so both ends of the scan are always included."""
    rng = np.random.Generator(np.random.PCG64(seed))
    k = min(k, n_visits)
    edges = (np.arange(k + 1, dtype=np.int64) * n_visits) // k
    lo, hi = edges[:-1], edges[1:]
    idx = lo + (rng.random(k) * (hi - lo)).astype(np.int64)
    idx = np.minimum(idx, hi - 1)
    idx[0], idx[-1] = 0, n_visits - 1
    return idx


# ---- general visit lists: per-visit position, start time and dwell -----------
@dataclass
class VisitList:
    """Visits with their own position (m), start time and dwell (s)."""
    x_m: np.ndarray
    y_m: np.ndarray
    t0_s: np.ndarray
    dwell_s: np.ndarray
    sigma_m: float
    D_m2s: float
    Q0_us: float = 1.0
    name: str = ""

    @property
    def n_visits(self) -> int:
        return int(self.x_m.size)

    @property
    def t_end(self) -> float:
        return float(np.max(self.t0_s + self.dwell_s))

    def kwargs(self) -> dict:
        return dict(sigma_m=self.sigma_m, D_m2s=self.D_m2s, Q0_us=self.Q0_us)


def visit_list(kind: str, nx: int, ny: int, seed: int = 0, pitch_m: float = 1 * NM,
               dwell_s: float = 1 * US, sigma_m: float = 0.5 * NM, D_m2s: float = 2.5e-13,
               Q0_us: float = 1.0) -> VisitList:
    """Seeded general visit lists on an nx-by-ny probe lattice:
    * "flyback": raster lines, dwell x U(0.5, 1.5) per visit, a dead time of
      nx/4 dwells at the end of each line (beam blanked while it returns);
    * "sparse": a random quarter of the probes in random order, dwell x
      U(0.5, 1.5), dead time U(0, 2) dwells before each visit;
    * "frames": 3 raster frames with dwells 1/2, 1/3, 1/6 of the dwell and a
      dead time of 10 dwells between frames (revisits at the same positions);
    * "drift": raster with each position displaced by a slow drift plus
      U(-0.1, 0.1) pitch noise (off the lattice), dwell x U(0.5, 1.5).
    Visits never overlap in time except where stated; visit order is the
    list order."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ids = np.arange(nx * ny)
    if kind == "flyback":
        col, row = ids % nx, ids // nx
        dw = dwell_s * rng.uniform(0.5, 1.5, ids.size)
        gap = np.where(col == 0, (nx / 4) * dwell_s, 0.0)
        gap[0] = 0.0
        x, y = col * pitch_m, row * pitch_m
    elif kind == "sparse":
        pick = rng.permutation(ids)[: max(1, ids.size // 4)]
        x, y = (pick % nx) * pitch_m, (pick // nx) * pitch_m
        dw = dwell_s * rng.uniform(0.5, 1.5, pick.size)
        gap = dwell_s * rng.uniform(0.0, 2.0, pick.size)
    elif kind == "frames":
        fr = np.repeat(np.arange(3), ids.size)
        base = np.tile(ids, 3)
        x, y = (base % nx) * pitch_m, (base // nx) * pitch_m
        dw = dwell_s * np.array([1 / 2, 1 / 3, 1 / 6])[fr]
        gap = np.where((np.arange(base.size) % ids.size == 0) & (fr > 0), 10 * dwell_s, 0.0)
    elif kind == "drift":
        col, row = ids % nx, ids // nx
        s = np.arange(ids.size) / ids.size
        x = (col + 0.3 * s + rng.uniform(-0.1, 0.1, ids.size)) * pitch_m
        y = (row + 0.2 * s * s + rng.uniform(-0.1, 0.1, ids.size)) * pitch_m
        dw = dwell_s * rng.uniform(0.5, 1.5, ids.size)
        gap = np.zeros(ids.size)
    else:
        raise ValueError(f"unknown visit list kind {kind!r}")
    t0 = np.cumsum(gap + np.concatenate([[0.0], dw[:-1]]))
    return VisitList(np.asarray(x, np.float64), np.asarray(y, np.float64), t0, dw, sigma_m,
                     D_m2s, Q0_us, kind)
